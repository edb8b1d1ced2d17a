"""Hashes of multiprecision arrays for the stored oracle outputs (shared by
the scripts that write them and the GPU tests that read them).  Holds no
arithmetic of the method: it only hashes the bytes of numbers."""
import hashlib

import numpy as np


def entry_hashes(x) -> list:
    """16-hex-digit hash of each number of a vector (limbs, exponent, sign)."""
    out = []
    for i in range(x.exp.shape[0]):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(x.limbs[i], "<u4").tobytes())
        h.update(np.int64(x.exp[i]).tobytes())
        h.update(np.int32(x.sign[i]).tobytes())
        out.append(h.hexdigest()[:16])
    return out


def digest(x) -> str:
    """SHA-256 of a whole array of numbers (limbs, then exponents, then signs)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x.limbs, "<u4").tobytes())
    h.update(np.ascontiguousarray(x.exp, "<i8").tobytes())
    h.update(np.ascontiguousarray(x.sign, "<i4").tobytes())
    return h.hexdigest()
