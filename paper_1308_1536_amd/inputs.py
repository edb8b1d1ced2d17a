"""Seeded synthetic inputs in the multiprecision number format.

This module only *encodes data*: it turns exact rationals (Python ``int`` /
``fractions.Fraction``) into the number format by one truncation toward zero,
and draws seeded random nodes, integers and mantissas.  It holds none of the
elimination arithmetic, and it is the only module that both the GPU path's
callers and the CPU oracle's callers share.

Number format: value = (-1)^s * m * 2^(e - 32P), where m has P little-endian
uint32 limbs with the top bit set; zero is s = e = m = 0.  Host layout is
element-contiguous: limbs [..., P] uint32, exp [...] int64, sign [...] int32.

The paper's matrices (Sec. 2, eqs. (det) and (betaNew)) need the zeros of the
zeta function to ~10^4 digits, which are not available; the stand-ins here
have the same character (nearly singular, the paper's N and precision): Cauchy
matrices 1/(x_i - y_j) with closely spaced nodes, Hilbert matrices, random
integers and random full-precision mantissas.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass
from fractions import Fraction
from typing import Sequence

import numpy as np


@dataclass
class MpArray:
    """Host container of numbers: limbs [..., P] uint32, exp [...] int64, sign [...] int32."""
    limbs: np.ndarray
    exp: np.ndarray
    sign: np.ndarray

    @property
    def P(self) -> int:
        return int(self.limbs.shape[-1])

    @property
    def shape(self):
        return tuple(self.exp.shape)

    def copy(self) -> "MpArray":
        return MpArray(self.limbs.copy(), self.exp.copy(), self.sign.copy())

    def __getitem__(self, idx) -> "MpArray":
        return MpArray(self.limbs[idx], self.exp[idx], self.sign[idx])

    @staticmethod
    def zeros(shape, P: int) -> "MpArray":
        shape = tuple(shape)
        return MpArray(np.zeros(shape + (P,), np.uint32), np.zeros(shape, np.int64),
                       np.zeros(shape, np.int32))


# ---------------------------------------------------------------------------
# exact <-> format
# ---------------------------------------------------------------------------

def encode(q, P: int) -> tuple[int, int, int]:
    """Truncate the exact rational q toward zero to p = 32P bits: (s, e, m)."""
    q = Fraction(q)
    if q == 0:
        return 0, 0, 0
    p = 32 * P
    s = 1 if q < 0 else 0
    n, d = abs(q.numerator), q.denominator
    # e with 2^(e-1) <= n/d < 2^e
    e = n.bit_length() - d.bit_length() + 1
    if e - 1 >= 0:
        below = n < (d << (e - 1))
    else:
        below = (n << (1 - e)) < d
    if below:
        e -= 1
    sh = p - e
    m = (n << sh) // d if sh >= 0 else n // (d << (-sh))
    assert (1 << (p - 1)) <= m < (1 << p)
    return s, e, m


def int_to_limbs(m: int, P: int) -> np.ndarray:
    return np.frombuffer(m.to_bytes(4 * P, "little"), dtype="<u4").astype(np.uint32)


def limbs_to_int(limbs: np.ndarray) -> int:
    return int.from_bytes(np.ascontiguousarray(limbs, dtype="<u4").tobytes(), "little")


def decode(x: MpArray, idx=()) -> Fraction:
    """Exact rational value of one stored number."""
    m = limbs_to_int(x.limbs[idx])
    if m == 0:
        return Fraction(0)
    e = int(x.exp[idx]) - 32 * x.P
    v = Fraction(m) * (Fraction(2) ** e)
    return -v if int(x.sign[idx]) else v


def from_values(values, P: int) -> MpArray:
    """Encode a (nested) array of exact rationals."""
    arr = np.asarray(values, dtype=object)
    out = MpArray.zeros(arr.shape, P)
    for idx in np.ndindex(arr.shape):
        s, e, m = encode(arr[idx], P)
        out.sign[idx] = s
        out.exp[idx] = e
        out.limbs[idx] = int_to_limbs(m, P)
    return out


# ---------------------------------------------------------------------------
# matrices
# ---------------------------------------------------------------------------

def _cauchy_fill(rows, xs_num, ys_num, F, P, out_l, out_e, out_s):
    """a_ij = 1 / (x_i - y_j) = 2^F / d, d = X_i - Y_j an integer, truncated to p bits."""
    p = 32 * P
    for i in rows:
        xi = xs_num[i]
        for j, yj in enumerate(ys_num):
            d = xi - yj
            if d == 0:
                raise ZeroDivisionError("Cauchy nodes collide")
            s = 1 if d < 0 else 0
            d = abs(d)
            # 2^(e-1) <= 2^F/d < 2^e
            e = F - d.bit_length() + 1
            if d & (d - 1) == 0:  # exact power of two
                e += 1
            m = (1 << (p - e + F)) // d
            out_s[i, j] = s
            out_e[i, j] = e
            out_l[i, j] = np.frombuffer(m.to_bytes(4 * P, "little"), dtype="<u4")


_SHARED = {}


def _cauchy_worker(rows):
    a = _SHARED
    _cauchy_fill(rows, a["xs"], a["ys"], a["F"], a["P"], a["l"], a["e"], a["s"])
    return len(rows)


def cauchy(x: Sequence, y: Sequence, P: int, workers: int | None = None) -> MpArray:
    """a_ij = RZ_p(1 / (x_i - y_j)) for exact dyadic or integer nodes.  Large
    matrices are filled by forked workers writing into one shared mapping."""
    import mmap
    xf = [Fraction(v) for v in x]
    yf = [Fraction(v) for v in y]
    dens = [f.denominator for f in xf + yf]
    for dd in dens:
        if dd & (dd - 1):
            raise ValueError("cauchy: nodes must be dyadic rationals")
    F = max(dd.bit_length() - 1 for dd in dens)
    xs = [int(v * (1 << F)) for v in xf]
    ys = [int(v * (1 << F)) for v in yf]
    n, m = len(xs), len(ys)
    if workers is None:
        # forked workers only for the largest matrices (32K-bit, N = 2048);
        # MPDET_GEN_WORKERS overrides (1: never fork, e.g. under a profiler
        # whose signal handlers the children would inherit)
        env = os.environ.get("MPDET_GEN_WORKERS")
        if env is not None:
            workers = max(1, int(env))
        else:
            workers = 1 if n * m * P < 1_000_000_000 else min(16, os.cpu_count() or 1)
    if workers <= 1 or n < 2:
        out = MpArray.zeros((n, m), P)
        _cauchy_fill(range(n), xs, ys, F, P, out.limbs, out.exp, out.sign)
        return out
    nl, ne, ns = n * m * P * 4, n * m * 8, n * m * 4
    buf = mmap.mmap(-1, nl + ne + ns)
    limbs = np.frombuffer(buf, dtype=np.uint32, count=n * m * P, offset=0).reshape(n, m, P)
    exp = np.frombuffer(buf, dtype=np.int64, count=n * m, offset=nl).reshape(n, m)
    sign = np.frombuffer(buf, dtype=np.int32, count=n * m, offset=nl + ne).reshape(n, m)
    _SHARED.update(xs=xs, ys=ys, F=F, P=P, l=limbs, e=exp, s=sign)
    step = max(1, -(-n // (4 * workers)))
    chunks = [list(range(i, min(n, i + step))) for i in range(0, n, step)]
    import multiprocessing as mpc
    import sys
    try:
        with mpc.get_context("fork").Pool(workers) as pool:
            done = 0
            for rows_done in pool.imap_unordered(_cauchy_worker, chunks):
                done += rows_done
                if n * m * P >= 4_000_000_000:  # minutes of work: say how far it is
                    print(f"[inputs] cauchy {n}x{m}: {done}/{n} rows", file=sys.stderr, flush=True)
    finally:
        _SHARED.clear()
    assert done == n
    return MpArray(limbs, exp, sign)


def cauchy_integer_nodes(N: int, P: int) -> tuple[MpArray, list, list]:
    """x_i = 2i+1, y_j = 2j (i, j = 0..N-1): a_ij = 1/(2(i-j)+1)."""
    x = [2 * i + 1 for i in range(N)]
    y = [2 * j for j in range(N)]
    return cauchy(x, y, P), x, y


def dyadic_nodes(N: int, seed: int, lo: float, hi: float, dmin: float = 1e-6,
                 dmax: float = 1e-3) -> tuple[list, list]:
    """Interlaced nodes x_1 < y_1 < x_2 < y_2 < ...: x sorted uniform float64 draws
    on [lo, hi], y_j = x_j + delta_j exactly, delta_j uniform float64 in [dmin, dmax].
    Draws are repeated (same generator stream) until the nodes interlace strictly."""
    rng = np.random.default_rng(seed)
    while True:
        xs = np.sort(rng.uniform(lo, hi, size=N))
        ds = rng.uniform(dmin, dmax, size=N)
        x = [Fraction(float(v)) for v in xs]
        y = [x[j] + Fraction(float(ds[j])) for j in range(N)]
        ok = all(x[j] < y[j] for j in range(N)) and \
            all(y[j] < x[j + 1] for j in range(N - 1))
        if ok:
            return x, y


def cauchy_dyadic(N: int, P: int, seed: int, lo: float = 0.0, hi: float = 1000.0,
                  workers: int | None = None) -> tuple[MpArray, list, list]:
    """Nearly singular Cauchy matrix on seeded interlaced dyadic nodes."""
    x, y = dyadic_nodes(N, seed, lo, hi)
    return cauchy(x, y, P, workers), x, y


def hilbert(N: int, P: int) -> MpArray:
    """H_ij = 1/(i+j-1) (1-based): the Cauchy matrix with x_i = i, y_j = 1-j."""
    x = list(range(1, N + 1))
    y = [1 - j for j in range(1, N + 1)]
    return cauchy(x, y, P)


def random_integers(N: int, P: int, seed: int, lo: int = -1000, hi: int = 1000) -> tuple[MpArray, np.ndarray]:
    """Entries uniform in [lo, hi] (exact in the format)."""
    rng = np.random.default_rng(seed)
    vals = rng.integers(lo, hi, size=(N, N), endpoint=True)
    out = MpArray.zeros((N, N), P)
    p = 32 * P
    for idx in np.ndindex(vals.shape):
        v = int(vals[idx])
        if v == 0:
            continue
        a = abs(v)
        e = a.bit_length()
        out.sign[idx] = 1 if v < 0 else 0
        out.exp[idx] = e
        out.limbs[idx] = int_to_limbs(a << (p - e), P)
    return out, vals


def random_mantissas(shape, P: int, seed: int, emin: int = -4, emax: int = 4) -> MpArray:
    """Uniform random p-bit mantissas (top bit forced), uniform signs and
    exponents uniform in [emin, emax]."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape) if not isinstance(shape, int) else (shape, shape)
    limbs = rng.integers(0, 2**32, size=shape + (P,), dtype=np.uint64).astype(np.uint32)
    limbs[..., P - 1] |= np.uint32(0x80000000)
    exp = rng.integers(emin, emax, size=shape, endpoint=True).astype(np.int64)
    sign = rng.integers(0, 2, size=shape).astype(np.int32)
    return MpArray(limbs, exp, sign)


def triangular_product(N: int, P: int, seed: int) -> tuple[MpArray, np.ndarray, np.ndarray]:
    """A = L U with L unit lower triangular (small integer multipliers) and U
    upper triangular with power-of-two diagonal and small integers above it.
    Every step of elimination without pivoting is then exact: the multipliers
    are the integers of L and every intermediate value is a small integer."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-3, 4, size=(N, N)), -1) + np.eye(N, dtype=np.int64)
    U = np.triu(rng.integers(-5, 6, size=(N, N)), 1)
    U += np.diag(2 ** rng.integers(0, 4, size=N) * rng.choice([-1, 1], size=N))
    A = (L.astype(object) @ U.astype(object))
    return from_values(A, P), L, U


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------

CONFIG_SEED_BASE = 1308_0000


def config_seed(cfg: int, k: int = 0) -> int:
    return CONFIG_SEED_BASE + 100 * cfg + k


def config_c1(P: int = 32) -> dict:
    """N=64, 1024 bits: integer-node Cauchy and random integers in [-1000, 1000]."""
    cau, x, y = cauchy_integer_nodes(64, P)
    ri, vals = random_integers(64, P, config_seed(1))
    return {"cauchy": (cau, x, y), "randint": (ri, vals)}


def config_c2(P: int = 128, N: int = 512) -> dict:
    """N=512, 4096 bits: dyadic Cauchy on [0, 1000] and random mantissas."""
    cau, x, y = cauchy_dyadic(N, P, config_seed(2), 0.0, 1000.0)
    rm = random_mantissas((N, N), P, config_seed(2, 1))
    return {"cauchy": (cau, x, y), "randmant": rm}


def config_c3(P: int = 1024, N: int = 2048) -> dict:
    """N=2048, 32768 bits: interlaced dyadic Cauchy on [0, 1000]."""
    cau, x, y = cauchy_dyadic(N, P, config_seed(3), 0.0, 1000.0)
    return {"cauchy": (cau, x, y)}


def config_c5(P: int = 1024, N: int = 6144) -> dict:
    """N=6144, 32768 bits (155 GB): dyadic Cauchy with sorted nodes on [0, 10000]."""
    cau, x, y = cauchy_dyadic(N, P, config_seed(5), 0.0, 10000.0)
    return {"cauchy": (cau, x, y)}


def config_c4_sizes(count: int = 256, lo: int = 16, hi: int = 384) -> list[int]:
    rng = np.random.default_rng(config_seed(4))
    return [int(v) for v in rng.integers(lo, hi, size=count, endpoint=True)]


def config_c4(P: int = 64, count: int = 256) -> list[tuple[str, MpArray]]:
    """256 matrices, N uniform in [16, 384], 2048 bits: even index random
    mantissas, odd index dyadic Cauchy."""
    out = []
    for b, n in enumerate(config_c4_sizes(count)):
        if b % 2 == 0:
            out.append(("randmant", random_mantissas((n, n), P, config_seed(4, 1 + b))))
        else:
            cau, _, _ = cauchy_dyadic(n, P, config_seed(4, 1 + b), 0.0, 1000.0)
            out.append(("cauchy", cau))
    return out


def u_count(N: int) -> int:
    """Number of trailing updates of elimination on an N x N matrix."""
    return (N - 1) * N * (2 * N - 1) // 6


def limb_macs_int8(N: int, P: int) -> int:
    """Algorithmic 8-bit limb MACs: U(N) * (p/8)^2."""
    return u_count(N) * (4 * P) ** 2

