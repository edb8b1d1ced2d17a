"""Write tests/golden/config2_oracle.json: the CPU oracle's outputs for the two
config-2 matrices (N=512, 4096-bit), as per-entry hashes of D_1..D_N and of the
last-column minors, and one digest of the factored matrix.  Calls only the
oracle and the seeded input generators.

    python tests/golden/make_config2_golden.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1308_1536_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_oracle.json")


def entry_hashes(x) -> list:
    """16-hex-digit hash of each number (limbs, exponent, sign)."""
    out = []
    for i in range(x.exp.shape[0]):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(x.limbs[i], "<u4").tobytes())
        h.update(np.int64(x.exp[i]).tobytes())
        h.update(np.int32(x.sign[i]).tobytes())
        out.append(h.hexdigest()[:16])
    return out


def digest(x) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x.limbs, "<u4").tobytes())
    h.update(np.ascontiguousarray(x.exp, "<i8").tobytes())
    h.update(np.ascontiguousarray(x.sign, "<i4").tobytes())
    return h.hexdigest()


def main():
    cfg = inputs.config_c2()
    mats = {"cauchy": cfg["cauchy"][0], "randmant": cfg["randmant"]}
    res = {"about": "oracle outputs for config 2 (N=512, 4096-bit); written by make_config2_golden.py",
           "matrices": {}}
    for name, A in mats.items():
        t0 = time.time()
        f, c = oracle.det_pipeline(A)
        print(f"{name}: {time.time() - t0:.1f} s, info {f.info}", flush=True)
        res["matrices"][name] = {"info": f.info, "input_sha256": digest(A), "D": entry_hashes(f.D),
                                 "c": entry_hashes(c), "LU_sha256": digest(f.LU)}
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=0)


if __name__ == "__main__":
    main()
