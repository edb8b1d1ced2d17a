"""Write tests/golden/config4_oracle.json: the CPU oracle's outputs for every
one of configuration 4's 256 matrices (N uniform in [16, 384], 2048-bit; even
index random mantissas, odd index dyadic Cauchy): per matrix the info code,
per-entry hashes of D_1..D_N and of the last-column minors, and a digest of
the factored matrix; for a sample of matrices (the smallest, the largest and
a few between) also a digest of adj(A)^T.  Calls only the oracle and the
seeded generators.

    python tests/golden/make_config4_golden.py      # about 10-20 minutes on 8 cores
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from golden_util import digest, entry_hashes  # noqa: E402
from paper_1308_1536_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "config4_oracle.json")


def adjugate_sample(sizes):
    """indices of the matrices whose adjugate is stored: smallest, largest,
    and six spread over the batch"""
    order = sorted(range(len(sizes)), key=lambda b: sizes[b])
    pick = {order[0], order[-1]}
    for t in range(1, 7):
        pick.add(order[t * (len(order) - 1) // 7])
    return sorted(pick)


def main():
    mats = inputs.config_c4()
    sizes = [m.exp.shape[0] for _, m in mats]
    adj = set(adjugate_sample(sizes))
    res = {"about": "oracle outputs for the 256 matrices of config 4 (2048-bit); written by "
                    "make_config4_golden.py", "sizes": sizes, "adjugate_sample": sorted(adj), "matrices": []}
    t0 = time.time()
    for b, (name, A) in enumerate(mats):
        f, c = oracle.det_pipeline(A)
        e = {"name": name, "N": sizes[b], "info": f.info, "input_sha256": digest(A), "D": entry_hashes(f.D),
             "c": entry_hashes(c) if c is not None else None, "LU_sha256": digest(f.LU)}
        if b in adj and f.info == 0:
            e["adjT_sha256"] = digest(oracle.adjugate_t(f))
        res["matrices"].append(e)
        if b % 16 == 15:
            print(f"{b + 1}/256 matrices, {time.time() - t0:.0f} s", flush=True)
    res["oracle_seconds"] = time.time() - t0
    res["oracle_threads"] = oracle.default_threads()
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=0)


if __name__ == "__main__":
    main()
