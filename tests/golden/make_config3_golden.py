"""Write tests/golden/config3_block_oracle.json: the CPU oracle's outputs for
the leading 320 x 320 block of configuration 3's matrix (the interlaced
dyadic Cauchy matrix, 32768-bit numbers): per-entry hashes of D_1..D_320 and
of the block's last-column minors, and a digest of its factored form.  By the
prefix property of elimination without pivoting, D_1..D_320 are also those of
the whole N = 2048 matrix.  Calls only the oracle and the seeded generators.

    python tests/golden/make_config3_golden.py      # about 15-30 minutes on 8 cores
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

OUT = os.path.join(HERE, "config3_block_oracle.json")
BLOCK = 320
P = 1024


def block_input(n=BLOCK):
    """The leading n x n block of configuration 3's matrix: the generator's
    nodes for N = 2048, the first n of each (a_ij depends on x_i and y_j only)."""
    x, y = inputs.dyadic_nodes(2048, inputs.config_seed(3), 0.0, 1000.0)
    return inputs.cauchy(x[:n], y[:n], P, workers=1)


def main():
    A = block_input()
    t0 = time.time()
    f, c = oracle.det_pipeline(A)
    secs = time.time() - t0
    print(f"config 3 leading {BLOCK} block: {secs:.1f} s, info {f.info}", flush=True)
    res = {"about": f"oracle outputs for the leading {BLOCK}x{BLOCK} block of config 3 (32768-bit); "
                    "written by make_config3_golden.py",
           "block": BLOCK, "P": P, "info": f.info, "input_sha256": digest(A), "D": entry_hashes(f.D),
           "c": entry_hashes(c), "LU_sha256": digest(f.LU), "oracle_seconds": secs,
           "oracle_threads": oracle.default_threads()}
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=0)


if __name__ == "__main__":
    main()
