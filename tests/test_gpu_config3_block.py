"""Configuration 3 at its own precision (32768-bit numbers, 1024 limbs):
the leading 320 x 320 block of its interlaced Cauchy matrix on both update
paths, against the oracle's outputs stored by
tests/golden/make_config3_golden.py (a hash of every D_k and every minor, a
digest of the factored block).  At 320 columns the MFMA update spans ten
32-column blocks, so its XCD column mapping (blocks spread over eight dies)
and the streaming finish run at the configuration's limb count.  By the
prefix property of elimination without pivoting, D_1..D_320 are also the
whole configuration's.  The two paths are also compared with each other on
the whole factored block."""
import json
import os
import sys

import pytest

from gpu_util import assert_same, gpu_det, say

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from golden_util import digest, entry_hashes  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(HERE, "golden", "config3_block_oracle.json")


@pytest.fixture(scope="module")
def block():
    import make_config3_golden
    with open(GOLDEN) as fh:
        g = json.load(fh)
    A = make_config3_golden.block_input(g["block"])
    assert digest(A) == g["input_sha256"], "the seeded generator changed"
    return g, A


@pytest.fixture(scope="module")
def runs(block):
    g, A = block
    out = {}
    for path in ("mfma", "valu"):
        say(f"[config3 block] path={path} N={g['block']} P={g['P']}")
        out[path] = gpu_det(A, path)
    return out


@pytest.mark.parametrize("path", ["mfma", "valu"])
def test_config3_block_against_oracle(block, runs, path):
    g, _ = block
    LU, D, c, info = runs[path]
    assert info == g["info"] == 0
    dh, ch = entry_hashes(D), entry_hashes(c)
    bad_d = [k for k in range(len(dh)) if dh[k] != g["D"][k]]
    bad_c = [k for k in range(len(ch)) if ch[k] != g["c"][k]]
    assert not bad_d, f"D differs at {bad_d[:5]} ({len(bad_d)} entries)"
    assert not bad_c, f"c differs at {bad_c[:5]} ({len(bad_c)} entries)"
    assert digest(LU) == g["LU_sha256"]


def test_config3_block_paths_agree(runs):
    """MFMA against VALU on the same inputs, every number of the outputs."""
    for k, what in enumerate(("LU", "D", "c")):
        assert_same(runs["mfma"][k], runs["valu"][k], f"MFMA vs VALU {what}")
