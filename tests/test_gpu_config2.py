"""Full-size parity at config 2 (N=512, 4096-bit, the bench workload): the GPU
outputs against the oracle's, stored by tests/golden/make_config2_golden.py as
per-entry hashes of every D_k and every minor plus a digest of the factored
matrix.  Both trailing-update paths are checked."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "config2_oracle.json")


def entry_hashes(x):
    out = []
    for i in range(x.exp.shape[0]):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(x.limbs[i], "<u4").tobytes())
        h.update(np.int64(x.exp[i]).tobytes())
        h.update(np.int32(x.sign[i]).tobytes())
        out.append(h.hexdigest()[:16])
    return out


def digest(x):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x.limbs, "<u4").tobytes())
    h.update(np.ascontiguousarray(x.exp, "<i8").tobytes())
    h.update(np.ascontiguousarray(x.sign, "<i4").tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def golden_and_inputs():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    cfg = inputs.config_c2()
    return g, {"cauchy": cfg["cauchy"][0], "randmant": cfg["randmant"]}


@pytest.mark.parametrize("path", ["mfma", "valu"])
@pytest.mark.parametrize("name", ["cauchy", "randmant"])
def test_config2_full_size(golden_and_inputs, name, path):
    g, mats = golden_and_inputs
    want = g["matrices"][name]
    A = mats[name]
    assert digest(A) == want["input_sha256"], "the seeded generator changed"
    say(f"[config2] {name} {path}")
    LU, D, c, info = gpu_det(A, path)
    assert info == want["info"] == 0
    dh, ch = entry_hashes(D), entry_hashes(c)
    bad_d = [k for k in range(len(dh)) if dh[k] != want["D"][k]]
    bad_c = [k for k in range(len(ch)) if ch[k] != want["c"][k]]
    assert not bad_d, f"D differs at {bad_d[:5]} ({len(bad_d)} entries)"
    assert not bad_c, f"c differs at {bad_c[:5]} ({len(bad_c)} entries)"
    assert digest(LU) == want["LU_sha256"]
