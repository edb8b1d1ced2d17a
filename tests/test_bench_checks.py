"""The bench's exact full-size checks, pinned on the CPU: on the oracle's
factorisation of a leading block of the config-2 Cauchy matrix the pivots
agree with the closed form and the minors satisfy sum_i c_i a_iN = det to
within a few bits of p, and an error of about 2^-108 planted in a pivot or in
the minor of the sum's dominant term is seen."""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_1308_1536_amd import inputs

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _run(N=12, P=4):
    x, y = inputs.dyadic_nodes(512, inputs.config_seed(2), 0.0, 1000.0)
    A = inputs.cauchy(x[:N], y[:N], P, workers=1)
    f, c = oracle.det_pipeline(A)
    return A, f, c


def _as_dev(mp):
    import torch
    return SimpleNamespace(limbs=torch.from_numpy(np.ascontiguousarray(mp.limbs).view(np.int32)),
                           exp=torch.from_numpy(np.ascontiguousarray(mp.exp)),
                           sign=torch.from_numpy(np.ascontiguousarray(mp.sign)))


def test_checks_hold_on_the_oracle_run():
    A, f, c = _run()
    r = bench.full_size_checks(2, "cauchy", A, _as_dev(f.LU), f.D, c, 0)
    assert r["cauchy_pivots_checked"] == 12
    assert -128 <= r["cauchy_pivot_max_rel_err_bits"] <= -120
    assert -128 <= r["minors_invariant_rel_err_bits"] <= -118


@pytest.mark.parametrize("where", ["pivot", "minor"])
def test_checks_see_a_planted_ulp(where):
    A, f, c = _run()
    LU, cc = f.LU.copy(), c.copy()
    if where == "pivot":
        LU.limbs[5, 5, 0] ^= np.uint32(1 << 20)  # about 2^-108 relative
    else:  # the dominant term of the sum (c_N a_NN is ~2^30 above the others here)
        cc.limbs[11, 0] ^= np.uint32(1 << 20)
    r = bench.full_size_checks(2, "cauchy", A, _as_dev(LU), f.D, cc, 0)
    key = "cauchy_pivot_max_rel_err_bits" if where == "pivot" else "minors_invariant_rel_err_bits"
    assert r[key] > -115


def test_all_minors_invariant_check():
    """The check of sampled rows of the minors of every leading block holds on
    the oracle's all_minors and sees an error of about 2^-76 (relative)
    planted in a row's largest term."""
    A, f, _ = _run()
    C = oracle.all_minors(A)
    rows = [0, 1, 5, 11]
    assert bench.all_minors_invariant_bits(A, C, f.D, rows) < -115
    Cb = C.copy()
    a = np.array([abs(float(np.ldexp(1.0, int(A.exp[i, 7])))) for i in range(8)])
    big = int(np.argmax(a * np.array([float(np.ldexp(1.0, int(Cb.exp[7, i]))) for i in range(8)])))
    Cb.limbs[7, big, 1] ^= np.uint32(1 << 20)
    assert bench.all_minors_invariant_bits(A, Cb, f.D, [7]) > -115


def test_adjugate_column_check():
    """Laplace's expansion along sampled columns of the oracle's adj(A)^T
    holds to within a few bits of p, and a 2^-76 (relative) error planted in
    a column's largest term is seen."""
    from paper_1308_1536_amd.binding import HostMp
    A, f, _ = _run()
    T = oracle.adjugate_t(f)
    det = HostMp(f.D.limbs[-1], f.D.exp[-1], f.D.sign[-1])
    assert bench.adjugate_column_bits(A, T, det, [0, 5, 11]) < -115
    Tb = T.copy()
    big = int(np.argmax([int(Tb.exp[i, 5]) + int(A.exp[i, 5]) for i in range(12)]))
    Tb.limbs[big, 5, 1] ^= np.uint32(1 << 20)
    assert bench.adjugate_column_bits(A, Tb, det, [5]) > -115
