"""Rigorous error bounds on the GPU (mp_det_factor_ball): the factorisation's
bits are mp_det_factor's, and the radius of every leading determinant equals
the oracle's bit for bit (integer ball arithmetic), on the one-wave update,
the lane product and the MFMA path, with exact and with rounded input; the
balls of a Cauchy matrix contain its closed-form leading determinants."""
from fractions import Fraction

import numpy as np
import pytest

import exact
import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def _gpu_ball(A_host, input_ulp, path):
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(A_host)
    D, rm, re, info = binding.factor_ball(A, input_ulp, path)
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), rm.cpu().numpy().view(np.uint32), re.cpu().numpy(), int(info.item())


@pytest.mark.parametrize("P,n,path", [(2, 20, "valu"), (8, 33, "valu"), (16, 30, "mfma"), (64, 25, "auto")])
@pytest.mark.parametrize("ulp", [False, True])
def test_ball_radii_match_oracle(P, n, path, ulp):
    A = inputs.random_mantissas((n, n), P, 9300 + n + P)
    say(f"[ball] P={P} n={n} {path} ulp={ulp}")
    LU, D, rm, re, info = _gpu_ball(A, ulp, path)
    f, orm, ore = oracle.factor_ball(A, ulp)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert np.array_equal(rm, orm) and np.array_equal(re, ore), "radii"


def test_ball_contains_cauchy_closed_forms():
    A, x, y = inputs.cauchy_dyadic(48, 8, 29)
    say("[ball] cauchy n=48 256 bits")
    LU, D, rm, re, info = _gpu_ball(A, True, "valu")
    assert info == 0
    for k in (0, 5, 17, 31, 47):
        assert re[k] != oracle.RAD_INF
        dk = exact.value(D.limbs[k], D.exp[k], D.sign[k])
        r = Fraction(int(rm[k])) * Fraction(2) ** int(re[k])
        assert abs(dk - exact.cauchy_det(x[:k + 1], y[:k + 1])) <= r, k


def test_ball_zero_pivot_marks_no_bound():
    A = inputs.from_values([[1, 2, 3], [2, 4, 5], [1, 1, 1]], 4)  # second pivot zero
    LU, D, rm, re, info = _gpu_ball(A, False, "valu")
    f, orm, ore = oracle.factor_ball(A)
    assert info == f.info == 2
    assert np.array_equal(rm, orm) and np.array_equal(re, ore)
    assert re[1] == oracle.RAD_INF and re[2] == oracle.RAD_INF
