"""Pins of the oracle's step ranges and truncation, the pieces of the
reduced-precision elimination: a truncation is RZ of the exact value to the
shorter precision (checked against exact rationals), step ranges applied in
order give the whole elimination, and the reduced pipeline is the
composition it is defined as (full-precision steps, truncation, the rest at
the shorter precision) with the pieces checked independently: at k_switch =
n it is the truncated full-precision result, at k_switch = 0 the elimination
of the truncated input."""
import numpy as np
import pytest

import exact
import oracle
from paper_1308_1536_amd import inputs


def test_truncate_is_rz_of_the_exact_value():
    rng = np.random.default_rng(5)
    x = inputs.random_mantissas((40,), 6, 3)
    for P2 in (1, 2, 3, 6):  # the oracle takes any limb count
        y = oracle.truncate(x, P2)
        for i in range(40):
            v = exact.value(x.limbs[i], x.exp[i], x.sign[i])
            l, e, s = exact.scalar(v, P2)   # exact value, then RZ to 32 P2 bits
            assert np.array_equal(y.limbs[i], l) and y.exp[i] == e and y.sign[i] == s
    z = inputs.MpArray.zeros((3,), 4)
    assert not oracle.truncate(z, 2).limbs.any()
    _ = rng


@pytest.mark.parametrize("cuts", [[0, 17], [5], [1, 2, 3], [16]])
def test_factor_ranges_compose_to_the_whole(cuts):
    A = inputs.random_mantissas((17, 17), 3, 11)
    whole = oracle.factor(A)
    n = 17
    f = oracle.Factorization(oracle._as_mp(A).copy(), oracle._zeros((n,), 3), 0)
    edges = [0] + [c for c in cuts if 0 < c < n] + [n]
    for a, b in zip(edges[:-1], edges[1:]):
        f = oracle.factor_range(f, a, b)
    assert f.info == whole.info
    for got, want in ((f.LU, whole.LU), (f.D, whole.D)):
        assert np.array_equal(got.limbs, want.limbs) and np.array_equal(got.exp, want.exp)
        assert np.array_equal(got.sign, want.sign)


def test_reduced_pipeline_end_points():
    A = inputs.random_mantissas((14, 14), 4, 21)
    n, P2 = 14, 2
    # k_switch = n: every step at full precision, then truncated
    f, c, lead = oracle.det_pipeline_reduced(A, n, P2)
    full = oracle.factor(A)
    t = oracle.truncate(full.D, P2)
    assert np.array_equal(f.D.limbs, t.limbs) and np.array_equal(f.D.exp, t.exp)
    assert np.array_equal(lead.limbs, full.D.limbs)
    # k_switch = 0: the elimination of the truncated input
    f0, c0, _ = oracle.det_pipeline_reduced(A, 0, P2)
    g, cg = oracle.det_pipeline(oracle.truncate(A, P2))
    assert np.array_equal(f0.LU.limbs, g.LU.limbs) and np.array_equal(f0.D.limbs, g.D.limbs)
    assert np.array_equal(c0.limbs, cg.limbs)


def test_reduced_precision_error_is_bounded_by_the_shorter_precision():
    """Cauchy matrix, closed-form det: switching to half the precision half
    way leaves the determinant accurate to about the shorter precision."""
    A, x, y = inputs.cauchy_dyadic(16, 8, 4)
    f, c, lead = oracle.det_pipeline_reduced(A, 8, 4)
    want = exact.cauchy_det(x, y)
    got = exact.value(f.D.limbs[-1], f.D.exp[-1], f.D.sign[-1])
    assert exact.bits_agree(got, want) > 128 - 16
