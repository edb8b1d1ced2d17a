"""Pins of the oracle's rigorous error bounds (ball arithmetic on the
elimination): each radius operation rounds up and stays tight (against exact
rationals), and every leading determinant's ball contains the exact leading
determinant of the input (exact rational elimination, and the closed forms
of Cauchy and Hilbert matrices), with the input exact or known only to one
unit in its last place.  A mutant that drops a term of the propagation (the
rounding of the product) leaves some exact value outside its ball."""
from fractions import Fraction

import numpy as np
import pytest

import exact
import oracle
from paper_1308_1536_amd import inputs


def rad(m, e) -> Fraction:
    assert int(e) != oracle.RAD_INF, "no bound"
    return Fraction(int(m)) * Fraction(2) ** int(e)


def _exact_leading_dets(A_host):
    M = [[Fraction(v) for v in row] for row in exact.values(A_host)]
    n = len(M)
    out, d = [], Fraction(1)
    for k in range(n):
        piv = M[k][k]
        d *= piv
        out.append(d)
        if piv == 0:
            break
        for i in range(k + 1, n):
            f = M[i][k] / piv
            for j in range(k + 1, n):
                M[i][j] -= f * M[k][j]
    return out


def _check_enclosure(A_host, input_ulp=False):
    """Every finite ball contains the exact D*_k; returns per k (bits the
    computed D_k actually agrees with D*_k, bits the ball guarantees)."""
    import math
    f, rm, re = oracle.factor_ball(A_host, input_ulp)
    assert f.info == 0
    out = []
    for k, ds in enumerate(_exact_leading_dets(A_host)):
        if re[k] == oracle.RAD_INF:  # no bound once a pivot's ball may hold zero
            assert all(e == oracle.RAD_INF for e in re[k:])
            break
        dk = exact.value(f.D.limbs[k], f.D.exp[k], f.D.sign[k])
        r = rad(rm[k], re[k])
        assert abs(dk - ds) <= r, (k, float(abs(dk - ds)), float(r))
        act = math.log2(abs(dk)) - math.log2(abs(dk - ds)) if dk != ds else math.inf
        out.append((act, math.log2(abs(dk)) - math.log2(r) if r else math.inf))
    return out


@pytest.mark.parametrize("P,n,seed", [(1, 6, 1), (1, 10, 2), (2, 12, 3), (3, 9, 4), (2, 24, 5)])
def test_ball_contains_exact_leading_determinants(P, n, seed):
    A = inputs.random_mantissas((n, n), P, 9000 + seed)
    rows = _check_enclosure(A)
    assert len(rows) >= min(n, 12)
    # a worst-case bound, pessimistic (as the paper expects of interval
    # bounds) but not useless: it gives up at most a few bits per step
    for k, (act, bnd) in enumerate(rows):
        assert bnd >= min(act, 32 * P) - (6 * k + 8), (k, act, bnd)


def test_ball_with_rounded_input_contains_the_exact_cauchy_determinants():
    """The input holds RZ of the exact Cauchy entries (one ulp each): the
    balls with input_ulp contain the closed-form leading determinants."""
    A, x, y = inputs.cauchy_dyadic(12, 2, 17)
    f, rm, re = oracle.factor_ball(A, input_ulp=True)
    for k in range(12):
        ds = exact.cauchy_det(x[:k + 1], y[:k + 1])
        dk = exact.value(f.D.limbs[k], f.D.exp[k], f.D.sign[k])
        assert abs(dk - ds) <= rad(rm[k], re[k]), k


def test_ball_hilbert_closed_form():
    n = 8
    A = inputs.hilbert(n, 4)
    f, rm, re = oracle.factor_ball(A, input_ulp=True)
    dn = exact.value(f.D.limbs[-1], f.D.exp[-1], f.D.sign[-1])
    assert abs(dn - exact.hilbert_det(n)) <= rad(rm[-1], re[-1])


def test_radius_arithmetic_rounds_up_tightly():
    """The radii as exposed: D_1's radius of a rounded input is one ulp of a_11;
    every later radius is at least the one before it times |u| (the
    propagation only adds) -- and exact input gives a zero first radius."""
    A = inputs.random_mantissas((5, 5), 2, 7)
    f0, rm0, re0 = oracle.factor_ball(A)
    assert rm0[0] == 0
    f1, rm1, re1 = oracle.factor_ball(A, input_ulp=True)
    ulp = Fraction(2) ** (int(A.exp[0, 0]) - 64)
    assert rad(rm1[0], re1[0]) == ulp
    for k in range(1, 5):
        assert rad(rm1[k], re1[k]) >= rad(rm0[k], re0[k])


def test_ball_exact_lu_products():
    """Entries of an exact L U product: every step is exact, yet the bound
    must still contain the (equal) exact values."""
    A, L, U = inputs.triangular_product(7, 2, 3)
    _check_enclosure(A)


def test_ball_survives_cancellation():
    """Nearly singular leading 2x2 blocks (d close to b c / a): the rounding of
    the multiplier and of the product l u dominate the error of D_2, so each
    of their terms in the propagation is needed for the ball to hold."""
    rng = np.random.default_rng(12)
    for t in range(60):
        P = 1 + t % 2
        a, b, c = (Fraction(int(rng.integers(1, 2 ** 30)), int(rng.integers(1, 2 ** 30))) for _ in range(3))
        d = b * c / a * (1 + Fraction(int(rng.integers(1, 1000)), 2 ** (20 + 8 * P)))
        M = [[a, b, Fraction(1)], [c, d, Fraction(2)], [Fraction(3), Fraction(5), Fraction(7)]]
        A = inputs.from_values(M, P)
        _check_enclosure(A)
