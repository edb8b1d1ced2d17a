"""Pins of the oracle's rounding sequence.

The method is a fixed sequence of truncated operations (Algorithm 1 steps
2.1-2.2.2; the minors from the [A I] derivation of Sec. 3; the adjugate as
the gradient of det, Sec. 3), so its results depend on where every rounding
falls, not only on the operations' definitions.  ``exact.ge_rz``,
``exact.minors_rz``, ``exact.adjugate_t_rz`` and ``exact.all_minors_rz``
execute that sequence in exact rationals with a truncation to p bits after
every product, difference, sum and quotient; these tests require the oracle
to agree with them bit for bit on inputs where nearly every step rounds
(random full-precision mantissas, Cauchy matrices at one and two limbs).  A
fused multiply-subtract, a single rounding of D_k, another sweep order of the
minors solve or another accumulation order of the adjugate each change some
of these bits.
"""
from fractions import Fraction

import numpy as np
import pytest

import exact
from paper_1308_1536_amd import inputs


def _vals(x):
    return exact.values(x)


def _cases():
    out = []
    for P in (1, 2):
        for N, seed in ((1, 11), (2, 12), (3, 13), (5, 14), (7, 15), (8, 16)):
            out.append(("randmant", P, N, inputs.random_mantissas((N, N), P, 5000 + 10 * seed + P)))
        for N, seed in ((4, 21), (6, 22)):
            x, y = inputs.dyadic_nodes(N, 6000 + seed, 0.0, 10.0)
            out.append(("cauchy", P, N, inputs.cauchy(x, y, P)))
    return out


CASES = _cases()


def _ids():
    return [f"{name}-P{P}-N{N}" for name, P, N, _ in CASES]


@pytest.mark.parametrize("case", CASES, ids=_ids())
def test_factor_and_minors_sequence(oracle_lib, case):
    _name, P, N, A = case
    M = _vals(A).tolist()
    LUx, Dx, infox = exact.ge_rz(M, P)
    f = oracle_lib.factor(A, threads=1)
    assert f.info == infox == 0
    LU = _vals(f.LU)
    D = _vals(f.D)
    for i in range(N):
        for j in range(N):
            assert LU[i, j] == LUx[i][j], ("LU", i, j)
    for k in range(N):
        assert D[k] == Dx[k], ("D", k)
    c = _vals(oracle_lib.minors(f, threads=1))
    cx = exact.minors_rz(LUx, Dx, P)
    assert list(c) == cx


@pytest.mark.parametrize("case", [c for c in CASES if c[2] <= 7], ids=[i for i, c in zip(_ids(), CASES) if c[2] <= 7])
def test_adjugate_sequence(oracle_lib, case):
    _name, P, N, A = case
    M = _vals(A).tolist()
    LUx, Dx, _ = exact.ge_rz(M, P)
    f = oracle_lib.factor(A, threads=1)
    T = _vals(oracle_lib.adjugate_t(f, threads=2))
    Tx = exact.adjugate_t_rz(LUx, Dx, P)
    for m in range(N):
        for i in range(N):
            assert T[m, i] == Tx[m][i], ("adjT", m, i)


@pytest.mark.parametrize("P", [1, 2])
def test_all_minors_sequence(oracle_lib, P):
    N = 6
    A = inputs.random_mantissas((N, N), P, 7100 + P)
    C = _vals(oracle_lib.all_minors(A, threads=1))
    Cx = exact.all_minors_rz(_vals(A).tolist(), P)
    for r in range(N):
        for i in range(N):
            assert C[r, i] == Cx[r][i], ("C", r, i)


def test_sequence_reference_is_not_exact_arithmetic():
    """The cases above round: the step-by-step reference differs from exact
    elimination on them (otherwise they could not tell roundings apart)."""
    _name, P, N, A = next(c for c in CASES if c[0] == "randmant" and c[1] == 1 and c[2] == 7)
    M = _vals(A).tolist()
    LUx, Dx, _ = exact.ge_rz(M, P)
    Ex, DEx = exact.exact_ge(M)
    differ = sum(1 for i in range(N) for j in range(N) if Fraction(LUx[i][j]) != Ex[i][j])
    assert differ >= N * N // 2
    assert Dx[-1] != DEx[-1]


def test_two_roundings_differ_from_one():
    """RZ(a - RZ(l u)) and RZ(a - l u) differ on some of these inputs, so the
    factor test above fixes the granularity of the update (two roundings)."""
    rng = np.random.default_rng(3)
    P = 1
    seen = False
    for _ in range(200):
        a, l, u = (inputs.decode(inputs.random_mantissas((1, 1), P, int(rng.integers(1 << 30))), (0, 0))
                   for _ in range(3))
        two = exact.truncate(a - exact.truncate(l * u, P), P)
        one = exact.truncate(a - l * u, P)
        if two != one:
            seen = True
            break
    assert seen
