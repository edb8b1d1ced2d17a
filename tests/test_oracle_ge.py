"""Pins for the oracle's elimination, leading determinants, minors and adjugate.

What fixes the expected values (none of it is the oracle itself):
* exact cases: A = L U with integer L (unit lower) and power-of-two pivots, where
  every step of elimination without pivoting is exact, so the oracle must
  return L, U, D_k = prod u_ii and the cofactors *bit for bit*;
* Laplace expansion (N <= 6) and Bareiss fraction-free elimination, whose k-th
  pivot is the k-th leading principal minor, on integer matrices;
* the Cauchy determinant closed form (every leading block and every minor of a
  Cauchy matrix is Cauchy), and det H_n = c_n^4 / c_2n for Hilbert matrices,
  itself checked against tabulated values in tests/golden/;
* the invariants sum_i c_i a_ij = 0 (j < N) and = det (j = N) of Sec. 3;
* the prefix property of elimination without pivoting;
* a p versus 2p agreement run (the paper's accuracy method, Sec. 4.3).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import exact
from paper_1308_1536_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def vals(x):
    return exact.values(x)


def exactly_equal(x, expected):
    got = vals(x)
    return all(got[idx] == Fraction(expected[idx]) for idx in np.ndindex(got.shape))


def test_exact_case_bit_for_bit(oracle_lib):
    for N, seed in [(1, 0), (2, 1), (5, 2), (12, 3), (24, 4)]:
        A, L, U = inputs.triangular_product(N, 4, seed)
        f = oracle_lib.factor(A, threads=2)
        assert f.info == 0
        LU = vals(f.LU)
        for i in range(N):
            for j in range(N):
                want = L[i, j] if i > j else U[i, j]
                assert LU[i, j] == want, (N, i, j)
        D = vals(f.D)
        prod = Fraction(1)
        for k in range(N):
            prod *= int(U[k, k])
            assert D[k] == prod
        if N <= 7:
            c = vals(oracle_lib.minors(f))
            M = (L.astype(object) @ U.astype(object)).tolist()
            assert list(c) == exact.last_col_cofactors_exact(M)
            adjT = vals(oracle_lib.adjugate_t(f))
            C = exact.cofactors_exact(M)
            assert all(adjT[i, j] == C[i][j] for i in range(N) for j in range(N))


def test_laplace_and_bareiss_small_integer(oracle_lib):
    P = 8
    rng = np.random.default_rng(7)
    for N in range(1, 7):
        for _ in range(3):
            while True:
                M = rng.integers(-20, 21, size=(N, N))
                Dex = exact.bareiss_leading(M)
                if len(Dex) == N and all(d != 0 for d in Dex):
                    break
            A = inputs.from_values(M.astype(object), P)
            f = oracle_lib.factor(A, threads=1)
            assert f.info == 0
            D = vals(f.D)
            assert exact.det_laplace(M.tolist()) == Dex[-1]
            for k in range(N):
                assert exact.bits_agree(D[k], Dex[k]) > 32 * P - 16
            c = vals(oracle_lib.minors(f))
            cex = exact.last_col_cofactors_exact(M.tolist())
            for i in range(N):
                if cex[i] == 0:
                    assert abs(c[i]) < Fraction(1, 2 ** (32 * P - 40))
                else:
                    assert exact.bits_agree(c[i], cex[i]) > 32 * P - 24


def test_c1_random_integers_vs_bareiss(oracle_lib):
    """Config 1 random-integer matrix (N=64, 1024 bits) against exact Bareiss."""
    cfg = inputs.config_c1()
    A, M = cfg["randint"]
    f = oracle_lib.factor(A)
    assert f.info == 0
    Dex = exact.bareiss_leading(M)
    D = vals(f.D)
    worst = min(exact.bits_agree(D[k], Dex[k]) for k in range(64))
    assert worst > 900, worst
    # last-column cofactors vs exact (via exact elimination of each minor)
    c = vals(oracle_lib.minors(f))
    Ml = M.tolist()
    worst_c = min(exact.bits_agree(c[i], (-1) ** (i + 63) * exact.det_exact(exact.minor(Ml, i, 63)))
                  for i in (0, 1, 31, 62, 63))
    assert worst_c > 880, worst_c


def test_c1_cauchy_closed_forms(oracle_lib):
    """Config 1 Cauchy matrix: D_k, det and every c_i against the closed form."""
    P = 32
    A, x, y = inputs.cauchy_integer_nodes(64, P)
    f = oracle_lib.factor(A)
    assert f.info == 0
    D = vals(f.D)
    for k in (1, 2, 3, 10, 33, 64):
        assert exact.bits_agree(D[k - 1], exact.cauchy_det(x[:k], y[:k])) > 32 * P - 24
    c = vals(oracle_lib.minors(f))
    cex = exact.cauchy_last_col_cofactors(x, y)
    for i in range(0, 64, 9):
        assert exact.bits_agree(c[i], cex[i]) > 32 * P - 24


def test_hilbert_closed_form_and_table(oracle_lib):
    with open(os.path.join(GOLDEN, "hilbert_det_reciprocal.txt")) as fh:
        table = [int(line.split()[1]) for line in fh if line.strip() and not line.startswith("#")]
    for n, recip in enumerate(table, start=1):
        assert exact.hilbert_det(n) == Fraction(1, recip)
    P = 16
    for n in (4, 8, 16, 24):
        A = inputs.hilbert(n, P)
        f = oracle_lib.factor(A)
        assert f.info == 0
        det = vals(f.D)[-1]
        want = exact.hilbert_det(n)
        # H_n is ill conditioned (cond ~ e^(3.5 n), i.e. ~5n bits): the rounding
        # of the inputs alone costs about that many bits
        assert exact.bits_agree(det, want) > 32 * P - 5.1 * n - 16


def test_invariants_of_minors(oracle_lib):
    """sum_i c_i a_ij = 0 for j < N and = det for j = N (Sec. 3), exactly evaluated."""
    for A, N in [(inputs.random_mantissas((40, 40), 8, 3), 40),
                 (inputs.cauchy_dyadic(30, 8, 11)[0], 30)]:
        f = oracle_lib.factor(A)
        c = vals(oracle_lib.minors(f))
        a = vals(A)
        det = vals(f.D)[-1]
        for j in range(N):
            s = sum(c[i] * a[i, j] for i in range(N))
            scale = sum(abs(c[i] * a[i, j]) for i in range(N))
            if j < N - 1:
                assert abs(s) / scale < Fraction(1, 2 ** (256 - 40))
            else:
                assert exact.bits_agree(s, det) > 256 - 40


def test_prefix_property(oracle_lib):
    """Elimination of the leading K x K block is bit-identical to the first K
    rows/columns of the full elimination (no pivoting: step k only reads
    entries with indices >= k of the current block)."""
    A = inputs.random_mantissas((48, 48), 4, 21)
    full = oracle_lib.factor(A)
    for K in (1, 7, 30):
        sub = inputs.MpArray(A.limbs[:K, :K].copy(), A.exp[:K, :K].copy(), A.sign[:K, :K].copy())
        part = oracle_lib.factor(sub)
        assert np.array_equal(part.D.limbs, full.D.limbs[:K])
        assert np.array_equal(part.D.exp, full.D.exp[:K])
        assert np.array_equal(part.D.sign, full.D.sign[:K])
        assert np.array_equal(part.LU.limbs, full.LU.limbs[:K, :K])


def test_all_minors_exact_case_and_cofactors(oracle_lib):
    """Every row of all_minors against the exact last-column cofactors of its
    leading block: bit for bit in the exact case (integer L, power-of-two
    pivots), to within rounding on small random integer matrices (Laplace)."""
    A, L, U = inputs.triangular_product(7, 4, 9)
    C = vals(oracle_lib.all_minors(A, threads=2))
    M = (L.astype(object) @ U.astype(object)).tolist()
    for r in range(1, 8):
        block = [row[:r] for row in M[:r]]
        assert list(C[r - 1, :r]) == exact.last_col_cofactors_exact(block), r
        assert all(C[r - 1, i] == 0 for i in range(r, 7))
    P = 8
    rng = np.random.default_rng(17)
    while True:
        Mi = rng.integers(-20, 21, size=(6, 6))
        if all(d != 0 for d in exact.bareiss_leading(Mi)):
            break
    C = vals(oracle_lib.all_minors(inputs.from_values(Mi.astype(object), P), threads=1))
    for r in range(1, 7):
        cex = exact.last_col_cofactors_exact(Mi[:r, :r].tolist())
        for i in range(r):
            if cex[i] == 0:
                assert abs(C[r - 1, i]) < Fraction(1, 2 ** (32 * P - 40))
            else:
                assert exact.bits_agree(C[r - 1, i], cex[i]) > 32 * P - 24, (r, i)


def test_all_minors_invariants(oracle_lib):
    """sum_i C[r-1][i] a_ij = 0 for j < r and = D_r for j = r (Sec. 3, each
    leading block), exactly evaluated on a random and a Cauchy matrix."""
    for A in (inputs.random_mantissas((24, 24), 8, 31), inputs.cauchy_dyadic(20, 8, 12)[0]):
        N = int(A.exp.shape[0])
        C = vals(oracle_lib.all_minors(A))
        a = vals(A)
        D = vals(oracle_lib.factor(A).D)
        for r in range(1, N + 1):
            for j in range(r):
                s = sum(C[r - 1, i] * a[i, j] for i in range(r))
                scale = sum(abs(C[r - 1, i] * a[i, j]) for i in range(r))
                if j < r - 1:
                    assert abs(s) / scale < Fraction(1, 2 ** (256 - 40)), (r, j)
                else:
                    assert exact.bits_agree(s, D[r - 1]) > 256 - 40, r


def test_thread_count_does_not_change_bits(oracle_lib):
    A = inputs.random_mantissas((33, 33), 3, 5)
    a = oracle_lib.factor(A, threads=1)
    b = oracle_lib.factor(A, threads=7)
    for x, y in ((a.LU, b.LU), (a.D, b.D)):
        assert np.array_equal(x.limbs, y.limbs) and np.array_equal(x.exp, y.exp)
        assert np.array_equal(x.sign, y.sign)
    ca, cb = oracle_lib.minors(a, threads=1), oracle_lib.minors(b, threads=5)
    assert np.array_equal(ca.limbs, cb.limbs) and np.array_equal(ca.exp, cb.exp)


def test_singular_last_pivot_keeps_minors(oracle_lib):
    """Only the last pivot is zero (A = L U with u_nn = 0, every step exact):
    info = n and D_n = 0, while the last-column minors and the adjugate --
    which never divide by u_nn -- are the exact cofactors of the singular
    matrix (eq. (minors) needs them exactly where det vanishes)."""
    for N, seed in [(2, 3), (4, 5), (6, 7)]:
        A, L, U = inputs.triangular_product(N, 4, seed)
        U[N - 1, N - 1] = 0
        M = (L.astype(object) @ U.astype(object))
        A = inputs.from_values(M, 4)
        f = oracle_lib.factor(A, threads=2)
        assert f.info == N
        D = vals(f.D)
        assert D[N - 1] == 0 and all(D[k] != 0 for k in range(N - 1))
        c = vals(oracle_lib.minors(f))
        assert list(c) == exact.last_col_cofactors_exact(M.tolist())
        adjT = vals(oracle_lib.adjugate_t(f))
        C = exact.cofactors_exact(M.tolist())
        assert all(adjT[i, j] == C[i][j] for i in range(N) for j in range(N))
        assert sum(c[i] * M[i, N - 1] for i in range(N)) == 0


def test_zero_pivot_and_overflow_info(oracle_lib):
    P = 2
    M = [[0, 1, 2], [3, 4, 5], [6, 7, 9]]
    f = oracle_lib.factor(inputs.from_values(M, P))
    assert f.info == 1 and not f.D.limbs.any() and not f.D.exp.any()
    M = [[1, 2, 3], [2, 4, 5], [1, 0, 1]]  # singular leading 2x2
    A = inputs.from_values(M, P)
    f = oracle_lib.factor(A)
    assert f.info == 2
    assert vals(f.D)[0] == 1 and not f.D.limbs[1:].any()
    # state after step 1 is kept: row 2 multiplier 2, a_22 = 0
    LU = vals(f.LU)
    assert LU[1, 0] == 2 and LU[1, 1] == 0 and LU[1, 2] == -1
    with pytest.raises(ValueError):
        oracle_lib.minors(f)
    # exponent overflow of the leading determinant
    A = inputs.from_values([[1, 0], [0, 1]], P)
    A.exp[0, 0] = 2 ** 62
    A.exp[1, 1] = 2 ** 62
    assert oracle_lib.factor(A).info == -1
    A.exp[1, 1] = 1
    assert oracle_lib.factor(A).info == 0


def test_n1_and_empty(oracle_lib):
    P = 2
    A = inputs.from_values([[Fraction(-3, 8)]], P)
    f = oracle_lib.factor(A)
    assert f.info == 0 and vals(f.D)[0] == Fraction(-3, 8)
    assert vals(oracle_lib.minors(f))[0] == 1
    assert vals(oracle_lib.adjugate_t(f))[0, 0] == 1
    E = inputs.MpArray.zeros((0, 0), P)
    f = oracle_lib.factor(E)
    assert f.info == 0 and f.D.exp.shape == (0,)


def test_adjugate_against_cofactors_and_minors(oracle_lib):
    P = 6
    rng = np.random.default_rng(3)
    M = rng.integers(-9, 10, size=(6, 6))
    while any(d == 0 for d in exact.bareiss_leading(M)) or len(exact.bareiss_leading(M)) < 6:
        M = rng.integers(-9, 10, size=(6, 6))
    A = inputs.from_values(M.astype(object), P)
    f = oracle_lib.factor(A)
    adjT = vals(oracle_lib.adjugate_t(f))
    C = exact.cofactors_exact(M.tolist())
    for i in range(6):
        for j in range(6):
            if C[i][j] == 0:
                assert abs(adjT[i, j]) < Fraction(1, 2 ** 150)
            else:
                assert exact.bits_agree(adjT[i, j], C[i][j]) > 32 * P - 24
    # column N of adj(A)^T is the minors vector, bit for bit
    B = inputs.random_mantissas((20, 20), 3, 8)
    fb = oracle_lib.factor(B)
    t = oracle_lib.adjugate_t(fb)
    c = oracle_lib.minors(fb)
    assert np.array_equal(t.limbs[:, -1], c.limbs) and np.array_equal(t.exp[:, -1], c.exp)
    assert np.array_equal(t.sign[:, -1], c.sign)
    # A adj(A) = det I, evaluated exactly
    a = vals(B)
    tv = vals(t)
    det = vals(fb.D)[-1]
    for i in (0, 7, 19):
        for m in (0, 11, 19):
            s = sum(a[i, k] * tv[m, k] for k in range(20))
            scale = sum(abs(a[i, k] * tv[m, k]) for k in range(20))
            if i == m:
                assert exact.bits_agree(s, det) > 96 - 40
            else:
                assert abs(s) / scale < Fraction(1, 2 ** (96 - 40))


def test_p_vs_2p_agreement(oracle_lib):
    """The paper's accuracy method: the same matrix at p and 2p bits; the
    leading determinants agree to roughly p bits minus a slowly growing loss."""
    A = inputs.random_mantissas((32, 32), 4, 99)
    A2 = inputs.MpArray(np.concatenate([np.zeros_like(A.limbs), A.limbs], axis=-1),
                        A.exp.copy(), A.sign.copy())
    f1, f2 = oracle_lib.factor(A), oracle_lib.factor(A2)
    d1, d2 = vals(f1.D), vals(f2.D)
    for k in range(32):
        assert exact.bits_agree(d1[k], d2[k]) > 128 - 40


def test_normalize_minors_is_rz_of_the_exact_ratio(oracle_lib):
    """The normalised minors of eq. (minors): in the exact case the minors are
    the exact cofactors, so row entry i must be RZ_p(c_i / c_1) of the exact
    rational (same sign, below it in magnitude by less than one unit in the
    last place); the first entry is exactly 1, and a row starting with zero
    gives zeros."""
    P = 4
    A, L, U = inputs.triangular_product(7, P, 9)
    C = oracle_lib.all_minors(A)
    Nrm = vals(oracle_lib.normalize_minors(C))
    M = (L.astype(object) @ U.astype(object)).tolist()
    for r in range(1, 8):
        c = exact.last_col_cofactors_exact([row[:r] for row in M[:r]])
        assert Nrm[r - 1, 0] == 1
        for i in range(r):
            want = Fraction(c[i], c[0])
            got = Nrm[r - 1, i]
            if want == 0:
                assert got == 0
                continue
            assert (got > 0) == (want > 0) and abs(got) <= abs(want)
            ulp = Fraction(2) ** (math.floor(math.log2(abs(got))) - (32 * P - 1))
            assert abs(want) - abs(got) < ulp, (r, i)
    Z = inputs.from_values([[0, 1, 2]], P)
    assert not oracle_lib.normalize_minors(Z).limbs.any()
