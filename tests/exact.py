"""Exact references used to pin the oracle (test-side only).

Everything here is independent of ``oracle/``: Python integers and
``fractions.Fraction`` (exact rationals), ``mpmath`` (an independent
correctly-rounded multiprecision engine), textbook determinant algorithms
(Laplace expansion, Bareiss fraction-free elimination) and closed forms
(Cauchy and Hilbert determinants).
"""
from __future__ import annotations

import math
from fractions import Fraction
from itertools import permutations

import numpy as np


# ---------------------------------------------------------------------------
# the format, decoded independently
# ---------------------------------------------------------------------------

def value(limbs, e, s) -> Fraction:
    limbs = np.ascontiguousarray(limbs, dtype="<u4")
    m = int.from_bytes(limbs.tobytes(), "little")
    if m == 0:
        return Fraction(0)
    P = limbs.shape[-1]
    v = Fraction(m) * Fraction(2) ** (int(e) - 32 * P)
    return -v if int(s) else v


def values(x) -> np.ndarray:
    """Object array of exact values of an MpArray/Mp-like container."""
    out = np.empty(x.exp.shape, dtype=object)
    for idx in np.ndindex(x.exp.shape):
        out[idx] = value(x.limbs[idx], x.exp[idx], x.sign[idx])
    return out


def truncate(q: Fraction, P: int) -> Fraction:
    """RZ_p(q) as an exact rational: keep the top p = 32P bits of |q|."""
    if q == 0:
        return Fraction(0)
    p = 32 * P
    a = abs(q)
    e = math.floor(math.log2(a.numerator)) - math.floor(math.log2(a.denominator))
    # fix e so that 2^(e-1) <= a < 2^e
    while a >= Fraction(2) ** e:
        e += 1
    while a < Fraction(2) ** (e - 1):
        e -= 1
    scale = Fraction(2) ** (p - e)
    m = math.floor(a * scale)
    r = Fraction(m) / scale
    return -r if q < 0 else r


def scalar(q: Fraction, P: int):
    """(limbs[P], e, s) of RZ_p(q), written independently of the generators."""
    t = truncate(Fraction(q), P)
    if t == 0:
        return np.zeros(P, np.uint32), 0, 0
    a = abs(t)
    p = 32 * P
    e = 0
    while a >= Fraction(2) ** e:
        e += 1
    while a < Fraction(2) ** (e - 1):
        e -= 1
    m = a * Fraction(2) ** (p - e)
    assert m.denominator == 1
    limbs = np.frombuffer(int(m).to_bytes(4 * P, "little"), "<u4").astype(np.uint32)
    return limbs, e, 1 if t < 0 else 0


# ---------------------------------------------------------------------------
# mpmath as a second, independent correctly-rounded engine
# ---------------------------------------------------------------------------

def mp_tuple(q: Fraction):
    """mpmath raw mpf tuple of an exact dyadic rational."""
    from mpmath.libmp import from_man_exp, fzero
    if q == 0:
        return fzero
    d = q.denominator
    assert d & (d - 1) == 0, "dyadic only"
    return from_man_exp(q.numerator, -(d.bit_length() - 1))


def mp_to_fraction(t) -> Fraction:
    from mpmath.libmp import fzero
    if t == fzero:
        return Fraction(0)
    sign, man, exp, _bc = t  # raw mpf: (-1)^sign * man * 2^exp
    v = Fraction(int(man)) * Fraction(2) ** int(exp)
    return -v if sign else v


def mp_op(op: str, a: Fraction, b: Fraction, P: int) -> Fraction:
    """RZ_p(a op b) computed by mpmath.libmp with rounding mode 'd' (toward zero)."""
    from mpmath import libmp
    prec = 32 * P
    fa, fb = mp_tuple(a), mp_tuple(b)
    f = {"mul": libmp.mpf_mul, "add": libmp.mpf_add, "sub": libmp.mpf_sub,
         "div": libmp.mpf_div}[op]
    return mp_to_fraction(f(fa, fb, prec, libmp.round_down))


# ---------------------------------------------------------------------------
# determinants
# ---------------------------------------------------------------------------

def det_laplace(M) -> Fraction:
    """Leibniz/Laplace expansion over all permutations (tiny N only)."""
    n = len(M)
    if n == 0:
        return Fraction(1)
    total = Fraction(0)
    for perm in permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = Fraction(1)
        for i in range(n):
            prod *= Fraction(M[i][perm[i]])
            if prod == 0:
                break
        total += -prod if inv % 2 else prod
    return total


def bareiss_leading(M) -> list[int]:
    """Bareiss fraction-free elimination on an integer matrix without pivoting.
    Its k-th pivot is the k-th leading principal minor D_k (exact)."""
    A = [[int(v) for v in row] for row in M]
    n = len(A)
    D = []
    prev = 1
    for k in range(n):
        piv = A[k][k]
        D.append(piv)
        if piv == 0:
            break
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                num = A[i][j] * piv - A[i][k] * A[k][j]
                assert num % prev == 0
                A[i][j] = num // prev
        prev = piv
    return D


def exact_ge(M):
    """Exact rational elimination without pivoting: (L multipliers, U, D list)."""
    A = [[Fraction(v) for v in row] for row in M]
    n = len(A)
    D = []
    det = Fraction(1)
    for k in range(n):
        piv = A[k][k]
        det *= piv
        D.append(det)
        if piv == 0:
            break
        for i in range(k + 1, n):
            A[i][k] = A[i][k] / piv
            z = A[i][k]
            if z:
                for j in range(k + 1, n):
                    A[i][j] -= z * A[k][j]
    return A, D


def minor(M, i, j):
    return [[M[r][c] for c in range(len(M)) if c != j] for r in range(len(M)) if r != i]


def cofactors_exact(M) -> list[list[Fraction]]:
    """C_ij = (-1)^(i+j) det(M without row i, column j), via exact GE on each minor."""
    n = len(M)
    C = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            sub = minor(M, i, j)
            C[i][j] = (-1) ** (i + j) * det_exact(sub)
    return C


def det_exact(M) -> Fraction:
    """Exact determinant by rational elimination with partial pivoting."""
    A = [[Fraction(v) for v in row] for row in M]
    n = len(A)
    det = Fraction(1)
    for k in range(n):
        p = next((r for r in range(k, n) if A[r][k] != 0), None)
        if p is None:
            return Fraction(0)
        if p != k:
            A[k], A[p] = A[p], A[k]
            det = -det
        det *= A[k][k]
        for i in range(k + 1, n):
            z = A[i][k] / A[k][k]
            if z:
                for j in range(k, n):
                    A[i][j] -= z * A[k][j]
    return det


def last_col_cofactors_exact(M) -> list[Fraction]:
    n = len(M)
    return [(-1) ** (i + n - 1) * det_exact(minor(M, i, n - 1)) for i in range(n)]


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def cauchy_det(x, y) -> Fraction:
    """det[1/(x_i - y_j)] = prod_{i<j} (x_j - x_i)(y_i - y_j) / prod_{i,j} (x_i - y_j)."""
    n = len(x)
    num = Fraction(1)
    den = Fraction(1)
    for i in range(n):
        for j in range(i + 1, n):
            num *= (Fraction(x[j]) - Fraction(x[i])) * (Fraction(y[i]) - Fraction(y[j]))
    for i in range(n):
        for j in range(n):
            den *= Fraction(x[i]) - Fraction(y[j])
    return num / den


def cauchy_det_mp(x, y, prec: int):
    """Cauchy determinant in mpmath at `prec` bits (relative error <= ~2n^2 2^-prec)."""
    import mpmath
    with mpmath.workprec(prec):
        xs = [mpmath.mpf(mp_tuple(Fraction(v))) for v in x]
        ys = [mpmath.mpf(mp_tuple(Fraction(v))) for v in y]
        n = len(xs)
        r = mpmath.mpf(1)
        for i in range(n):
            for j in range(i + 1, n):
                r *= (xs[j] - xs[i]) * (ys[i] - ys[j])
        for i in range(n):
            for j in range(n):
                r /= xs[i] - ys[j]
        return r


def cauchy_last_col_cofactors(x, y) -> list[Fraction]:
    """c_i = (-1)^(i+n) det Cauchy(x without x_i, y without y_n)."""
    n = len(x)
    out = []
    for i in range(n):
        xi = [x[k] for k in range(n) if k != i]
        out.append((-1) ** (i + n - 1) * cauchy_det(xi, y[:n - 1]))
    return out


def superfactorial(n: int) -> int:
    """c_n = prod_{k<n} k!."""
    r = 1
    f = 1
    for k in range(1, n):
        f *= k
        r *= f
    return r


def hilbert_det(n: int) -> Fraction:
    """det H_n = c_n^4 / c_{2n} with c_n = prod_{k<n} k!."""
    return Fraction(superfactorial(n) ** 4, superfactorial(2 * n))


# ---------------------------------------------------------------------------
# error in bits
# ---------------------------------------------------------------------------

def bits_agree(approx, exact) -> float:
    """-log2(|approx - exact| / |exact|) for exact rationals; inf when equal."""
    approx, exact = Fraction(approx), Fraction(exact)
    if approx == exact:
        return math.inf
    if exact == 0:
        return -math.inf
    rel = abs(approx - exact) / abs(exact)
    return -(math.log2(rel.numerator) - math.log2(rel.denominator))


def bits_agree_mp(approx, exact_mpf, prec: int) -> float:
    """Same, against an mpmath value computed at `prec` bits."""
    import mpmath
    with mpmath.workprec(prec + 64):
        a = mpmath.mpf(mp_tuple(Fraction(approx)))
        if a == exact_mpf:
            return math.inf
        return float(-mpmath.log(abs(a - exact_mpf) / abs(exact_mpf), 2))


# ---------------------------------------------------------------------------
# the method's rounding sequence, step by step in exact rationals
# ---------------------------------------------------------------------------
# Each function below executes the elimination (Algorithm 1 steps 2.1-2.2.2),
# the last-column minors (Sec. 3, [A I] derivation, solved as x^T L = e_N^T)
# and the adjugate in the orders the method fixes, with every product,
# difference and quotient formed exactly in Fractions and then truncated
# toward zero to p = 32P bits (``truncate``).  Nothing here shares code with
# the oracle; tiny sizes only.

def ge_rz(M, P: int):
    """Elimination without pivoting with two roundings per update:
    a_ij <- RZ(a_ij - RZ(l_ik a_kj)), l_ik = RZ(a_ik / a_kk),
    D_k = RZ(D_{k-1} a_kk).  Returns (LU as a list of lists, D list, info)."""
    A = [[Fraction(v) for v in row] for row in M]
    n = len(A)
    D = [Fraction(0)] * n
    for k in range(n):
        piv = A[k][k]
        if piv == 0:
            return A, D, k + 1
        D[k] = piv if k == 0 else truncate(D[k - 1] * piv, P)
        for i in range(k + 1, n):
            A[i][k] = truncate(A[i][k] / piv, P)
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                A[i][j] = truncate(A[i][j] - truncate(A[i][k] * A[k][j], P), P)
    return A, D, 0


def minors_rz(LU, D, P: int):
    """x^T L = e_N^T by sweeps j = N..2 (axpy form, one rounding per product
    and per difference), then c_i = RZ(D_{N-1} x_i), c_N = D_{N-1}."""
    n = len(LU)
    if n == 1:
        return [Fraction(1)]
    s = [Fraction(0)] * n
    for j in range(n - 1, 0, -1):
        x = Fraction(1) if j == n - 1 else s[j]
        for i in range(j):
            s[i] = truncate(s[i] - truncate(x * LU[j][i], P), P)
    c = [truncate(D[n - 2] * s[i], P) for i in range(n - 1)]
    return c + [D[n - 2]]


def adjugate_t_rz(LU, D, P: int):
    """adj(A)^T in the fixed order adj(A) = adj(U) W, W = L^-1:
    - row r of W: the minors sweep with e_r (j descending);
    - S_{N+1} = 1, S_i = RZ(u_ii S_{i+1}); adj(U)_ii = RZ(D_{i-1} S_{i+1}) (D_0 = 1
      gives S_2 itself);
    - strict upper part of adj(U): right-looking back substitution of
      U x = det(U) e_j: for k = N..2, t_i <- RZ(t_i - RZ(u_ik x_k)) for i < k,
      then x_{k-1} = RZ(t_{k-1} / u_{k-1,k-1});
    - adj(A)_im = sum over k >= max(i, m) of RZ(adj(U)_ik W_km), accumulated
      in ascending k, one rounding per product and per sum.
    Returned as T[m][i] = adj(A)_im."""
    n = len(LU)
    Z = Fraction(0)
    W = [[Z] * n for _ in range(n)]
    for r in range(n):
        W[r][r] = Fraction(1)
        for j in range(r, 0, -1):
            x = W[r][j]
            for i in range(j):
                W[r][i] = truncate(W[r][i] - truncate(x * LU[j][i], P), P)
    S = [Z] * (n + 1)
    S[n] = Fraction(1)
    for i in range(n - 1, -1, -1):
        S[i] = truncate(LU[i][i] * S[i + 1], P)
    J = [[Z] * n for _ in range(n)]
    for i in range(n):
        J[i][i] = S[1] if i == 0 else truncate(D[i - 1] * S[i + 1], P)
    for k in range(n - 1, 0, -1):
        for j in range(k, n):
            for i in range(k):
                J[i][j] = truncate(J[i][j] - truncate(LU[i][k] * J[k][j], P), P)
            J[k - 1][j] = truncate(J[k - 1][j] / LU[k - 1][k - 1], P)
    T = [[Z] * n for _ in range(n)]
    for i in range(n):
        for m in range(n):
            acc = Z
            for k in range(max(i, m), n):
                acc = truncate(acc + truncate(J[i][k] * W[k][m], P), P)
            T[m][i] = acc
    return T


def all_minors_rz(M, P: int):
    """Row r-1: minors_rz of the leading r x r block, factored afresh."""
    n = len(M)
    C = [[Fraction(0)] * n for _ in range(n)]
    for r in range(1, n + 1):
        LU, D, info = ge_rz([row[:r] for row in M[:r]], P)
        assert info == 0
        C[r - 1][:r] = minors_rz(LU, D, P)
    return C
