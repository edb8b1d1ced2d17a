"""CPU oracle for multiprecision Gaussian elimination without pivoting.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1308_1536_amd``) never imports, loads or calls it, and the two share no
code: this package wraps ``mpref.c`` (plain C, its own limb bignum, OpenMP row
blocks), which is an independent, deliberately plain implementation of:

* the number format: value = (-1)^s * m * 2^(e - 32P), m with P little-endian
  uint32 limbs and its top bit set, canonical zero (s = e = m = 0);
* RZ_p (exact result, then truncation toward zero to p = 32P bits) for
  multiplication, addition, subtraction and division;
* Gaussian elimination without pivoting, Algorithm 1 steps 1-2.2.2 of the paper
  (multipliers stored below the diagonal, Sec. 3 storage paragraph);
* the leading determinants D_k (Algorithm 1 step 2.1);
* the signed last-column minors from the [A I] derivation (Sec. 3);
* the adjugate adj(A)^T = d det / d A (Sec. 3, Baur-Strassen remark);
* the last-column minors of every leading block (the minors above applied to
  each leading block, factored afresh), and the normalised minors (each row
  divided by its first entry, eq. (minors));
* conversion of a number to a (float64 mantissa, int64 exponent) pair.

Arrays use the element-contiguous host layout: limbs [..., P] uint32,
exp [...] int64, sign [...] int32.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpref.c")
_LIB = os.path.join(_HERE, "libmpref.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile mpref.c into libmpref.so with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        num = [ctypes.c_int32, _u32p, ctypes.c_int64, ctypes.c_int32,
               _u32p, ctypes.c_int64, ctypes.c_int32, _u32p, _i64p, _i32p]
        for name in ("mpref_mul", "mpref_add", "mpref_sub"):
            getattr(lib, name).argtypes = num
            getattr(lib, name).restype = None
        lib.mpref_div.argtypes = num
        lib.mpref_div.restype = ctypes.c_int
        lib.mpref_bn_mul.argtypes = [_u32p, _u32p, ctypes.c_int32, _u32p, ctypes.c_int32]
        lib.mpref_bn_mul.restype = None
        lib.mpref_bn_divmod.argtypes = [_u32p, _u32p, _u32p, ctypes.c_int32, _u32p,
                                        ctypes.c_int32]
        lib.mpref_bn_divmod.restype = ctypes.c_int
        mat = [ctypes.c_int64, ctypes.c_int32, _u32p, _i64p, _i32p]
        lib.mpref_factor.argtypes = mat + [_u32p, _i64p, _i32p, _i32p, ctypes.c_int32]
        lib.mpref_factor.restype = ctypes.c_int
        lib.mpref_factor_range.argtypes = mat + [_u32p, _i64p, _i32p, _i32p, ctypes.c_int64, ctypes.c_int64,
                                                 ctypes.c_int32]
        lib.mpref_factor_range.restype = ctypes.c_int
        lib.mpref_truncate.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _u32p, _i64p, _i32p,
                                       _u32p, _i64p, _i32p]
        lib.mpref_truncate.restype = ctypes.c_int
        lib.mpref_factor_ball.argtypes = mat + [_u32p, _i64p, _i32p, _i32p, ctypes.c_int32, _u32p, _i64p,
                                                ctypes.c_int32]
        lib.mpref_factor_ball.restype = ctypes.c_int
        lib.mpref_minors.argtypes = mat + [_u32p, _i64p, _i32p, _u32p, _i64p, _i32p,
                                           ctypes.c_int32]
        lib.mpref_minors.restype = ctypes.c_int
        lib.mpref_adjugate_t.argtypes = mat + [_u32p, _i64p, _i32p, _u32p, _i64p, _i32p,
                                               ctypes.c_int32]
        lib.mpref_adjugate_t.restype = ctypes.c_int
        lib.mpref_to_f64.argtypes = [ctypes.c_int64, ctypes.c_int32, _u32p, _i64p, _i32p,
                                     _f64p, _i64p]
        lib.mpref_to_f64.restype = None
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


@dataclass
class Mp:
    """Numbers in the host layout: limbs [..., P], exp [...], sign [...]."""
    limbs: np.ndarray
    exp: np.ndarray
    sign: np.ndarray

    @property
    def P(self) -> int:
        return int(self.limbs.shape[-1])

    def copy(self) -> "Mp":
        return Mp(self.limbs.copy(), self.exp.copy(), self.sign.copy())


def _as_mp(x) -> Mp:
    return Mp(np.ascontiguousarray(x.limbs, dtype=np.uint32),
              np.ascontiguousarray(x.exp, dtype=np.int64),
              np.ascontiguousarray(x.sign, dtype=np.int32))


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _zeros(shape, P) -> Mp:
    return Mp(np.zeros(tuple(shape) + (P,), np.uint32), np.zeros(shape, np.int64),
              np.zeros(shape, np.int32))


def _binop(name, a, b):
    a, b = _as_mp(a), _as_mp(b)
    P = a.P
    r = _zeros((), P)
    fn = getattr(_load(), name)
    rc = fn(P, _p(a.limbs, _u32p), int(a.exp.reshape(())), int(a.sign.reshape(())), _p(b.limbs, _u32p),
            int(b.exp.reshape(())), int(b.sign.reshape(())), _p(r.limbs, _u32p), _p(r.exp, _i64p),
            _p(r.sign, _i32p))
    if rc not in (None, 0):
        raise ZeroDivisionError("mpref_div: division by zero")
    return r


def mul(a, b) -> Mp:
    """RZ_p(a * b) of two scalars (limbs shape [P])."""
    return _binop("mpref_mul", a, b)


def add(a, b) -> Mp:
    """RZ_p(a + b)."""
    return _binop("mpref_add", a, b)


def sub(a, b) -> Mp:
    """RZ_p(a - b)."""
    return _binop("mpref_sub", a, b)


def div(a, b) -> Mp:
    """RZ_p(a / b); raises ZeroDivisionError for b == 0."""
    return _binop("mpref_div", a, b)


def bn_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    out = np.zeros(a.size + b.size, np.uint32)
    _load().mpref_bn_mul(_p(out, _u32p), _p(a, _u32p), a.size, _p(b, _u32p), b.size)
    return out


def bn_divmod(u: np.ndarray, v: np.ndarray):
    u = np.ascontiguousarray(u, np.uint32)
    v = np.ascontiguousarray(v, np.uint32)
    q = np.zeros(u.size - v.size + 1, np.uint32)
    r = np.zeros(v.size, np.uint32)
    rc = _load().mpref_bn_divmod(_p(q, _u32p), _p(r, _u32p), _p(u, _u32p), u.size,
                                 _p(v, _u32p), v.size)
    if rc != 0:
        raise ValueError("mpref_bn_divmod: bad argument")
    return q, r


@dataclass
class Factorization:
    LU: Mp        # U on/above the diagonal, multipliers below
    D: Mp         # D_1..D_n
    info: int     # 0 ok, k>0 zero pivot at step k, -1 exponent overflow


def factor(A, threads: int | None = None) -> Factorization:
    """Gaussian elimination without pivoting on a copy of A (Algorithm 1)."""
    A = _as_mp(A).copy()
    n = int(A.exp.shape[0])
    if A.exp.shape != (n, n):
        raise ValueError("factor: A must be square")
    P = A.P
    D = _zeros((n,), P)
    info = np.zeros((), np.int32)
    rc = _load().mpref_factor(n, P, _p(A.limbs, _u32p), _p(A.exp, _i64p), _p(A.sign, _i32p),
                              _p(D.limbs, _u32p), _p(D.exp, _i64p), _p(D.sign, _i32p),
                              _p(info, _i32p), threads or default_threads())
    if rc != 0:
        raise ValueError("mpref_factor: bad argument")
    return Factorization(A, D, int(info))


def _complete(f: Factorization, n: int) -> bool:
    """Elimination ran all its steps: info 0, or info n (only the last pivot
    u_nn is zero, so det = 0 while the minors and the adjugate, which never
    divide by u_nn, stay defined -- eq. (minors) needs them where det = 0)."""
    return f.info == 0 or f.info == n


def minors(f: Factorization, threads: int | None = None) -> Mp:
    """Signed last-column cofactors c (c . A[:, n] = det) from a factorization."""
    LU, D = _as_mp(f.LU), _as_mp(f.D)
    n, P = int(LU.exp.shape[0]), LU.P
    if not _complete(f, n):
        raise ValueError("minors: factorization did not complete (info=%d)" % f.info)
    c = _zeros((n,), P)
    rc = _load().mpref_minors(n, P, _p(LU.limbs, _u32p), _p(LU.exp, _i64p),
                              _p(LU.sign, _i32p), _p(D.limbs, _u32p), _p(D.exp, _i64p),
                              _p(D.sign, _i32p), _p(c.limbs, _u32p), _p(c.exp, _i64p),
                              _p(c.sign, _i32p), threads or default_threads())
    if rc != 0:
        raise ValueError("mpref_minors: bad argument")
    return c


def adjugate_t(f: Factorization, threads: int | None = None) -> Mp:
    """adj(A)^T = d det / d A from a factorization (column n equals minors())."""
    LU, D = _as_mp(f.LU), _as_mp(f.D)
    n, P = int(LU.exp.shape[0]), LU.P
    if not _complete(f, n):
        raise ValueError("adjugate_t: factorization did not complete (info=%d)" % f.info)
    t = _zeros((n, n), P)
    rc = _load().mpref_adjugate_t(n, P, _p(LU.limbs, _u32p), _p(LU.exp, _i64p),
                                  _p(LU.sign, _i32p), _p(D.limbs, _u32p), _p(D.exp, _i64p),
                                  _p(D.sign, _i32p), _p(t.limbs, _u32p), _p(t.exp, _i64p),
                                  _p(t.sign, _i32p), threads or default_threads())
    if rc != 0:
        raise ValueError("mpref_adjugate_t: bad argument")
    return t


def all_minors(A, threads: int | None = None) -> Mp:
    """The last-column cofactors of every leading block: row r-1 is minors()
    of the factorization of A_r, the leading r x r block, on its first r
    entries (eq. (minorsdef) per block), zeros above the diagonal.  Each block
    is factored afresh from A, so nothing is shared between rows."""
    A = _as_mp(A)
    n = int(A.exp.shape[0])
    if A.exp.shape != (n, n):
        raise ValueError("all_minors: A must be square")
    C = _zeros((n, n), A.P)
    for r in range(1, n + 1):
        block = Mp(A.limbs[:r, :r].copy(), A.exp[:r, :r].copy(), A.sign[:r, :r].copy())
        f = factor(block, threads)
        if not _complete(f, r):
            raise ValueError("all_minors: leading block %d did not factor (info=%d)" % (r, f.info))
        c = minors(f, threads)
        C.limbs[r - 1, :r], C.exp[r - 1, :r], C.sign[r - 1, :r] = c.limbs, c.exp, c.sign
    return C


def normalize_minors(C) -> Mp:
    """The normalised minors of eq. (minors): every row of C divided by its
    first entry, RZ_p(C[r][i] / C[r][0]); a row whose first entry is zero
    becomes zeros."""
    C = _as_mp(C)
    if C.exp.ndim == 1:
        C = Mp(C.limbs[None], C.exp[None], C.sign[None])
    rows, cols = C.exp.shape
    out = _zeros((rows, cols), C.P)
    for r in range(rows):
        den = Mp(C.limbs[r, 0], C.exp[r, 0], C.sign[r, 0])
        if not den.limbs.any():
            continue
        for i in range(cols):
            q = div(Mp(C.limbs[r, i], C.exp[r, i], C.sign[r, i]), den)
            out.limbs[r, i], out.exp[r, i], out.sign[r, i] = q.limbs, q.exp, q.sign
    return out


def to_f64(x) -> tuple[np.ndarray, np.ndarray]:
    """(mantissa in +-[0.5, 1) truncated to 53 bits, int64 exponent) per number."""
    x = _as_mp(x)
    P = x.P
    cnt = int(x.exp.size)
    mant = np.zeros(x.exp.shape, np.float64)
    ex = np.zeros(x.exp.shape, np.int64)
    _load().mpref_to_f64(cnt, P, _p(x.limbs, _u32p), _p(x.exp, _i64p), _p(x.sign, _i32p),
                         _p(mant, _f64p), _p(ex, _i64p))
    return mant, ex


def factor_range(f: Factorization, k_begin: int, k_end: int, threads: int | None = None) -> Factorization:
    """Elimination steps k_begin .. k_end-1 continued from the state of f (a
    copy); Algorithm 1's steps in order, each reading only what the steps
    before it left."""
    LU = f.LU.copy()
    D = f.D.copy()
    n, P = int(LU.exp.shape[0]), LU.P
    info = np.array(f.info, np.int32)
    rc = _load().mpref_factor_range(n, P, _p(LU.limbs, _u32p), _p(LU.exp, _i64p), _p(LU.sign, _i32p),
                                    _p(D.limbs, _u32p), _p(D.exp, _i64p), _p(D.sign, _i32p), _p(info, _i32p),
                                    int(k_begin), int(k_end), threads or default_threads())
    if rc != 0:
        raise ValueError("mpref_factor_range: bad argument")
    return Factorization(LU, D, int(info))


RAD_INF = np.iinfo(np.int64).max


def factor_ball(A, input_ulp: bool = False, threads: int | None = None):
    """factor(A) and a rigorous radius per leading determinant: |D_k - D*_k| <=
    rad_m[k] * 2^rad_e[k] (D*_k exact; rad_e == RAD_INF: no bound).  Returns
    (Factorization, rad_m uint32[n], rad_e int64[n])."""
    A = _as_mp(A).copy()
    n = int(A.exp.shape[0])
    P = A.P
    D = _zeros((n,), P)
    info = np.zeros((), np.int32)
    rm = np.zeros(n, np.uint32)
    re = np.zeros(n, np.int64)
    rc = _load().mpref_factor_ball(n, P, _p(A.limbs, _u32p), _p(A.exp, _i64p), _p(A.sign, _i32p),
                                   _p(D.limbs, _u32p), _p(D.exp, _i64p), _p(D.sign, _i32p), _p(info, _i32p),
                                   1 if input_ulp else 0, _p(rm, _u32p), _p(re, _i64p), threads or default_threads())
    if rc != 0:
        raise ValueError("mpref_factor_ball: bad argument")
    return Factorization(A, D, int(info)), rm, re


def truncate(x, P2: int) -> Mp:
    """RZ to 32 * P2 bits of every number of x (P2 <= x's limbs)."""
    x = _as_mp(x)
    out = _zeros(x.exp.shape, P2)
    rc = _load().mpref_truncate(int(x.exp.size), x.P, int(P2), _p(np.ascontiguousarray(x.limbs), _u32p),
                                _p(np.ascontiguousarray(x.exp), _i64p), _p(np.ascontiguousarray(x.sign), _i32p),
                                _p(out.limbs, _u32p), _p(out.exp, _i64p), _p(out.sign, _i32p))
    if rc != 0:
        raise ValueError("mpref_truncate: bad argument")
    return out


def det_pipeline_reduced(A, k_switch: int, P2: int, threads: int | None = None):
    """The elimination with reduced precision in its later steps (Sec. 4.3's
    remark that the later iterations need not run at full precision): steps
    0 .. k_switch-1 at A's precision, then the whole state (the factored
    matrix so far and D_1..D_{k_switch}) truncated to 32 * P2 bits, the
    remaining steps and the minors at that precision.  Returns
    (Factorization at P2, c or None, D_1..D_{k_switch} at full precision)."""
    A = _as_mp(A)
    n = int(A.exp.shape[0])
    f0 = Factorization(A.copy(), _zeros((n,), A.P), 0)
    f1 = factor_range(f0, 0, k_switch, threads)
    lead = f1.D.copy()
    f2 = Factorization(truncate(f1.LU, P2), truncate(f1.D, P2), f1.info)
    f3 = factor_range(f2, k_switch, n, threads)
    c = minors(f3, threads) if _complete(f3, n) else None
    return f3, c, lead


def det_pipeline(A, threads: int | None = None):
    """factor + minors, the whole hot path: returns (Factorization, c or None)."""
    f = factor(A, threads)
    n = int(f.LU.exp.shape[0])
    c = minors(f, threads) if _complete(f, n) else None
    return f, c
