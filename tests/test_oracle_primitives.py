"""Pins for the oracle's big-integer helpers and RZ_p primitives.

Each primitive is checked against two engines that share nothing with the
oracle: Python integers / ``fractions.Fraction`` (exact value, then truncation
toward zero written out in the test) and ``mpmath.libmp`` with rounding mode
``'d'`` (round toward zero).  Adversarial cases cover exponent gaps from 0 to
beyond the clamp, exact cancellation, powers of two, all-ones mantissas and
zero operands.
"""
from fractions import Fraction

import numpy as np
import pytest

import exact

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def rand_int(rng, bits):
    return int.from_bytes(rng.bytes((bits + 7) // 8), "little") % (1 << bits)


def to_limbs(v, n):
    return np.frombuffer(v.to_bytes(4 * n, "little"), "<u4").astype(np.uint32)


def from_limbs(a):
    return int.from_bytes(np.ascontiguousarray(a, "<u4").tobytes(), "little")


def test_bn_mul_matches_python_int(oracle_lib):
    rng = np.random.default_rng(1)
    for na, nb in [(1, 1), (1, 7), (5, 3), (32, 32), (64, 17), (128, 128)]:
        for _ in range(5):
            a = rand_int(rng, 32 * na)
            b = rand_int(rng, 32 * nb)
            out = oracle_lib.bn_mul(to_limbs(a, na), to_limbs(b, nb))
            assert from_limbs(out) == a * b
    # all-ones operands maximise every carry
    a = (1 << (32 * 40)) - 1
    assert from_limbs(oracle_lib.bn_mul(to_limbs(a, 40), to_limbs(a, 40))) == a * a


def test_bn_divmod_matches_python_divmod(oracle_lib):
    rng = np.random.default_rng(2)
    cases = []
    for m, n in [(1, 1), (3, 1), (4, 2), (9, 4), (33, 16), (65, 32), (257, 128)]:
        for _ in range(6):
            v = rand_int(rng, 32 * n) | (1 << (32 * n - 1 - int(rng.integers(0, 31))))
            u = rand_int(rng, 32 * m)
            cases.append((u, v, m, n))
    # quotient digits that need the add-back correction / qhat = B-1 paths
    for n in (2, 3, 8):
        v = (1 << (32 * n - 1)) + 1
        for k in (1, 2, (1 << 32) - 1):
            u = v * k * (1 << 64) - 1
            m = max(n, (u.bit_length() + 31) // 32)
            cases.append((u, v, m, n))
        v = (1 << (32 * n)) - 1
        u = v * ((1 << 64) - 1) + v - 1
        cases.append((u, v, (u.bit_length() + 31) // 32, n))
    for u, v, m, n in cases:
        nv = (v.bit_length() + 31) // 32
        q, r = oracle_lib.bn_divmod(to_limbs(u, m), to_limbs(v, nv))
        assert (from_limbs(q), from_limbs(r)) == divmod(u, v), (u, v)


def _num(q, P):
    limbs, e, s = exact.scalar(q, P)
    return type("N", (), {"limbs": limbs, "exp": np.int64(e), "sign": np.int32(s)})()


def _val(r):
    return exact.value(r.limbs, r.exp, r.sign)


def _random_value(rng, P, emin=-40, emax=40):
    p = 32 * P
    m = rand_int(rng, p) | (1 << (p - 1))
    e = int(rng.integers(emin, emax + 1))
    v = Fraction(m) * Fraction(2) ** (e - p)
    return -v if rng.integers(0, 2) else v


def _adversarial_pairs(rng, P):
    p = 32 * P
    one = Fraction(1)
    pairs = []
    allones = Fraction((1 << p) - 1, 1 << p)  # 0.111...1b
    for gap in list(range(0, 6)) + [p - 2, p - 1, p, p + 1, p + 2, p + 3, 2 * p, 2 * p + 3,
                                    2 * p + 4, 2 * p + 5, 3 * p + 7, 5000]:
        small = Fraction(2) ** (-gap)
        pairs += [(one, small), (one, -small), (allones, small), (allones, -small),
                  (one, small * allones), (one, -small * allones),
                  (Fraction(1, 2), small * (1 + Fraction(1, 1 << (p - 1)))),
                  (-one, small), (-one, -small)]
    pairs += [(one, one), (one, -one), (allones, allones), (Fraction(3, 4), Fraction(3, 4)),
              (one, Fraction(0)), (Fraction(0), one), (Fraction(0), Fraction(0)),
              (Fraction(0), -one)]
    for _ in range(30):
        a = _random_value(rng, P)
        pairs.append((a, a * (1 + Fraction(int(rng.integers(1, 8)), 1 << (32 * P)))))
        pairs.append((a, -a))
    return pairs


@pytest.mark.parametrize("P", [1, 2, 3, 8])
def test_rz_primitives_vs_fraction_and_mpmath(oracle_lib, P):
    rng = np.random.default_rng(10 + P)
    pairs = [(_random_value(rng, P), _random_value(rng, P)) for _ in range(150)]
    pairs += [(_random_value(rng, P, -3, 3), _random_value(rng, P, -3, 3)) for _ in range(150)]
    pairs += _adversarial_pairs(rng, P)
    for a, b in pairs:
        # inputs are representable numbers
        a = exact.truncate(a, P)
        b = exact.truncate(b, P)
        na, nb = _num(a, P), _num(b, P)
        for op, fn, exact_val in (("mul", oracle_lib.mul, a * b), ("add", oracle_lib.add, a + b),
                                  ("sub", oracle_lib.sub, a - b)):
            got = _val(fn(na, nb))
            want = exact.truncate(exact_val, P)
            assert got == want, (op, a, b)
            assert got == exact.mp_op(op, a, b, P), (op, a, b)
        if b != 0:
            got = _val(oracle_lib.div(na, nb))
            want = exact.truncate(a / b, P)
            assert got == want, ("div", a, b)
            assert got == exact.mp_op("div", a, b, P), ("div", a, b)
        else:
            with pytest.raises(ZeroDivisionError):
                oracle_lib.div(na, nb)


def test_results_are_canonical(oracle_lib):
    """Results are normalised (top bit set) or the canonical zero."""
    rng = np.random.default_rng(5)
    P = 4
    for _ in range(200):
        a, b = _random_value(rng, P, -2, 2), _random_value(rng, P, -2, 2)
        for fn in (oracle_lib.mul, oracle_lib.add, oracle_lib.sub, oracle_lib.div):
            r = fn(_num(a, P), _num(b, P))
            if not r.limbs.any():
                assert int(r.exp) == 0 and int(r.sign) == 0
            else:
                assert r.limbs[-1] & 0x80000000
    r = oracle_lib.sub(_num(Fraction(5, 8), P), _num(Fraction(5, 8), P))
    assert not r.limbs.any() and int(r.exp) == 0 and int(r.sign) == 0


@pytest.mark.parametrize("P", [1, 2, 5])
def test_to_f64_is_top_53_bits(oracle_lib, P):
    rng = np.random.default_rng(20 + P)
    vals = [_random_value(rng, P, -1000, 1000) for _ in range(50)] + [Fraction(0), Fraction(-1)]
    for v in vals:
        v = exact.truncate(v, P)
        n = _num(v, P)
        mant, e = oracle_lib.to_f64(n)
        if v == 0:
            assert float(mant) == 0.0 and int(e) == 0
            continue
        frac = abs(v) / Fraction(2) ** int(n.exp)  # in [1/2, 1)
        want = Fraction(int(frac * (1 << 53)), 1 << 53)
        assert Fraction(abs(float(mant))) == want
        assert (float(mant) < 0) == (v < 0)
        assert int(e) == int(n.exp)
