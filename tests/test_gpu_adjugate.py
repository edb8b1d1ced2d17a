"""GPU adjugate (the determinant's backward) against the oracle, bit for bit,
and the autograd wrapper against the oracle's cofactors and multiprecision
central finite differences (det is affine in each entry, so the central
difference with h = 2^-1000 equals C_ij up to rounding)."""
from fractions import Fraction

import numpy as np
import pytest

import exact
import oracle
from gpu_util import assert_same, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def gpu_adj(A_host, path):
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, path)
    adjT = binding.adjugate(A, D, info)
    torch.cuda.synchronize()
    return adjT.to_host(), int(info.item())


@pytest.mark.parametrize("N,P,path", [(1, 2, "valu"), (1, 8, "valu"), (2, 8, "valu"), (2, 8, "mfma"),
                                      (7, 3, "valu"), (20, 8, "mfma"),
                                      (33, 16, "auto"), (48, 64, "mfma")])
def test_adjugate_matches_oracle(N, P, path):
    say(f"[adj] N={N} P={P} {path}")
    A = inputs.random_mantissas((N, N), P, 500 + N + P)
    got, info = gpu_adj(A, path)
    f = oracle.factor(A)
    assert info == f.info == 0
    want = oracle.adjugate_t(f)
    assert_same(got, want, f"adjT N={N} P={P}")
    # column n of adj(A)^T is the minors vector
    c = oracle.minors(f)
    assert np.array_equal(got.limbs[:, -1], c.limbs) and np.array_equal(got.exp[:, -1], c.exp)


def test_adjugate_cauchy_config4_sized():
    say("[adj] cauchy N=40 P=64")
    A, _, _ = inputs.cauchy_dyadic(40, 64, 77)
    got, info = gpu_adj(A, "auto")
    assert_same(got, oracle.adjugate_t(oracle.factor(A)), "adjT cauchy")


def test_adjugate_zero_pivot_gives_zeros():
    A = inputs.from_values([[0, 1], [1, 1]], 8)
    got, info = gpu_adj(A, "auto")
    assert info == 1 and not got.limbs.any()


@pytest.mark.parametrize("N,P,path", [(2, 8, "valu"), (6, 8, "mfma"), (30, 64, "auto"), (12, 264, "mfma")])
def test_adjugate_singular_last_pivot(N, P, path):
    """Only u_nn is zero (info = n): adj(A)^T is still defined (the back
    substitution never divides by u_nn) and must be the oracle's."""
    say(f"[adj] singular last pivot N={N} P={P} {path}")
    A, L, U = inputs.triangular_product(N, P, 60 + N)
    U[N - 1, N - 1] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), P)
    got, info = gpu_adj(A, path)
    f = oracle.factor(A)
    assert info == f.info == N
    assert_same(got, oracle.adjugate_t(f), f"adjT singular N={N}")
    assert got.limbs.any()


def test_autograd_backward_equals_cofactors_and_finite_differences():
    import torch
    from paper_1308_1536_amd import binding
    from paper_1308_1536_amd.autograd import GradHolder, mp_det
    N, P = 12, 64  # 2048 bits, as config 4
    A_host = inputs.random_mantissas((N, N), P, 4242)
    A = binding.DeviceMp.from_host(A_host)
    holder = GradHolder()
    proxy = torch.zeros((N, N), dtype=torch.float64, device="cuda", requires_grad=True)
    mant, e = mp_det(A, proxy, "auto", holder)
    mant.backward()
    torch.cuda.synchronize()
    # exact multiprecision gradient == oracle adjugate, bit for bit
    f = oracle.factor(A_host)
    assert_same(holder.adjT.to_host(), oracle.adjugate_t(f), "autograd adjT")
    # the float64 gradient is adj(A)^T scaled by 2^-e_det
    dm, de = oracle.to_f64(f.D)
    assert float(mant.item()) == float(dm[-1]) and int(e.item()) == int(de[-1])
    am, ae = oracle.to_f64(oracle.adjugate_t(f))
    gm, ge = binding.to_f64(holder.adjT)
    assert np.array_equal(gm.cpu().numpy(), am) and np.array_equal(ge.cpu().numpy(), ae), "to_f64 of adjT"
    want = np.ldexp(am, (ae - de[-1]).astype(np.int64))
    got = proxy.grad.cpu().numpy()
    bad = np.argwhere(got != want)
    assert bad.size == 0, [(tuple(b), got[tuple(b)], want[tuple(b)]) for b in bad[:4]]
    # central finite differences at 4096 bits, h = 2^-1000, on sampled entries
    P2 = 2 * P
    base = inputs.MpArray(np.concatenate([np.zeros_like(A_host.limbs), A_host.limbs], axis=-1),
                          A_host.exp.copy(), A_host.sign.copy())
    h = Fraction(1, 2 ** 1000)
    C = exact.values(oracle.adjugate_t(f))
    rng = np.random.default_rng(1)
    for _ in range(6):
        i, j = (int(v) for v in rng.integers(0, N, size=2))
        dets = []
        for sgn in (1, -1):
            Ap = base.copy()
            aij = exact.value(A_host.limbs[i, j], A_host.exp[i, j], A_host.sign[i, j]) + sgn * h
            l, ee, ss = exact.scalar(aij, P2)
            Ap.limbs[i, j], Ap.exp[i, j], Ap.sign[i, j] = l, ee, ss
            dets.append(exact.values(oracle.factor(Ap).D)[-1])
        fd = (dets[0] - dets[1]) / (2 * h)
        assert exact.bits_agree(fd, C[i, j]) > 900, (i, j)


def test_autograd_zero_pivot_raises_and_singular_last_pivot_differentiates():
    """A zero pivot before the last step makes the forward raise (the method
    cannot give det there); a zero last pivot gives det = 0 exactly and the
    backward still returns adj(A)^T (the oracle's, bit for bit)."""
    import torch
    from paper_1308_1536_amd import binding
    from paper_1308_1536_amd.autograd import GradHolder, ZeroPivotError, mp_det
    say("[adj] autograd zero pivots")
    A = binding.DeviceMp.from_host(inputs.from_values([[0, 1], [1, 1]], 8))
    with pytest.raises(ZeroPivotError) as e:
        mp_det(A)
    assert e.value.info == 1
    N = 7
    A_host, L, U = inputs.triangular_product(N, 8, 5)
    U[N - 1, N - 1] = 0
    A_host = inputs.from_values((L.astype(object) @ U.astype(object)), 8)
    holder = GradHolder()
    proxy = torch.zeros((N, N), dtype=torch.float64, device="cuda", requires_grad=True)
    mant, e = mp_det(binding.DeviceMp.from_host(A_host), proxy, "auto", holder)
    assert float(mant.item()) == 0.0 and int(e.item()) == 0
    mant.backward()
    torch.cuda.synchronize()
    f = oracle.factor(A_host)
    assert f.info == N and int(holder.info.item()) == N
    assert_same(holder.adjT.to_host(), oracle.adjugate_t(f), "autograd adjT singular")
    am, ae = oracle.to_f64(oracle.adjugate_t(f))
    assert np.array_equal(proxy.grad.cpu().numpy(), np.ldexp(am, ae))
