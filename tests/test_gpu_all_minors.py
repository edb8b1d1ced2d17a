"""GPU last-column minors of every leading block against the oracle (each
block factored afresh on the CPU), bit for bit, and row n against the GPU's
own minors of the whole matrix."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def gpu_all(A_host, path):
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, path)
    C = binding.all_minors(A, D, info)
    c = binding.minors(A, D, info)
    torch.cuda.synchronize()
    return C.to_host(), c.to_host(), int(info.item())


@pytest.mark.parametrize("N,P,path", [(1, 2, "valu"), (1, 8, "valu"), (2, 8, "mfma"), (9, 3, "valu"), (20, 8, "mfma"),
                                      (33, 16, "auto"), (48, 64, "mfma"), (70, 4, "valu")])
def test_all_minors_match_oracle(N, P, path):
    say(f"[all_minors] N={N} P={P} {path}")
    A = inputs.random_mantissas((N, N), P, 900 + N + P)
    got, c, info = gpu_all(A, path)
    assert info == 0
    assert_same(got, oracle.all_minors(A), f"all_minors N={N} P={P}")
    # row N-1 is the minors vector of the whole matrix
    assert np.array_equal(got.limbs[-1], c.limbs[0]) and np.array_equal(got.exp[-1], c.exp[0])
    assert np.array_equal(got.sign[-1], c.sign[0])


def test_all_minors_cauchy():
    say("[all_minors] cauchy N=40 P=64")
    A, _, _ = inputs.cauchy_dyadic(40, 64, 78)
    got, _, info = gpu_all(A, "auto")
    assert info == 0
    assert_same(got, oracle.all_minors(A), "all_minors cauchy")


def test_all_minors_zero_pivot_gives_zeros():
    say("[all_minors] zero pivot")
    A = inputs.from_values([[1, 2, 3], [2, 4, 5], [1, 1, 1]], 8)
    got, _, info = gpu_all(A, "auto")
    assert info == 2 and not got.limbs.any() and not got.exp.any() and not got.sign.any()


@pytest.mark.parametrize("path", ["valu", "mfma"])
def test_all_minors_singular_last_pivot(path):
    """Only u_nn is zero (info = n): every leading block's minors, the whole
    matrix's included, are still the oracle's."""
    say(f"[all_minors] singular last pivot {path}")
    N = 14
    A, L, U = inputs.triangular_product(N, 8, 71)
    U[N - 1, N - 1] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), 8)
    got, c, info = gpu_all(A, path)
    assert info == N
    assert_same(got, oracle.all_minors(A), "all_minors singular")
    assert np.array_equal(got.limbs[-1], c.limbs[0]) and got.limbs[-1].any()


@pytest.mark.parametrize("P", [8, 64])
def test_padded_leading_dimensions(P):
    """Factor, adjugate and all-minors with every matrix at a padded leading
    dimension (the rank-1 kernels step through rows and columns by ld)."""
    import torch
    from paper_1308_1536_amd import binding
    N = 37
    say(f"[all_minors] padded ld N={N} P={P}")
    A_host = inputs.random_mantissas((N, N), P, 4100 + P)
    A = binding.DeviceMp.from_host(A_host, ld=N + 5)
    D, info = binding.factor(A, "valu")
    C = binding.all_minors(A, D, info, binding.DeviceMp.empty(N, N, P, "cuda", ld=N + 3))
    T = binding.adjugate(A, D, info, binding.DeviceMp.empty(N, N, P, "cuda", ld=N + 7))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    f = oracle.factor(A_host)
    assert_same(C.to_host(), oracle.all_minors(A_host), "all_minors padded ld")
    assert_same(T.to_host(), oracle.adjugate_t(f), "adjugate padded ld")


@pytest.mark.parametrize("N,P", [(20, 8), (33, 64)])
def test_normalized_minors_match_oracle(N, P):
    """mp_det_normalize_minors on the minors vector and on every leading
    block's minors, bit for bit against the oracle's divisions."""
    import torch
    from paper_1308_1536_amd import binding
    say(f"[normalize] N={N} P={P}")
    A_host = inputs.random_mantissas((N, N), P, 7000 + N + P)
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, "valu")
    c = binding.minors(A, D, info)
    C = binding.all_minors(A, D, info)
    nc = binding.normalize_minors(c)
    nC = binding.normalize_minors(C)
    torch.cuda.synchronize()
    f = oracle.factor(A_host)
    assert_same(nc.to_host(), oracle.normalize_minors(oracle.minors(f)), "normalised minors")
    assert_same(nC.to_host(), oracle.normalize_minors(oracle.all_minors(A_host)), "normalised all minors")
