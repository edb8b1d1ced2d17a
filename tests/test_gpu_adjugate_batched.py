"""The determinant's backward for a batch in one persistent launch
(mp_det_adjugate_batched): bit-identical to one mp_det_adjugate call per
matrix and to the oracle, on the lane product (rank-1 updates) and on the
one-wave kernels; incomplete factors give zeros and their info as status; an
expired wait drains the launch; the batched autograd Function returns every
matrix's gradient."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def _batch(sizes, P, seed):
    hosts = []
    for b, n in enumerate(sizes):
        if b % 2:
            hosts.append(inputs.cauchy_dyadic(n, P, seed + b)[0])
        else:
            hosts.append(inputs.random_mantissas((n, n), P, seed + b))
    return hosts


def _factored(hosts):
    import torch
    from paper_1308_1536_amd import binding
    mats = [binding.DeviceMp.from_host(h) for h in hosts]
    Ds, _, info = binding.batched(mats, "valu", minors=False)
    torch.cuda.synchronize()
    return mats, Ds, info


@pytest.mark.parametrize("P", [64, 16, 6])
def test_batched_backward_matches_per_matrix_and_oracle(P):
    import torch
    from paper_1308_1536_amd import binding
    sizes = [1, 2, 17, 40, 5, 33, 3, 64]
    hosts = _batch(sizes, P, 5200 + P)
    mats, Ds, info = _factored(hosts)
    say(f"[adj batched] P={P} sizes={sizes}")
    got, status = binding.adjugate_batched(mats, Ds, info)
    want, status2 = binding.adjugate_batched(mats, Ds, info, schedule="lockstep")
    torch.cuda.synchronize()
    assert not status.cpu().numpy().any() and not status2.cpu().numpy().any()
    for b in range(len(sizes)):
        assert_same(got[b].to_host(), want[b].to_host(), f"adjT[{b}] persistent vs per matrix")
    for b in (2, 3, 7):
        f = oracle.factor(hosts[b])
        assert_same(got[b].to_host(), oracle.adjugate_t(f), f"adjT[{b}] vs oracle")


def test_batched_backward_incomplete_factors_and_last_pivot_zero():
    import torch
    from paper_1308_1536_amd import binding
    P = 8
    zero_first = inputs.from_values([[0, 1, 2], [1, 1, 0], [3, 1, 1]], P)   # info = 1
    N = 6
    A_sing, L, U = inputs.triangular_product(N, P, 9)
    U[N - 1, N - 1] = 0
    A_sing = inputs.from_values((L.astype(object) @ U.astype(object)), P)  # info = n
    good = inputs.random_mantissas((9, 9), P, 11)
    hosts = [zero_first, A_sing, good]
    mats, Ds, info = _factored(hosts)
    assert info.cpu().tolist() == [1, N, 0]
    say("[adj batched] zero pivots")
    got, status = binding.adjugate_batched(mats, Ds, info)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [1, 0, 0]
    assert not got[0].to_host().limbs.any()
    for b in (1, 2):
        assert_same(got[b].to_host(), oracle.adjugate_t(oracle.factor(hosts[b])), f"adjT[{b}]")


def test_batched_backward_expired_wait_drains():
    import torch
    from paper_1308_1536_amd import binding
    hosts = _batch([60, 45, 30], 16, 5300)
    mats, Ds, info = _factored(hosts)
    say("[adj batched] wait limit 0")
    binding.set_wait_limit(0.0)
    try:
        got, status = binding.adjugate_batched(mats, Ds, info)
        torch.cuda.synchronize()
    finally:
        binding.set_wait_limit(10.0)
    st = status.cpu().numpy()
    assert set(st.tolist()) <= {0, -2} and (st == -2).any()
    got, status = binding.adjugate_batched(mats, Ds, info)
    torch.cuda.synchronize()
    assert not status.cpu().numpy().any()
    assert_same(got[0].to_host(), oracle.adjugate_t(oracle.factor(hosts[0])), "after the limit is restored")


def test_batched_autograd_gradients():
    """MpDetBatch: forward on the batch, backward in one launch; every proxy
    gets the same gradient as the single-matrix Function's."""
    import torch
    from paper_1308_1536_amd import binding
    from paper_1308_1536_amd.autograd import GradHolder, mp_det, mp_det_batch
    P = 64
    hosts = _batch([12, 5, 20, 1], P, 5400)
    mats = [binding.DeviceMp.from_host(h) for h in hosts]
    holders = [GradHolder() for _ in hosts]
    proxies = [torch.zeros((m.rows, m.rows), dtype=torch.float64, device="cuda", requires_grad=True) for m in mats]
    say("[adj batched] autograd")
    mant, e = mp_det_batch(mats, proxies, holders=holders)
    mant.sum().backward()
    torch.cuda.synchronize()
    for b, (A, h) in enumerate(zip(mats, hosts)):
        p1 = torch.zeros((A.rows, A.rows), dtype=torch.float64, device="cuda", requires_grad=True)
        m1, e1 = mp_det(binding.DeviceMp.from_host(h), p1)
        m1.backward()
        assert float(m1.item()) == float(mant[b].item()) and int(e1.item()) == int(e[b].item())
        assert torch.equal(p1.grad, proxies[b].grad), f"gradient {b}"
        assert_same(holders[b].adjT.to_host(), oracle.adjugate_t(oracle.factor(h)), f"holder adjT {b}")
