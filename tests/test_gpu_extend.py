"""Growing a factorisation (mp_det_extend): factor the leading block, add the
remaining rows and columns later, and the result -- every entry of the
factored matrix, every D_k, the minors -- equals one factorisation of the
whole matrix bit for bit (and the oracle's), on the lane product, the
one-wave update and the MFMA path, including a chain N_b, 2 N_b, 3 N_b."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def _grown(A_host, cuts, path):
    """Factor the leading cuts[0] block, then extend to cuts[1], ..., n."""
    import torch
    from paper_1308_1536_amd import binding
    n = A_host.exp.shape[0]
    A = binding.DeviceMp.from_host(A_host)
    D = binding.DeviceMp.empty(1, n, A.P)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    first = cuts[0]
    # the leading block alone, factored in a buffer of its own, copied back
    B = binding.DeviceMp.from_host(inputs.MpArray(A_host.limbs[:first, :first].copy(),
                                                  A_host.exp[:first, :first].copy(),
                                                  A_host.sign[:first, :first].copy()))
    DB, infoB = binding.factor(B, path)
    A.limbs[:first, :first].copy_(B.limbs)
    A.exp[:first, :first].copy_(B.exp)
    A.sign[:first, :first].copy_(B.sign)
    D.limbs[:, :first].copy_(DB.limbs)
    D.exp[:, :first].copy_(DB.exp)
    D.sign[:, :first].copy_(DB.sign)
    info.copy_(infoB)
    prev = first
    for nxt in list(cuts[1:]) + [n]:
        # the matrix grown so far is the leading nxt block of A
        Anow = binding.DeviceMp(A.limbs[:nxt, :nxt], A.exp[:nxt, :nxt], A.sign[:nxt, :nxt], nxt, nxt)
        sub = binding.DeviceMp(Anow.limbs.contiguous(), Anow.exp.contiguous(), Anow.sign.contiguous(), nxt, nxt)
        binding.extend(sub, D, info, prev, path)
        A.limbs[:nxt, :nxt].copy_(sub.limbs)
        A.exp[:nxt, :nxt].copy_(sub.exp)
        A.sign[:nxt, :nxt].copy_(sub.sign)
        prev = nxt
    c = binding.minors(A, D, info)
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), c.row(0), int(info.item())


@pytest.mark.parametrize("path,P,n,cuts", [("valu", 64, 40, [24]), ("valu", 6, 23, [9]), ("mfma", 16, 37, [20]),
                                           ("valu", 8, 33, [11, 22]), ("mfma", 8, 30, [0]),
                                           ("auto", 128, 27, [26])])
def test_extend_matches_one_factorisation(path, P, n, cuts):
    A = inputs.random_mantissas((n, n), P, 8800 + n + P)
    say(f"[extend] path={path} P={P} n={n} cuts={cuts}")
    LU, D, c, info = _grown(A, cuts, path)
    LU1, D1, c1, info1 = gpu_det(A, path)
    assert info == info1 == 0
    assert_same(D, D1, "D")
    assert_same(LU, LU1, "LU")
    assert_same(c, c1, "c")
    f, cw = oracle.det_pipeline(A)
    assert_same(D, f.D, "oracle D")
    assert_same(c, cw, "oracle c")


def test_extend_cauchy_doubling():
    """N_b, 2 N_b, 3 N_b on a Cauchy matrix at 2048 bits."""
    A, _, _ = inputs.cauchy_dyadic(48, 64, 91)
    say("[extend] cauchy 16 -> 32 -> 48")
    LU, D, c, info = _grown(A, [16, 32], "valu")
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")
