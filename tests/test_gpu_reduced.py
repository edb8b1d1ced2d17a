"""Reduced precision in the later steps (mp_det_factor_reduced): the first
k_switch steps at the full precision, the state truncated (mp_truncate), the
rest at the shorter one -- bit for bit the oracle's composition of the same
pieces, on the lane product, the one-wave update and the MFMA path."""
import pytest

import oracle
from gpu_util import assert_same, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,P,P2,k,path,path2", [(30, 64, 32, 10, "valu", "valu"), (25, 8, 4, 0, "valu", "valu"),
                                                 (25, 8, 4, 25, "valu", "valu"), (19, 6, 3, 7, "valu", "valu"),
                                                 (20, 1024, 512, 7, "mfma", "mfma"),
                                                 (24, 128, 64, 12, "mfma", "valu")])
def test_reduced_matches_oracle(n, P, P2, k, path, path2):
    import torch
    from paper_1308_1536_amd import binding
    A_host = inputs.random_mantissas((n, n), P, 7700 + n + k)
    say(f"[reduced] n={n} P={P}->{P2} at k={k} {path}/{path2}")
    A = binding.DeviceMp.from_host(A_host)
    A2, D2, Dlead, info = binding.factor_reduced(A, k, P2, path, path2)
    c = binding.minors(A2, D2, info)
    torch.cuda.synchronize()
    f, cw, lead = oracle.det_pipeline_reduced(A_host, k, P2)
    assert int(info.item()) == f.info == 0
    assert_same(D2.row(0), f.D, "D at P2")
    assert_same(A2.to_host(), f.LU, "factors at P2")
    assert_same(c.row(0), cw, "minors at P2")
    if k:
        got = Dlead.row(0)
        from paper_1308_1536_amd.binding import HostMp
        assert_same(HostMp(got.limbs[:k], got.exp[:k], got.sign[:k]),
                    HostMp(lead.limbs[:k], lead.exp[:k], lead.sign[:k]), "leading D at P")


def test_truncate_matches_oracle():
    from paper_1308_1536_amd import binding
    x = inputs.random_mantissas((7, 9), 12, 3)
    for P2 in (2, 5, 12):
        y = binding.truncate(binding.DeviceMp.from_host(x), P2)
        assert_same(y.to_host(), oracle.truncate(x, P2), f"P2={P2}")
    with pytest.raises(binding.MpdetError) as e:  # the format needs at least 2 limbs
        binding.truncate(binding.DeviceMp.from_host(x), 1)
    assert e.value.status == binding.MPDET_EINVAL
