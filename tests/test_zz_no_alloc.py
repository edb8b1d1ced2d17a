"""mp_det_factor_noalloc (the factorisation on the library's static
per-device scratch, for callers that cannot allocate) against mp_det_factor
on the same inputs, bit for bit, on two calls in a row with the second one
smaller, for each path: the VALU lane product, the one-wave VALU update, and
the MFMA path (at 1024 limbs its update runs over several row panels sized
to the scratch).  Sizes beyond the scratch are refused before any launch."""
import pytest

from gpu_util import assert_same, say
from paper_1308_1536_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _handle_path(A_host, path):
    import torch
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, path)
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), int(info.item())


def _noalloc_path(A_host, path):
    import torch
    A = binding.DeviceMp.from_host(A_host)
    D = binding.DeviceMp.empty(1, A.rows, A.P)
    info = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    binding.factor_noalloc(A, D, info, path)
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), int(info.item())


@pytest.mark.parametrize("path,P,sizes", [("valu", 64, (40, 23)), ("valu", 6, (20, 11)),
                                          ("mfma", 16, (41, 19)), ("mfma", 1024, (200, 70))])
def test_noalloc_matches_factor_twice(path, P, sizes):
    for t, n in enumerate(sizes):
        A = inputs.random_mantissas((n, n), P, 7100 + 10 * P + t)
        say(f"[noalloc] path={path} P={P} n={n} call {t + 1}")
        LU0, D0, info0 = _handle_path(A, path)
        LU1, D1, info1 = _noalloc_path(A, path)
        assert info1 == info0 == 0
        assert_same(D1, D0, "D")
        assert_same(LU1, LU0, "LU")


def test_noalloc_refuses_oversize_before_launch():
    import torch
    n, P = 400, 128  # lane-product records of 399 x 416 numbers: 87 MB > 64 MiB
    A = binding.DeviceMp.empty(n, n, P)
    D = binding.DeviceMp.empty(1, n, P)
    info = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    say(f"[noalloc] oversize n={n} P={P}")
    with pytest.raises(binding.MpdetError) as e:
        binding.factor_noalloc(A, D, info, "valu")
    assert e.value.status == binding.MPDET_ERANGE
    torch.cuda.synchronize()
    assert int(info.item()) == 77  # nothing was launched
