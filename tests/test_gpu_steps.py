"""Row panels of the MFMA path's trailing update and factorisations split
into step ranges (mp_det_factor_steps): both must leave the bits of one
mp_det_factor call, which the oracle fixes."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows", [1, 3, 7, 32])
@pytest.mark.parametrize("N,P", [(45, 64), (21, 264)])
def test_mfma_row_panels(rows, N, P):
    """Panels of `rows` rows (not multiples of the two rows a workgroup takes,
    nor of the 32-column blocks) against the oracle."""
    from paper_1308_1536_amd import binding
    A = inputs.random_mantissas((N, N), P, 500 + rows + N)
    say(f"[panels] rows={rows} N={N} P={P}")
    binding.set_panel_rows(rows)
    try:
        LU, D, c, info = gpu_det(A, "mfma")
    finally:
        binding.set_panel_rows(0)
    f, cw = oracle.det_pipeline(A)
    assert info == f.info
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


def _split_run(A_host, path, cuts):
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(A_host)
    n = A.rows
    D = binding.DeviceMp.empty(1, n, A.P)
    info = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    edges = [0] + list(cuts) + [n]
    for a, b in zip(edges[:-1], edges[1:]):
        binding.factor_steps(A, D, info, a, b, path)
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), int(info.item())


@pytest.mark.parametrize("path,P", [("valu", 32), ("valu", 130), ("mfma", 64), ("mfma", 264)])
def test_factor_steps_split(path, P):
    """Ranges [0, 5), [5, 6), [6, 23), [23, n) give the one-call bits."""
    N = 37 if P < 200 else 19
    A = inputs.random_mantissas((N, N), P, 600 + P)
    say(f"[steps] path={path} N={N} P={P}")
    LU, D, info = _split_run(A, path, [5, 6, min(23, N - 1)])
    f, _ = oracle.det_pipeline(A)
    assert info == f.info
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")


@pytest.mark.parametrize("path", ["valu", "mfma"])
def test_factor_steps_zero_pivot(path):
    """A zero pivot inside the first range stops the later ranges too."""
    A, L, U = inputs.triangular_product(14, 16, 9)
    U[4, 4] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), 16)
    say(f"[steps] zero pivot path={path}")
    LU, D, info = _split_run(A, path, [7, 10])
    f, _ = oracle.det_pipeline(A)
    assert info == f.info and info != 0
    assert_same(D, f.D, "D")


def test_factor_steps_rejects_bad_ranges():
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(inputs.random_mantissas((6, 6), 8, 5))
    D = binding.DeviceMp.empty(1, 6, 8)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    for a, b in ((-1, 3), (4, 3), (0, 7)):
        with pytest.raises(binding.MpdetError) as e:
            binding.factor_steps(A, D, info, a, b, "valu")
        assert e.value.status == binding.MPDET_EINVAL


@pytest.mark.parametrize("N,P", [(70, 264), (45, 520), (40, 1024)])
def test_mfma_finish_in_update_launch(N, P):
    """Above 256 limbs each wave of the update launch finishes its own 32
    products (the default); overlap setting 1 keeps the finish a launch of its
    own.  Both give the oracle's bits (several 32-column blocks, a ragged one)."""
    from paper_1308_1536_amd import binding
    A = inputs.random_mantissas((N, N), P, 900 + N)
    f, cw = oracle.det_pipeline(A)
    for setting in (0, 1):
        say(f"[finish] overlap setting {setting} N={N} P={P}")
        binding.set_overlap(setting)
        try:
            LU, D, c, info = gpu_det(A, "mfma")
        finally:
            binding.set_overlap(0)
        assert info == f.info
        assert_same(D, f.D, "D")
        assert_same(LU, f.LU, "LU")
        assert_same(c, cw, "c")


@pytest.mark.parametrize("panels", [2, 3, 5])
@pytest.mark.parametrize("N,P", [(45, 64), (21, 264), (24, 1024)])
def test_mfma_overlapped_panels(panels, N, P):
    """The finish of each row panel on a second stream beside the next panel's
    update, two record buffers alternating: the oracle's bits."""
    from paper_1308_1536_amd import binding
    A = inputs.random_mantissas((N, N), P, 700 + panels + N)
    say(f"[overlap] panels={panels} N={N} P={P}")
    binding.set_overlap(panels)
    try:
        LU, D, c, info = gpu_det(A, "mfma")
    finally:
        binding.set_overlap(0)
    f, cw = oracle.det_pipeline(A)
    assert info == f.info
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")
