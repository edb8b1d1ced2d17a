"""The C-ABI boundary on the CPU: the library loads, exports every function
include/mpdet.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os

import pytest

from paper_1308_1536_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmpdet.so is not built (run __graft_entry__.build())")
    return binding.lib()


# the boundary's calls: handle life cycle, workspace query, factorisation,
# minors, the batch, the gradient, output conversion, status names
BOUNDARY = ("mpdet_create", "mpdet_destroy", "mpdet_workspace_size", "mp_det_factor", "mp_det_minors",
            "mp_det_batched", "mp_det_adjugate", "mp_to_f64", "mpdet_strerror")


def test_header_declares_the_entry_points():
    names = binding.header_functions()
    for fn in BOUNDARY + ("mp_det_factor_steps", "mp_det_all_minors", "mp_det_normalize_minors",
                          "mp_to_f64_scaled", "mp_det_factor_noalloc"):
        assert fn in names, fn


def test_library_exports_every_declared_symbol(lib):
    for fn in binding.header_functions():
        assert hasattr(lib, fn), fn


def test_strerror(lib):
    assert binding.strerror(0) == "ok"
    assert binding.strerror(binding.MPDET_EINVAL) == "invalid argument"
    assert binding.strerror(binding.MPDET_ENOTSUP) == "not supported"
    assert binding.strerror(12345) == "unknown status"
    assert "scratch" in binding.strerror(binding.MPDET_ERANGE)


def test_workspace_size_on_host(lib):
    """mpdet_workspace_size needs no GPU (NULL handle: default panels) and
    follows the layout the header states."""
    ws = binding.workspace_size
    assert ws(0, 8, "valu") == 0
    assert ws(1, 8, "valu") == ws(1, 8, "mfma") == 256      # the reciprocal only
    assert ws(100, 6, "valu") == 256                         # one-wave update: no records
    # lane product (P <= 128, P % 4 == 0): records of the whole trailing block
    rec = lambda rows, m, P: (rows * ((m + 31) // 32) * 32 * (P + 4) + (P + 40) * 32) * 4
    up = lambda x: (x + 255) // 256 * 256
    assert ws(64, 32, "valu") == 256 + up(rec(63, 63, 32))
    # MFMA adds the digit strings; the records stay one panel up to 24 GiB
    assert ws(512, 128, "mfma") > ws(512, 128, "valu")
    assert ws(2048, 1024, "mfma") >= rec(2047, 2047, 1024)
    big = ws(6144, 1024, "mfma")  # 155 GB matrix: panels keep the records under 24 GiB
    assert rec(6143, 6143, 1024) > 24 << 30 > big - 6143 * 2 * (4 * 1024 + 608)
    sizes = [ws(n, 64, "valu") for n in range(0, 200, 7)]
    assert sizes == sorted(sizes)
    out = ctypes.c_size_t()
    assert lib.mpdet_workspace_size(None, -1, 8, 0, ctypes.byref(out)) == binding.MPDET_EINVAL
    assert lib.mpdet_workspace_size(None, 8, 1, 0, ctypes.byref(out)) == binding.MPDET_EINVAL
    assert lib.mpdet_workspace_size(None, 8, 12, 2, ctypes.byref(out)) == binding.MPDET_ENOTSUP
    assert lib.mpdet_workspace_size(None, 8, 8, 0, None) == binding.MPDET_EINVAL


def test_null_handle_and_bad_args_rejected_on_host(lib):
    m = binding.MpdetMat(None, None, None, 4, 4, 4, 8)
    assert lib.mp_det_factor(None, m, m, None, 0, None) == binding.MPDET_EINVAL
    assert lib.mp_det_minors(None, m, m, m, None, None) == binding.MPDET_EINVAL
    assert lib.mp_to_f64(None, m, None, None, None) == binding.MPDET_EINVAL
    assert lib.mpdet_create(None, 0) == binding.MPDET_EINVAL
    assert lib.mp_det_factor_noalloc(m, m, None, 0, None) == binding.MPDET_EINVAL  # no info
    bad = binding.MpdetMat(None, None, None, 4, 5, 5, 8)  # not square
    assert lib.mp_det_factor_noalloc(bad, m, 8, 0, None) == binding.MPDET_EINVAL
    assert lib.mpdet_destroy(None) == binding.MPDET_EINVAL
    assert lib.mpdet_set_long_division(None, 1) == binding.MPDET_EINVAL
    assert lib.mpdet_set_wait_limit(None, 1.0) == binding.MPDET_EINVAL


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = lib.mpdet_create(ctypes.byref(h), 0)
    assert rc in (binding.MPDET_EHIP, binding.MPDET_EINVAL)


def test_product_path_has_no_oracle_dependency():
    """The package never imports, loads or names the oracle."""
    pkg = os.path.join(ROOT, "paper_1308_1536_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "mpref" not in text, f


def test_normalize_minors_rejects_any_overlap_on_host(lib):
    """mp_det_normalize_minors refuses an output sharing any byte with its
    input (not only the same start), before it touches a device."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the host-side rejection without a device")
    fake = ctypes.create_string_buffer(4096)  # never dereferenced before the checks
    h = ctypes.cast(fake, ctypes.c_void_p)
    rows, cols, P = 3, 4, 2
    base = 1 << 32  # addresses only compared, never read
    limbs, exps, signs = base, base + (1 << 20), base + (2 << 20)
    C = binding.MpdetMat(limbs, exps, signs, rows, cols, cols, P)
    for shift in (4, 8 * P * 4, (rows * cols - 1) * P * 4):  # partial overlaps of the limbs
        out = binding.MpdetMat(limbs + shift, base + (3 << 20), base + (4 << 20), rows, cols, cols, P)
        assert lib.mp_det_normalize_minors(h, C, out, None) == binding.MPDET_EINVAL, shift
    out = binding.MpdetMat(base + (3 << 20), exps + 8, base + (4 << 20), rows, cols, cols, P)
    assert lib.mp_det_normalize_minors(h, C, out, None) == binding.MPDET_EINVAL
    out = binding.MpdetMat(base + (3 << 20), base + (4 << 20), limbs, rows, cols, cols, P)  # signs over limbs
    assert lib.mp_det_normalize_minors(h, C, out, None) == binding.MPDET_EINVAL
    # disjoint: passes the checks and fails only at the device (none here)
    out = binding.MpdetMat(base + (3 << 20), base + (4 << 20), base + (5 << 20), rows, cols, cols, P)
    assert lib.mp_det_normalize_minors(h, C, out, None) == binding.MPDET_EHIP
