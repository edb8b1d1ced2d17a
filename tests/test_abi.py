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


def test_header_declares_the_entry_points():
    names = binding.header_functions()
    for fn in ("mpdet_create", "mpdet_destroy", "mpdet_strerror", "mp_det_factor",
               "mp_det_minors", "mp_to_f64"):
        assert fn in names


def test_library_exports_every_declared_symbol(lib):
    for fn in binding.header_functions():
        assert hasattr(lib, fn), fn


def test_strerror(lib):
    assert binding.strerror(0) == "ok"
    assert binding.strerror(binding.MPDET_EINVAL) == "invalid argument"
    assert binding.strerror(binding.MPDET_ENOTSUP) == "not supported"
    assert binding.strerror(12345) == "unknown status"


def test_null_handle_and_bad_args_rejected_on_host(lib):
    m = binding.MpdetMat(None, None, None, 4, 4, 4, 8)
    assert lib.mp_det_factor(None, m, m, None, 0, None) == binding.MPDET_EINVAL
    assert lib.mp_det_minors(None, m, m, m, None, None) == binding.MPDET_EINVAL
    assert lib.mp_to_f64(None, m, None, None, None) == binding.MPDET_EINVAL
    assert lib.mpdet_create(None, 0) == binding.MPDET_EINVAL
    assert lib.mpdet_destroy(None) == binding.MPDET_EINVAL


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
