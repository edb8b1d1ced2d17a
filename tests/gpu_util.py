"""Helpers for the GPU tests: run the library through the C-ABI binding and
compare with the oracle bit for bit."""
import sys

import numpy as np


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def assert_same(got, want, what=""):
    """Bit-exact comparison of two host containers (limbs, exp, sign)."""
    gl = np.asarray(got.limbs, dtype=np.uint32)
    wl = np.asarray(want.limbs, dtype=np.uint32)
    assert gl.shape == wl.shape, (what, gl.shape, wl.shape)
    ge, we = np.asarray(got.exp), np.asarray(want.exp)
    gs, ws = np.asarray(got.sign), np.asarray(want.sign)
    bad = ~(np.all(gl == wl, axis=-1) & (ge == we) & (gs == ws))
    if bad.any():
        idx = np.argwhere(bad)
        first = tuple(idx[0])
        raise AssertionError(f"{what}: {len(idx)} of {bad.size} entries differ; first at {first}: "
                             f"gpu exp={ge[first]} sign={gs[first]} top={gl[first][-1]:#x} / "
                             f"oracle exp={we[first]} sign={ws[first]} top={wl[first][-1]:#x}")


def gpu_det(A_host, path="valu", ld=None):
    """Upload, factor + minors through the C-ABI; return host (LU, D, c, info)."""
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.from_host(A_host, ld=ld)
    n = A.rows
    D, info = binding.factor(A, path)
    c = binding.minors(A, D, info) if n > 0 else None
    torch.cuda.synchronize()
    return A.to_host(), D.row(0), (c.row(0) if c is not None else None), int(info.item())
