"""Thin ctypes binding over libmpdet.so (C-ABI in include/mpdet.h).

Argument marshalling only: every arithmetic step runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  The
library is loaded from this package directory; if it has not been built the
first call raises (there is no CPU fallback).

Device layout of a multiprecision array (``DeviceMp``): limbs int32 tensor
[rows, ld, P] holding the uint32 limb bit patterns, exp int64 [rows, ld],
sign int32 [rows, ld]; value = (-1)^sign * m * 2^(exp - 32P).
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpdet.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpdet.h")

MPDET_OK, MPDET_EINVAL, MPDET_ENOMEM, MPDET_EHIP, MPDET_ENOTSUP, MPDET_ERANGE = 0, -1, -2, -3, -4, -5
NOALLOC_SCRATCH_BYTES = 64 << 20  # MPDET_NOALLOC_SCRATCH_BYTES
PATH_AUTO, PATH_VALU, PATH_MFMA = 0, 1, 2
PATHS = {"auto": PATH_AUTO, "valu": PATH_VALU, "mfma": PATH_MFMA}


class MpdetMat(ctypes.Structure):
    _fields_ = [("limbs", ctypes.c_void_p), ("exp", ctypes.c_void_p), ("sign", ctypes.c_void_p),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("nlimbs", ctypes.c_int32)]


class MpdetError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status} ({strerror(status)})")
        self.status = status


_lib = None


def header_functions() -> list[str]:
    """Names of the functions include/mpdet.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)


def lib() -> ctypes.CDLL:
    """Load libmpdet.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1308_1536_amd.build` (no CPU fallback exists)")
        # torch's own HIP runtime (it ships one) must be loaded before the
        # library: the library then binds to that runtime instead of loading
        # the system's, and torch and the library share devices, streams and
        # memory (two runtimes in one process leave one of them without a device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.mpdet_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.mpdet_destroy.argtypes = [vp]
        L.mpdet_strerror.argtypes = [ctypes.c_int]
        L.mpdet_strerror.restype = ctypes.c_char_p
        L.mp_det_factor.argtypes = [vp, MpdetMat, MpdetMat, vp, ctypes.c_int, vp]
        L.mp_det_factor_steps.argtypes = [vp, MpdetMat, MpdetMat, vp, i64, i64, ctypes.c_int, vp]
        L.mpdet_set_panel_rows.argtypes = [vp, i64]
        L.mp_det_factor_ball.argtypes = [vp, MpdetMat, MpdetMat, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
        L.mp_det_factor_ball.restype = ctypes.c_int
        L.mp_truncate.argtypes = [vp, MpdetMat, MpdetMat, vp]
        L.mp_truncate.restype = ctypes.c_int
        L.mp_det_factor_reduced.argtypes = [vp, MpdetMat, MpdetMat, MpdetMat, MpdetMat, vp, i64, ctypes.c_int,
                                            ctypes.c_int, vp]
        L.mp_det_factor_reduced.restype = ctypes.c_int
        L.mpdet_set_overlap.argtypes = [vp, i32]
        L.mpdet_set_overlap.restype = ctypes.c_int
        L.mpdet_set_tuning.argtypes = [vp, i32, i32]
        L.mpdet_set_tuning.restype = ctypes.c_int
        L.mp_det_extend.argtypes = [vp, MpdetMat, MpdetMat, vp, i64, ctypes.c_int, vp]
        L.mp_det_extend.restype = ctypes.c_int
        L.mp_det_factor_noalloc.argtypes = [MpdetMat, MpdetMat, vp, ctypes.c_int, vp]
        L.mp_det_factor_noalloc.restype = ctypes.c_int
        L.mpdet_workspace_size.argtypes = [vp, i64, i32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.mpdet_workspace_size.restype = ctypes.c_int
        L.mp_det_minors.argtypes = [vp, MpdetMat, MpdetMat, MpdetMat, vp, vp]
        L.mp_to_f64.argtypes = [vp, MpdetMat, vp, vp, vp]
        L.mpdet_profile_begin.argtypes = [vp]
        L.mpdet_profile_end.argtypes = [vp]
        L.mpdet_profile_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
        for name in ("mpdet_create", "mpdet_destroy", "mp_det_factor", "mp_det_minors", "mp_to_f64",
                     "mpdet_profile_begin", "mpdet_profile_end", "mpdet_profile_get"):
            getattr(L, name).restype = ctypes.c_int
        L.mp_det_batched.argtypes = [vp, i64, ctypes.POINTER(MpdetMat), ctypes.POINTER(MpdetMat),
                                     ctypes.POINTER(MpdetMat), vp, ctypes.c_int, ctypes.c_int, vp]
        L.mp_det_batched.restype = ctypes.c_int
        L.mpdet_set_wait_limit.argtypes = [vp, ctypes.c_double]
        L.mpdet_set_long_division.argtypes = [vp, i32]
        L.mpdet_set_wait_limit.restype = ctypes.c_int
        L.mpdet_batched_plan.argtypes = [i64, ctypes.POINTER(ctypes.c_int64), i32, ctypes.c_int, ctypes.c_int, vp, i64,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.mpdet_batched_plan.restype = ctypes.c_int
        L.mp_det_adjugate.argtypes = [vp, MpdetMat, MpdetMat, MpdetMat, vp, vp]
        L.mp_det_adjugate.restype = ctypes.c_int
        L.mp_det_adjugate_batched.argtypes = [vp, i64, ctypes.POINTER(MpdetMat), ctypes.POINTER(MpdetMat),
                                              ctypes.POINTER(MpdetMat), vp, vp, ctypes.c_int, vp]
        L.mp_det_adjugate_batched.restype = ctypes.c_int
        L.mp_det_all_minors.argtypes = [vp, MpdetMat, MpdetMat, MpdetMat, vp, vp]
        L.mp_det_all_minors.restype = ctypes.c_int
        L.mp_det_normalize_minors.argtypes = [vp, MpdetMat, MpdetMat, vp]
        L.mp_det_normalize_minors.restype = ctypes.c_int
        L.mp_to_f64_scaled.argtypes = [vp, MpdetMat, vp, vp, vp]
        L.mp_to_f64_scaled.restype = ctypes.c_int
        L.mpdet_measure_peak.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.mpdet_measure_peak.restype = ctypes.c_int
        _ = (i32,)
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().mpdet_strerror(int(status)).decode()


def _check(fn: str, rc: int):
    if rc != MPDET_OK:
        raise MpdetError(fn, rc)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Handle:
    """Owns an mpdet_handle bound to one device."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        _check("mpdet_create", lib().mpdet_create(ctypes.byref(h), self.device))
        self.ptr = h

    def close(self):
        if self.ptr:
            lib().mpdet_destroy(self.ptr)
            self.ptr = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order varies
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


@dataclass
class DeviceMp:
    """Multiprecision array in device memory (see module docstring)."""
    limbs: "object"  # torch.int32 [rows, ld, P]
    exp: "object"    # torch.int64 [rows, ld]
    sign: "object"   # torch.int32 [rows, ld]
    rows: int
    cols: int

    @property
    def P(self) -> int:
        return int(self.limbs.shape[-1])

    @property
    def ld(self) -> int:
        return int(self.limbs.shape[1])

    def mat(self) -> MpdetMat:
        return MpdetMat(self.limbs.data_ptr(), self.exp.data_ptr(), self.sign.data_ptr(),
                        self.rows, self.cols, self.ld, self.P)

    @staticmethod
    def empty(rows: int, cols: int, P: int, device="cuda", ld: int | None = None) -> "DeviceMp":
        import torch
        ld = cols if ld is None else ld
        return DeviceMp(torch.zeros((rows, ld, P), dtype=torch.int32, device=device),
                        torch.zeros((rows, ld), dtype=torch.int64, device=device),
                        torch.zeros((rows, ld), dtype=torch.int32, device=device), rows, cols)

    @staticmethod
    def from_host(x, device="cuda", ld: int | None = None) -> "DeviceMp":
        """Upload any host container with .limbs [..., P] uint32, .exp, .sign.
        A 1-D container becomes a 1 x n row vector."""
        import torch
        limbs = np.ascontiguousarray(x.limbs, dtype=np.uint32)
        exp = np.ascontiguousarray(x.exp, dtype=np.int64)
        sign = np.ascontiguousarray(x.sign, dtype=np.int32)
        if exp.ndim == 1:
            limbs, exp, sign = limbs[None], exp[None], sign[None]
        rows, cols = exp.shape
        P = limbs.shape[-1]
        out = DeviceMp.empty(rows, cols, P, device, ld)
        out.limbs[:, :cols].copy_(torch.from_numpy(limbs.view(np.int32)))
        out.exp[:, :cols].copy_(torch.from_numpy(exp))
        out.sign[:, :cols].copy_(torch.from_numpy(sign))
        return out

    def to_host(self):
        """(limbs uint32 [rows, cols, P], exp int64 [rows, cols], sign int32 [rows, cols])."""
        limbs = self.limbs[:, :self.cols].cpu().numpy().view(np.uint32)
        return HostMp(limbs, self.exp[:, :self.cols].cpu().numpy(),
                      self.sign[:, :self.cols].cpu().numpy())

    def row(self, i: int = 0):
        """Host copy of one row as a 1-D container (vectors: row 0)."""
        h = self.to_host()
        return HostMp(h.limbs[i], h.exp[i], h.sign[i])


@dataclass
class HostMp:
    limbs: np.ndarray
    exp: np.ndarray
    sign: np.ndarray

    @property
    def P(self) -> int:
        return int(self.limbs.shape[-1])


def _resolve(path: str, n: int, P: int) -> int:
    """Path name -> MPDET_PATH_*; "tuned" asks the autotuner (measured, cached)."""
    if path == "tuned":
        from . import autotune
        path = autotune.choose_path(n, P)
    if path not in PATHS:
        raise ValueError(f"unknown path {path!r}: one of {sorted(PATHS) + ['tuned']}")
    return PATHS[path]


def factor(A: DeviceMp, path: str = "auto", D: DeviceMp | None = None, info=None, stream=None):
    """mp_det_factor in place on A.  Returns (D, info) device tensors.
    path: "auto" (MFMA where the limb count allows and is above 64), "valu",
    "mfma" or "tuned"."""
    import torch
    n = A.rows
    if D is None:
        D = DeviceMp.empty(1, n, A.P, A.limbs.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.limbs.device)
    h = handle(A.limbs.device.index or 0)
    _check("mp_det_factor", lib().mp_det_factor(h.ptr, A.mat(), D.mat(), info.data_ptr(),
                                                _resolve(path, n, A.P), _stream(stream)))
    return D, info


def factor_steps(A: DeviceMp, D: DeviceMp, info, k_begin: int, k_end: int, path: str = "auto", stream=None):
    """mp_det_factor_steps: elimination steps k_begin .. k_end-1 in place (D, info
    carried between calls; k_begin == 0 resets info)."""
    h = handle(A.limbs.device.index or 0)
    _check("mp_det_factor_steps", lib().mp_det_factor_steps(h.ptr, A.mat(), D.mat(), info.data_ptr(), int(k_begin),
                                                            int(k_end), _resolve(path, A.rows, A.P),
                                                            _stream(stream)))
    return D, info


def factor_noalloc(A: DeviceMp, D: DeviceMp, info, path: str = "auto", stream=None):
    """mp_det_factor_noalloc: mp_det_factor in place on A with the library's
    static per-device scratch (no device allocation; the caller passes D and
    info).  Runs on A's device."""
    import torch
    with torch.cuda.device(A.limbs.device):
        _check("mp_det_factor_noalloc", lib().mp_det_factor_noalloc(A.mat(), D.mat(), info.data_ptr(),
                                                                    _resolve(path, A.rows, A.P), _stream(stream)))
    return D, info


def workspace_size(n: int, P: int, path: str = "auto", device: int | None = None) -> int:
    """mpdet_workspace_size: device bytes mp_det_factor takes from the handle
    for an n x n matrix of P-limb numbers (device None: the default panel
    setting, no handle and no GPU needed)."""
    out = ctypes.c_size_t()
    h = handle(device).ptr if device is not None else None
    _check("mpdet_workspace_size", lib().mpdet_workspace_size(h, int(n), int(P), _resolve(path, n, P),
                                                              ctypes.byref(out)))
    return out.value


def extend(A: DeviceMp, D: DeviceMp, info, n_old: int, path: str = "auto", stream=None):
    """mp_det_extend: A's leading n_old x n_old block (and D_1..D_{n_old}) hold
    a factorisation; eliminate the new rows and columns and continue, in
    place, to the factorisation of the whole matrix."""
    h = handle(A.limbs.device.index or 0)
    _check("mp_det_extend", lib().mp_det_extend(h.ptr, A.mat(), D.mat(), info.data_ptr(), int(n_old),
                                                _resolve(path, A.rows, A.P), _stream(stream)))
    return D, info


RAD_INF = (1 << 63) - 1


def factor_ball(A: DeviceMp, input_ulp: bool = False, path: str = "auto", stream=None):
    """mp_det_factor_ball in place on A: returns (D, rad_mant uint32 [n], rad_exp
    int64 [n], info) device tensors; |D_k - D*_k| <= rad_mant * 2^rad_exp."""
    import torch
    n = A.rows
    dev = A.limbs.device
    D = DeviceMp.empty(1, n, A.P, dev)
    rm = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    re = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    h = handle(dev.index or 0)
    _check("mp_det_factor_ball", lib().mp_det_factor_ball(h.ptr, A.mat(), D.mat(), rm.data_ptr(), re.data_ptr(),
                                                          info.data_ptr(), 1 if input_ulp else 0,
                                                          _resolve(path, n, A.P), _stream(stream)))
    return D, rm, re, info


def truncate(x: DeviceMp, P2: int, stream=None) -> DeviceMp:
    """mp_truncate: x rounded toward zero to P2 limbs (a new array)."""
    y = DeviceMp.empty(x.rows, x.cols, P2, x.limbs.device)
    h = handle(x.limbs.device.index or 0)
    _check("mp_truncate", lib().mp_truncate(h.ptr, x.mat(), y.mat(), _stream(stream)))
    return y


def factor_reduced(A: DeviceMp, k_switch: int, P2: int, path: str = "auto", path2: str = "auto", stream=None):
    """mp_det_factor_reduced: steps before k_switch at A's precision (in place
    on A), the rest at P2 limbs.  Returns (A2, D2, D_lead, info): A2 and D2 the
    factors and D_1..D_n at P2, D_lead D_1..D_{k_switch} at full precision."""
    import torch
    n = A.rows
    dev = A.limbs.device
    D = DeviceMp.empty(1, n, A.P, dev)
    A2 = DeviceMp.empty(n, n, P2, dev)
    D2 = DeviceMp.empty(1, n, P2, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    h = handle(dev.index or 0)
    _check("mp_det_factor_reduced",
           lib().mp_det_factor_reduced(h.ptr, A.mat(), D.mat(), A2.mat(), D2.mat(), info.data_ptr(), int(k_switch),
                                       _resolve(path, n, A.P), _resolve(path2, n, P2), _stream(stream)))
    return A2, D2, D, info


def set_tuning(lane_rows: int = 0, mfma_waves: int = 0, panel_rows: int | None = None, device: int = 0):
    """mpdet_set_tuning (and mpdet_set_panel_rows) on the device's handle:
    rows per workgroup of the lane product (2, 4, 8), waves per workgroup of
    the MFMA update (1, 2, 4); 0 restores a default."""
    h = handle(device).ptr
    _check("mpdet_set_tuning", lib().mpdet_set_tuning(h, int(lane_rows), int(mfma_waves)))
    if panel_rows is not None:
        _check("mpdet_set_panel_rows", lib().mpdet_set_panel_rows(h, int(panel_rows)))


def set_overlap(panels: int, device: int = 0):
    """mpdet_set_overlap on the device's handle: how the MFMA path schedules
    the finish -- 0 inside the update launch above 256 limbs (the default), 1
    a launch of its own, 2..64 row panels whose finish runs on a second stream
    beside the next panel's update."""
    _check("mpdet_set_overlap", lib().mpdet_set_overlap(handle(device).ptr, int(panels)))


def set_panel_rows(rows: int, device: int = 0):
    """mpdet_set_panel_rows on the device's handle (0: automatic)."""
    _check("mpdet_set_panel_rows", lib().mpdet_set_panel_rows(handle(device).ptr, int(rows)))


def minors(LU: DeviceMp, D: DeviceMp, info, c: DeviceMp | None = None, stream=None) -> DeviceMp:
    """mp_det_minors: signed last-column cofactors of the factored matrix."""
    n = LU.rows
    if c is None:
        c = DeviceMp.empty(1, n, LU.P, LU.limbs.device)
    h = handle(LU.limbs.device.index or 0)
    _check("mp_det_minors", lib().mp_det_minors(h.ptr, LU.mat(), D.mat(), c.mat(), info.data_ptr(),
                                                _stream(stream)))
    return c


def adjugate(LU: DeviceMp, D: DeviceMp, info, adjT: DeviceMp | None = None, stream=None,
             h: Handle | None = None) -> DeviceMp:
    """mp_det_adjugate: adj(A)^T = d det / d A from the factored matrix.  `h`:
    a handle of one's own (its workspace), e.g. to run calls on several
    streams at once; default: the device's shared handle."""
    n = LU.rows
    if adjT is None:
        adjT = DeviceMp.empty(n, n, LU.P, LU.limbs.device)
    h = h or handle(LU.limbs.device.index or 0)
    _check("mp_det_adjugate", lib().mp_det_adjugate(h.ptr, LU.mat(), D.mat(), adjT.mat(), info.data_ptr(),
                                                    _stream(stream)))
    return adjT


def adjugate_batched(LUs: list, Ds: list, info, adjTs: list | None = None, status=None, stream=None,
                     schedule: str = "persistent"):
    """mp_det_adjugate_batched: adj(A)^T of every factored matrix of a batch
    (info: the factorisations' int32[batch] device tensor).  schedule:
    "persistent" (one launch) or "lockstep" (one mp_det_adjugate call per
    matrix).  Returns (adjTs, status int32[batch])."""
    import torch
    B = len(LUs)
    dev = LUs[0].limbs.device
    if adjTs is None:
        adjTs = [DeviceMp.empty(m.rows, m.rows, m.P, dev) for m in LUs]
    if status is None:
        status = torch.zeros(B, dtype=torch.int32, device=dev)
    La = (MpdetMat * B)(*[m.mat() for m in LUs])
    Da = (MpdetMat * B)(*[d.mat() for d in Ds])
    Ta = (MpdetMat * B)(*[t.mat() for t in adjTs])
    if schedule not in ("persistent", "lockstep"):
        raise ValueError(f"schedule {schedule!r}: persistent or lockstep")
    flags = MPDET_BATCH_LOCKSTEP if schedule == "lockstep" else 0
    h = handle(dev.index or 0)
    _check("mp_det_adjugate_batched", lib().mp_det_adjugate_batched(h.ptr, B, La, Da, Ta, info.data_ptr(),
                                                                    status.data_ptr(), flags, _stream(stream)))
    return adjTs, status


def all_minors(LU: DeviceMp, D: DeviceMp, info, C: DeviceMp | None = None, stream=None,
               h: Handle | None = None) -> DeviceMp:
    """mp_det_all_minors: row r of C holds the signed last-column cofactors of
    the leading (r+1) x (r+1) block (zeros above the diagonal).  `h` as for
    adjugate()."""
    n = LU.rows
    if C is None:
        C = DeviceMp.empty(n, n, LU.P, LU.limbs.device)
    h = h or handle(LU.limbs.device.index or 0)
    _check("mp_det_all_minors", lib().mp_det_all_minors(h.ptr, LU.mat(), D.mat(), C.mat(), info.data_ptr(),
                                                        _stream(stream)))
    return C


def normalize_minors(C: DeviceMp, out: DeviceMp | None = None, stream=None) -> DeviceMp:
    """mp_det_normalize_minors: every row of C divided by its first entry
    (the normalised minors delta_{N,n} = c_n / c_1)."""
    if out is None:
        out = DeviceMp.empty(C.rows, C.cols, C.P, C.limbs.device)
    h = handle(C.limbs.device.index or 0)
    _check("mp_det_normalize_minors", lib().mp_det_normalize_minors(h.ptr, C.mat(), out.mat(), _stream(stream)))
    return out


MPDET_WANT_MINORS, MPDET_BATCH_LOCKSTEP, MPDET_BATCH_PERSISTENT = 1, 2, 4
SCHEDULES = {"auto": 0, "lockstep": MPDET_BATCH_LOCKSTEP, "persistent": MPDET_BATCH_PERSISTENT}

# one record of mpdet_batched_plan
PLAN_DTYPE = np.dtype([("need", "<i8"), ("units", "<i8"), ("k", "<i8"), ("mat", "<i4"), ("kind", "<i4")])
PLAN_KINDS = ("init", "pivot", "divide", "prod", "finish", "updv", "pend", "msweep", "mfinal")


def batched_plan(sizes, P: int, path: str = "auto", minors: bool = True):
    """mpdet_batched_plan (host only): the persistent launch's records in queue
    order (PLAN_DTYPE) and the total number of tickets."""
    B = len(sizes)
    n = (ctypes.c_int64 * max(B, 1))(*[int(x) for x in sizes])
    nrec, nt = ctypes.c_int64(), ctypes.c_int64()
    flags = MPDET_WANT_MINORS if minors else 0
    pid = PATHS[path]
    _check("mpdet_batched_plan", lib().mpdet_batched_plan(B, n, int(P), pid, flags, None, 0, ctypes.byref(nrec),
                                                          ctypes.byref(nt)))
    out = np.zeros(nrec.value, dtype=PLAN_DTYPE)
    _check("mpdet_batched_plan", lib().mpdet_batched_plan(B, n, int(P), pid, flags, out.ctypes.data, nrec.value,
                                                          ctypes.byref(nrec), ctypes.byref(nt)))
    return out, nt.value


def set_long_division(on: bool, device: int = 0):
    """mpdet_set_long_division on the device's handle: every multiplier of the
    single-matrix calls by long division instead of the pivot's reciprocal
    (the same bits; the reciprocal's fallback path)."""
    _check("mpdet_set_long_division", lib().mpdet_set_long_division(handle(device).ptr, 1 if on else 0))


def set_wait_limit(seconds: float, device: int = 0):
    """mpdet_set_wait_limit on the device's handle: bound on every wait of the
    persistent batched launch."""
    _check("mpdet_set_wait_limit", lib().mpdet_set_wait_limit(handle(device).ptr, float(seconds)))


def batched(mats: list, path: str = "auto", minors: bool = True, Ds=None, cs=None, info=None,
            stream=None, schedule: str = "auto"):
    """mp_det_batched on a list of square DeviceMp matrices (factored in place).
    schedule: "auto" (the library's default, lockstep), "persistent" (one
    launch over a task queue; VALU path) or "lockstep".  Returns (Ds, cs or
    None, info[batch])."""
    import torch
    B = len(mats)
    dev = mats[0].limbs.device
    if Ds is None:
        Ds = [DeviceMp.empty(1, m.rows, m.P, dev) for m in mats]
    if minors and cs is None:
        cs = [DeviceMp.empty(1, m.rows, m.P, dev) for m in mats]
    if info is None:
        info = torch.zeros(B, dtype=torch.int32, device=dev)
    Aa = (MpdetMat * B)(*[m.mat() for m in mats])
    Da = (MpdetMat * B)(*[d.mat() for d in Ds])
    Ca = (MpdetMat * B)(*[c.mat() for c in cs]) if minors else None
    h = handle(dev.index or 0)
    _check("mp_det_batched", lib().mp_det_batched(h.ptr, B, Aa, Da, Ca, info.data_ptr(),
                                                  (MPDET_WANT_MINORS if minors else 0) | SCHEDULES[schedule],
                                                  _resolve(path, max(m.rows for m in mats), mats[0].P),
                                                  _stream(stream)))
    return Ds, (cs if minors else None), info


def to_f64(x: DeviceMp, stream=None):
    """mp_to_f64: (mantissa float64 [rows, cols], exponent int64 [rows, cols]) device tensors."""
    import torch
    mant = torch.zeros((x.rows, x.cols), dtype=torch.float64, device=x.limbs.device)
    e = torch.zeros((x.rows, x.cols), dtype=torch.int64, device=x.limbs.device)
    h = handle(x.limbs.device.index or 0)
    _check("mp_to_f64", lib().mp_to_f64(h.ptr, x.mat(), mant.data_ptr(), e.data_ptr(), _stream(stream)))
    return mant, e


def to_f64_scaled(x: DeviceMp, shift, stream=None):
    """mp_to_f64_scaled: float64 [rows, cols] = RZ_53 value of x * 2^-shift
    (shift: a one-element int64 device tensor)."""
    import torch
    val = torch.zeros((x.rows, x.cols), dtype=torch.float64, device=x.limbs.device)
    shift = shift.reshape(1)
    if shift.dtype != torch.int64 or shift.device != x.limbs.device:
        raise ValueError("shift must be an int64 tensor on the device of x")
    shift = shift.contiguous()
    h = handle(x.limbs.device.index or 0)
    _check("mp_to_f64_scaled",
           lib().mp_to_f64_scaled(h.ptr, x.mat(), shift.data_ptr(), val.data_ptr(), _stream(stream)))
    return val


PEAK_KINDS = {"mad64": 0, "mfma_i8": 1, "mfma_clock": 2}


def measure_peak(kind: str, device: int = 0) -> float:
    """mpdet_measure_peak: measured multiply-adds per second of one unit
    ("mad64": 32x32->64 VALU, "mfma_i8": int8 MFMA), or the shader clock in
    Hz while the MFMA probe runs ("mfma_clock")."""
    out = ctypes.c_double()
    _check("mpdet_measure_peak", lib().mpdet_measure_peak(handle(device).ptr, PEAK_KINDS[kind], ctypes.byref(out)))
    return out.value


KERNELS = ("pivot_divide", "divide", "update_valu", "update_mfma", "mfma_prep", "minors_sweep",
           "minors_final", "update_finish", "adjugate", "all_minors", "batch_persistent", "other")


def profile_begin(device: int = 0):
    _check("mpdet_profile_begin", lib().mpdet_profile_begin(handle(device).ptr))


def profile_end(device: int = 0) -> dict:
    """Stop per-kernel event timing; returns {kernel: (total_ms, launches)}."""
    h = handle(device)
    _check("mpdet_profile_end", lib().mpdet_profile_end(h.ptr))
    out = {}
    for k in KERNELS:
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check("mpdet_profile_get", lib().mpdet_profile_get(h.ptr, k.encode(), ctypes.byref(ms),
                                                            ctypes.byref(n)))
        out[k] = (ms.value, n.value)
    return out


def det(A: DeviceMp, path: str = "auto", stream=None):
    """The whole hot path on A (in place): factor, then minors.
    Returns (D, c, info); det(A) = D[n-1]."""
    D, info = factor(A, path, stream=stream)
    c = minors(A, D, info, stream=stream)
    return D, c, info
