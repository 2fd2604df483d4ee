"""Thin ctypes binding of libqmc.so (include/qmc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory and the current stream.  The library
is loaded on first use; if it is missing the call raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmc.so")

# qmc_family
EXP_SUM, PRODUCT_PEAK, GAUSSIAN, OSCILLATORY = 0, 1, 2, 3
# qmc_precision
FP64, FP32_COMPENSATED = 0, 1
# qmc_n_mode
N_A_POW_D, N_ONE_PLUS_A_POW_D, N_EXPLICIT = 0, 1, 2
# qmc_status
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_OUT_OF_MEMORY, ERR_DEVICE = range(6)

_lib = None
_lock = threading.Lock()


class QmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise QmcError(ERR_UNSUPPORTED, f"{LIB_PATH} is missing: run "
                           "`python -m paper_2404_08867_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, sz, vp, dp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                                ctypes.c_void_p, ctypes.c_void_p)
        L.qmc_version.restype = ctypes.c_char_p
        L.qmc_status_string.restype = ctypes.c_char_p
        L.qmc_status_string.argtypes = [ctypes.c_int]
        L.qmc_last_error.restype = ctypes.c_char_p
        L.qmc_korobov.argtypes = [i32, i64, i64, vp]
        L.qmc_mdi_lr_dims.argtypes = [i32, i64, i32, i64, vp]
        L.qmc_param_count.argtypes = [i32, i32, vp]
        L.qmc_workspace_size.argtypes = [i32, i64, i32, vp]
        L.qmc_lattice_sum.argtypes = [i32, i64, dp, dp, i32, dp, i32, i32, dp, vp, sz, vp]
        L.qmc_lattice_sum_ex.argtypes = [i32, i64, dp, dp, i32, dp, i32, i32, dp, vp, sz, vp, vp]
        L.qmc_lattice_points.argtypes = [i32, i64, dp, i64, i64, dp, vp]
        L.qmc_mdi_lr.argtypes = [i32, dp, i32, dp, i32, i32, dp, vp, sz, vp]
        for name in ("qmc_korobov", "qmc_mdi_lr_dims", "qmc_param_count", "qmc_workspace_size",
                     "qmc_lattice_sum", "qmc_lattice_sum_ex", "qmc_lattice_points", "qmc_mdi_lr"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().qmc_last_error().decode()


def _check(status: int, what: str):
    if status != OK:
        raise QmcError(status, f"{what}: {last_error() or lib().qmc_status_string(status).decode()}")


def version() -> str:
    return lib().qmc_version().decode()


# ---- host helpers --------------------------------------------------------------
def korobov(d: int, n: int, a: int) -> np.ndarray:
    z = np.zeros(d, dtype=np.int64)
    _check(lib().qmc_korobov(d, n, a, z.ctypes.data), "qmc_korobov")
    return z


def mdi_lr_dims(d: int, a: int, n_mode: int = N_A_POW_D, n_explicit: int = 0) -> np.ndarray:
    N = np.zeros(d, dtype=np.int32)
    _check(lib().qmc_mdi_lr_dims(d, a, n_mode, n_explicit, N.ctypes.data), "qmc_mdi_lr_dims")
    return N


def param_count(family: int, d: int) -> int:
    c = ctypes.c_int32(0)
    _check(lib().qmc_param_count(family, d, ctypes.byref(c)), "qmc_param_count")
    return int(c.value)


def workspace_size(max_d: int, max_n: int, max_sets: int = 1) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().qmc_workspace_size(max_d, max_n, max_sets, ctypes.byref(b)), "qmc_workspace_size")
    return int(b.value)


# ---- device calls ----------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _dev(x, dtype, device):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        if x.dtype != dtype or x.device != torch.device(device):
            x = x.to(device=device, dtype=dtype)
        return x.contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


class LaunchConfig(ctypes.Structure):
    """qmc_launch_config: points per thread (0/4/8/16) and workgroups per set (0 = auto)."""
    _fields_ = [("points_per_thread", ctypes.c_int32), ("max_blocks", ctypes.c_int32)]


class Workspace:
    """Zero-filled device scratch buffer reused across calls (see include/qmc.h)."""

    def __init__(self, nbytes: int, device="cuda"):
        torch = _torch()
        self.nbytes = max(256, int(nbytes))
        self.buf = torch.zeros(self.nbytes, dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0

    @property
    def ptr(self) -> int:
        return int(self.buf.data_ptr())


_ws_cache: dict = {}


def _workspace(d, n, nsets, device, ws):
    if ws is not None:
        return ws
    need = workspace_size(d, n, nsets)
    key = (str(device), _torch().cuda.current_stream(device).cuda_stream)
    cur = _ws_cache.get(key)
    if cur is None or cur.nbytes < need:
        cur = Workspace(need, device)
        _ws_cache[key] = cur
    return cur


def lattice_sum(z, n: int, family: int, params, precision: int = FP64, shift=None,
                ws: Workspace | None = None, device="cuda", points_per_thread: int = 0,
                max_blocks: int = 0, out=None):
    """Q_s = (1/n) sum_i f_s(x_i) for each parameter row s (qmc_lattice_sum).

    z: int64 [d]; params: float64 [P] or [nsets, P]; shift: float64 [d] or None.
    Returns a float64 device tensor of shape [nsets] (or a 0-d tensor for 1-D params).
    """
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    pt = _dev(params, torch.float64, device)
    squeeze = pt.dim() == 1
    if squeeze:
        pt = pt.unsqueeze(0)
    d = int(zt.numel())
    nsets = int(pt.shape[0])
    st = None if shift is None else _dev(shift, torch.float64, device)
    if out is not None:
        if out.dtype != torch.float64 or out.numel() < nsets or not out.is_contiguous():
            raise QmcError(ERR_INVALID_ARG, "out must be a contiguous float64 tensor of >= nsets values")
        q = out
    else:
        q = torch.empty(nsets, dtype=torch.float64, device=device)
    w = _workspace(d, n, nsets, device, ws)
    cfg = LaunchConfig(points_per_thread, max_blocks)
    _check(lib().qmc_lattice_sum_ex(d, n, _ptr(zt), _ptr(st), family, _ptr(pt), nsets, precision,
                                    _ptr(q), w.ptr, w.nbytes, _stream(), ctypes.byref(cfg)),
           "qmc_lattice_sum")
    if out is not None:
        return out
    return q[0] if squeeze else q


def lattice_points(z, n: int, i0: int, count: int, device="cuda"):
    """Point indices k[r, j] = ((i0 + r) z_j) mod n from the device generator."""
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    d = int(zt.numel())
    k = torch.empty((count, d), dtype=torch.int32, device=device)
    _check(lib().qmc_lattice_points(d, n, _ptr(zt), i0, count, _ptr(k) if count else None,
                                    _stream()), "qmc_lattice_points")
    return k


def mdi_lr(N, family: int, params, precision: int = FP64, device="cuda", out=None):
    """MDI-LR value(s) of the improved tensor rule with node counts N (qmc_mdi_lr)."""
    torch = _torch()
    Nt = _dev(N, torch.int32, device)
    pt = _dev(params, torch.float64, device)
    squeeze = pt.dim() == 1
    if squeeze:
        pt = pt.unsqueeze(0)
    d = int(Nt.numel())
    nsets = int(pt.shape[0])
    q = out if out is not None else torch.empty(nsets, dtype=torch.float64, device=device)
    _check(lib().qmc_mdi_lr(d, _ptr(Nt), family, _ptr(pt), nsets, precision, _ptr(q), None, 0,
                            _stream()), "qmc_mdi_lr")
    if out is not None:
        return out
    return q[0] if squeeze else q
