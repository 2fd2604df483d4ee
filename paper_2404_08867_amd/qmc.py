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
EXP_SUM, PRODUCT_PEAK, GAUSSIAN, OSCILLATORY, EXP_QUADRATIC = 0, 1, 2, 3, 4
# qmc_precision
FP64, FP32_COMPENSATED = 0, 1
# qmc_n_mode
N_A_POW_D, N_ONE_PLUS_A_POW_D, N_EXPLICIT = 0, 1, 2
# qmc_implr_method
IMPLR_AUTO, IMPLR_BITMAP = 0, 1
# qmc_criterion_kind
CRIT_P_ALPHA, CRIT_WCE2 = 0, 1
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
        L.qmc_lattice_sum_noalloc.argtypes = [i32, i64, dp, dp, i32, dp, i32, i32, dp, vp]
        L.qmc_lattice_sum_shifts.argtypes = [i32, i64, dp, dp, i32, i32, dp, i32, dp, dp, vp, sz, vp]
        L.qmc_lattice_points.argtypes = [i32, i64, dp, i64, i64, dp, vp]
        L.qmc_criteria_workspace_size.argtypes = [i32, i64, vp]
        L.qmc_mdi_lr_sum_workspace_size.argtypes = [i32, i32, vp]
        L.qmc_mdi_lr_sum.argtypes = [i32, i32, i32, i32, dp, i32, i32, dp, vp, sz, vp]
        L.qmc_bernoulli_sum.argtypes = [i32, i64, dp, i32, i32, dp, dp, vp, sz, vp]
        L.qmc_p_alpha.argtypes = [i32, i64, dp, i32, i32, dp, vp, sz, vp]
        L.qmc_shift_avg_wce2.argtypes = [i32, i64, dp, i32, dp, ctypes.c_double, dp, vp, sz, vp]
        L.qmc_korobov_search.argtypes = [i32, i64, vp, i64, i32, dp, dp, vp, sz, vp]
        L.qmc_cbc.argtypes = [i32, i64, vp, dp, dp, vp, sz, vp]
        L.qmc_implr_workspace_size.argtypes = [i32, i64, i64, vp]
        L.qmc_implr_grid.argtypes = [i32, i64, i64, i32, vp, dp, vp, sz, vp]
        L.qmc_implr_points.argtypes = [i32, i64, i64, i64, i64, dp, i64, vp]
        L.qmc_mdi_lr.argtypes = [i32, dp, i32, dp, i32, i32, dp, vp, sz, vp]
        L.qmc_lattice_sum_adjoint.argtypes = [i32, i64, dp, dp, i32, dp, i32, i32, dp, dp, dp, vp, sz, vp]
        L.qmc_batch_plan_create.argtypes = [i32, vp, i32, vp, vp]
        L.qmc_batch_plan_destroy.argtypes = [vp]
        L.qmc_batch_plan_config.argtypes = [vp, vp]
        L.qmc_batch_plan_set_config.argtypes = [vp, vp]
        L.qmc_batch_workspace_size.argtypes = [vp, vp]
        L.qmc_lattice_sum_batched.argtypes = [vp, dp, vp, sz, vp]
        L.qmc_batch_autotune.argtypes = [vp, dp, vp, sz, vp, i32, vp]
        L.qmc_batch_graph_create.argtypes = [vp, dp, vp, sz, vp]
        L.qmc_graph_launch.argtypes = [vp, vp]
        L.qmc_graph_destroy.argtypes = [vp]
        for name in ("qmc_korobov", "qmc_mdi_lr_dims", "qmc_param_count", "qmc_workspace_size",
                     "qmc_lattice_sum", "qmc_lattice_sum_ex", "qmc_lattice_sum_noalloc",
                     "qmc_lattice_points", "qmc_mdi_lr",
                     "qmc_lattice_sum_adjoint",
                     "qmc_batch_plan_create", "qmc_batch_plan_destroy", "qmc_batch_plan_config",
                     "qmc_batch_plan_set_config", "qmc_batch_workspace_size",
                     "qmc_lattice_sum_batched", "qmc_batch_autotune", "qmc_batch_graph_create",
                     "qmc_graph_launch", "qmc_graph_destroy"):
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


class _on:
    """Makes the device of tensor `t` current around a library call: the library
    launches on the current device, and _stream() is that device's current stream."""

    def __init__(self, t):
        self._ctx = _torch().cuda.device(t.device) if t is not None and t.is_cuda else None

    def __enter__(self):
        if self._ctx is not None:
            self._ctx.__enter__()
        return self

    def __exit__(self, *exc):
        if self._ctx is not None:
            self._ctx.__exit__(*exc)
        return False


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
    with _on(q):
        _check(lib().qmc_lattice_sum_ex(d, n, _ptr(zt), _ptr(st), family, _ptr(pt), nsets, precision,
                                        _ptr(q), w.ptr, w.nbytes, _stream(), ctypes.byref(cfg)),
               "qmc_lattice_sum")
    if out is not None:
        return out
    return q[0] if squeeze else q


def lattice_sum_noalloc(z, n: int, family: int, params, precision: int = FP64, shift=None,
                        device="cuda", out=None):
    """qmc_lattice_sum_noalloc: lattice_sum with the library's static per-device
    scratch instead of a workspace (the library allocates nothing; calls that
    overlap on one device race).  Same arguments and result as lattice_sum."""
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
    with _on(q):
        _check(lib().qmc_lattice_sum_noalloc(d, n, _ptr(zt), _ptr(st), family, _ptr(pt), nsets, precision,
                                             _ptr(q), _stream()), "qmc_lattice_sum_noalloc")
    if out is not None:
        return out
    return q[0] if squeeze else q


def lattice_sum_shifts(z, n: int, family: int, params, shifts, precision: int = FP64,
                       ws: Workspace | None = None, device="cuda", out=None, stats_out=None):
    """Randomly shifted rule (qmc_lattice_sum_shifts): Q_r for each shift row r of
    `shifts` ([R, d], drawn by the caller) with one shared parameter set, and
    (mean, standard error of the mean).  Returns (q [R], stats [2]) device tensors."""
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    pt = _dev(params, torch.float64, device)
    st = _dev(shifts, torch.float64, device)
    d = int(zt.numel())
    if st.dim() == 1:
        st = st.unsqueeze(0)
    if st.dim() != 2 or st.shape[1] != d:
        raise QmcError(ERR_INVALID_ARG, "shifts must have shape [R, d]")
    R = int(st.shape[0])
    if pt.dim() != 1:
        raise QmcError(ERR_INVALID_ARG, "params must be one parameter row")
    q = out if out is not None else torch.empty(R, dtype=torch.float64, device=device)
    stats = stats_out if stats_out is not None else torch.empty(2, dtype=torch.float64, device=device)
    for t, m in ((q, R), (stats, 2)):
        if t.dtype != torch.float64 or t.numel() < m or not t.is_contiguous():
            raise QmcError(ERR_INVALID_ARG, "outputs must be contiguous float64 tensors")
    w = _workspace(d, n, R, device, ws)
    with _on(q):
        _check(lib().qmc_lattice_sum_shifts(d, n, _ptr(zt), _ptr(st), R, family, _ptr(pt), precision,
                                            _ptr(q), _ptr(stats), w.ptr, w.nbytes, _stream()),
               "qmc_lattice_sum_shifts")
    return q, stats


# --------------------------------------------- MDI-LR of the coordinate sum
SUM_POWER, SUM_GAUSS = 0, 1


def mdi_lr_sum_workspace_size(d: int, N: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qmc_mdi_lr_sum_workspace_size(d, N, ctypes.byref(out)), "qmc_mdi_lr_sum_workspace_size")
    return int(out.value)


def mdi_lr_sum(d: int, N: int, N_last: int, gfamily: int, params, precision: int = FP64,
               ws: Workspace | None = None, device="cuda", out=None):
    """Tensor midpoint rule of g(x_1 + ... + x_d) (qmc_mdi_lr_sum) for each parameter
    row of g: (b, c, p) for SUM_POWER, (c, w) for SUM_GAUSS."""
    torch = _torch()
    pt = _dev(params, torch.float64, device)
    squeeze = pt.dim() == 1
    if squeeze:
        pt = pt.unsqueeze(0)
    nsets = int(pt.shape[0])
    q = out if out is not None else torch.empty(nsets, dtype=torch.float64, device=device)
    if ws is None:
        need = mdi_lr_sum_workspace_size(d, N)
        key = ("mdi_sum", str(device), _torch().cuda.current_stream(device).cuda_stream)
        ws = _ws_cache.get(key)
        if ws is None or ws.nbytes < need:
            ws = Workspace(need, device)
            _ws_cache[key] = ws
    with _on(q):
        _check(lib().qmc_mdi_lr_sum(d, N, N_last, gfamily, _ptr(pt), nsets, precision, _ptr(q), ws.ptr,
                                    ws.nbytes, _stream()), "qmc_mdi_lr_sum")
    return q[0] if squeeze and out is None else q


# ----------------------------------------------------------- lattice criteria
def criteria_workspace_size(d: int, n: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qmc_criteria_workspace_size(d, n, ctypes.byref(out)), "qmc_criteria_workspace_size")
    return int(out.value)


def _criteria_workspace(d, n, device, ws):
    if ws is not None:
        return ws
    need = criteria_workspace_size(d, n)
    key = ("criteria", str(device), _torch().cuda.current_stream(device).cuda_stream)
    cur = _ws_cache.get(key)
    if cur is None or cur.nbytes < need:
        cur = Workspace(need, device)
        _ws_cache[key] = cur
    return cur


class Criterion(ctypes.Structure):
    """qmc_criterion: P_alpha of eq. 2.4, or e^2 of eq. 2.12 with product weights."""
    _fields_ = [("kind", ctypes.c_int32), ("alpha", ctypes.c_int32), ("gamma", ctypes.c_void_p),
                ("beta", ctypes.c_double)]


def _criterion(d, alpha, gamma, beta, device):
    """(qmc_criterion, the device tensor of gamma it points to or None)."""
    if gamma is None:
        return Criterion(CRIT_P_ALPHA, alpha, None, 0.0), None
    gt = _dev(gamma, _torch().float64, device)
    if gt.numel() != d:
        raise QmcError(ERR_INVALID_ARG, "gamma must hold d weights")
    return Criterion(CRIT_WCE2, 2, _ptr(gt), float(beta)), gt


def bernoulli_sum(z, n: int, alpha: int, a, ws: Workspace | None = None, device="cuda"):
    """S for each row of z ([nz, d] or [d]): (1/n) sum_k [prod_j (1 + a_j B_alpha({k z_j/n})) - 1]."""
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    if zt.dim() == 1:
        zt = zt.unsqueeze(0)
    nz, d = int(zt.shape[0]), int(zt.shape[1])
    at = _dev(a, torch.float64, device)
    if at.numel() != d:
        raise QmcError(ERR_INVALID_ARG, "a must hold d weights")
    s = torch.empty(nz, dtype=torch.float64, device=device)
    w = _workspace(d, n, nz, device, ws)
    with _on(s):
        _check(lib().qmc_bernoulli_sum(d, n, _ptr(zt), nz, alpha, _ptr(at), _ptr(s), w.ptr, w.nbytes,
                                       _stream()), "qmc_bernoulli_sum")
    return s


def _rows(z, device):
    zt = _dev(z, _torch().int64, device)
    return zt.unsqueeze(0) if zt.dim() == 1 else zt


def p_alpha(z, n: int, alpha: int, ws: Workspace | None = None, device="cuda"):
    """P_alpha(z) of eq. 2.4 for each row of z (qmc_p_alpha); a device tensor [nz]."""
    torch = _torch()
    zt = _rows(z, device)
    nz, d = int(zt.shape[0]), int(zt.shape[1])
    out = torch.empty(nz, dtype=torch.float64, device=device)
    w = _criteria_workspace(d, n, device, ws)
    with _on(out):
        _check(lib().qmc_p_alpha(d, n, _ptr(zt), nz, alpha, _ptr(out), w.ptr, w.nbytes, _stream()),
               "qmc_p_alpha")
    return out


def shift_avg_wce2(z, n: int, gamma, beta: float, ws: Workspace | None = None, device="cuda"):
    """e^2(z) of eq. 2.12 (product weights gamma_j, beta) for each row of z
    (qmc_shift_avg_wce2); a device tensor [nz]."""
    torch = _torch()
    zt = _rows(z, device)
    nz, d = int(zt.shape[0]), int(zt.shape[1])
    gt = _dev(gamma, torch.float64, device)
    if gt.numel() != d:
        raise QmcError(ERR_INVALID_ARG, "gamma must hold d weights")
    out = torch.empty(nz, dtype=torch.float64, device=device)
    w = _criteria_workspace(d, n, device, ws)
    with _on(out):
        _check(lib().qmc_shift_avg_wce2(d, n, _ptr(zt), nz, _ptr(gt), float(beta), _ptr(out), w.ptr,
                                        w.nbytes, _stream()), "qmc_shift_avg_wce2")
    return out


def korobov_search(d: int, n: int, alpha: int = 2, gamma=None, beta: float = 0.0, a0: int = 1,
                   count: int | None = None, ws: Workspace | None = None, device="cuda"):
    """The criterion of z(a) for a = a0 .. a0+count-1 (qmc_korobov_search): P_alpha of
    eq. 2.4 when gamma is None, else e^2 of eq. 2.12 with weights gamma and beta.
    Returns (values [count] device tensor, best [2] device tensor: value, a)."""
    torch = _torch()
    count = (n - a0) if count is None else count
    crit, keep = _criterion(d, alpha, gamma, beta, device)
    vals = torch.empty(count, dtype=torch.float64, device=device)
    best = torch.empty(2, dtype=torch.float64, device=device)
    w = _criteria_workspace(d, n, device, ws)
    with _on(vals):
        _check(lib().qmc_korobov_search(d, n, ctypes.byref(crit), a0, count, _ptr(vals), _ptr(best), w.ptr,
                                        w.nbytes, _stream()), "qmc_korobov_search")
    del keep
    return vals, best


def cbc(d: int, n: int, gamma=None, beta: float = 0.0, alpha: int = 2, ws: Workspace | None = None,
        device="cuda"):
    """CBC generating vector (qmc_cbc) minimising e^2 of eq. 2.12 (weights gamma, beta),
    or P_alpha of eq. 2.4 when gamma is None.  Returns (z [d] int64 device tensor,
    the criterion of (z_1..z_j) for each j [d])."""
    torch = _torch()
    crit, keep = _criterion(d, alpha, gamma, beta, device)
    z = torch.empty(d, dtype=torch.int64, device=device)
    sv = torch.empty(d, dtype=torch.float64, device=device)
    w = _criteria_workspace(d, n, device, ws)
    with _on(z):
        _check(lib().qmc_cbc(d, n, ctypes.byref(crit), _ptr(z), _ptr(sv), w.ptr, w.nbytes, _stream()),
               "qmc_cbc")
    del keep
    return z, sv


# ------------------------------------------------ the improved rule's tensor grid
def implr_workspace_size(d: int, n: int, a: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qmc_implr_workspace_size(d, n, a, ctypes.byref(out)), "qmc_implr_workspace_size")
    return int(out.value)


def implr_grid(d: int, n: int, a: int, method: int = IMPLR_AUTO, ws: Workspace | None = None, out=None,
               device="cuda"):
    """Theorem 3.1's grid for the Korobov lattice z = (1, a, ..., a^{d-1}) (qmc_implr_grid).
    Returns (per-direction counts [d] int64 numpy array, n* [1] int64 device tensor)."""
    torch = _torch()
    counts = np.zeros(d, dtype=np.int64)
    nstar = torch.empty(1, dtype=torch.int64, device=device) if out is None else out
    if ws is None:
        ws = Workspace(implr_workspace_size(d, n, a), device)
    with _on(nstar):
        _check(lib().qmc_implr_grid(d, n, a, method, counts.ctypes.data, _ptr(nstar), ws.ptr, ws.nbytes,
                                    _stream()),
               "qmc_implr_grid")
    return counts, nstar


def implr_points(d: int, n: int, a: int, j0: int, count: int, out=None, device="cuda"):
    """Grid ranks s[i, j - j0] of lattice points j0 .. j0+count-1, direction-major
    (qmc_implr_points).  `out` may be a [d, ld] int32 tensor (ld >= count, rows
    contiguous); the result is its first `count` columns."""
    torch = _torch()
    if out is None:
        ld = (count + 3) // 4 * 4
        out = torch.empty((d, ld), dtype=torch.int32, device=device)
    if out.dtype != torch.int32 or out.dim() != 2 or out.shape[0] != d or out.shape[1] < count or \
            out.stride(1) != 1:
        raise QmcError(ERR_INVALID_ARG, "out must be an int32 [d, ld] tensor with ld >= count and unit column stride")
    ld = int(out.stride(0)) if d > 1 else int(out.shape[1])
    with _on(out):
        _check(lib().qmc_implr_points(d, n, a, j0, count, _ptr(out) if count else None, ld, _stream()),
               "qmc_implr_points")
    return out[:, :count]


def lattice_points(z, n: int, i0: int, count: int, device="cuda"):
    """Point indices k[r, j] = ((i0 + r) z_j) mod n from the device generator."""
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    d = int(zt.numel())
    k = torch.empty((count, d), dtype=torch.int32, device=device)
    with _on(k):
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
    with _on(q):
        _check(lib().qmc_mdi_lr(d, _ptr(Nt), family, _ptr(pt), nsets, precision, _ptr(q), None, 0,
                                _stream()), "qmc_mdi_lr")
    if out is not None:
        return out
    return q[0] if squeeze else q


# ---- batched sums ---------------------------------------------------------------
class Problem(ctypes.Structure):
    """qmc_problem: one integrand of a batch (device pointers)."""
    _fields_ = [("family", ctypes.c_int32), ("d", ctypes.c_int32), ("n", ctypes.c_int64),
                ("z", ctypes.c_void_p), ("params", ctypes.c_void_p), ("shift", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    """qmc_batch_config: points per thread, workgroups per CU, order (0 = longest first)."""
    _fields_ = [("points_per_thread", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32)]

    def as_dict(self):
        return {"points_per_thread": self.points_per_thread,
                "workgroups_per_cu": self.workgroups_per_cu, "order": self.order}


class BatchPlan:
    """A batch of plain lattice sums evaluated in one persistent launch.

    `problems` is a list of (family, z, n, params, shift) with z, params, shift as
    1-D host arrays or tensors; they are packed into three flat device tensors
    that this object keeps alive (the plan holds pointers into them)."""

    def __init__(self, problems, precision: int = FP32_COMPENSATED, config: dict | None = None,
                 device="cuda"):
        torch = _torch()
        self.device = device
        self.count = len(problems)
        zs, ps, ss, descs = [], [], [], []
        zoff = poff = soff = 0
        for fam, z, n, params, shift in problems:
            z = np.asarray(z.cpu() if hasattr(z, "cpu") else z, dtype=np.int64).ravel()
            params = np.asarray(params.cpu() if hasattr(params, "cpu") else params, dtype=np.float64).ravel()
            descs.append((int(fam), int(z.size), int(n), zoff, poff, None if shift is None else soff))
            zs.append(z)
            ps.append(params)
            zoff += z.size
            poff += params.size
            if shift is not None:
                sh = np.asarray(shift.cpu() if hasattr(shift, "cpu") else shift, dtype=np.float64).ravel()
                ss.append(sh)
                soff += sh.size
        self.z = torch.as_tensor(np.concatenate(zs), device=device)
        self.params = torch.as_tensor(np.concatenate(ps), device=device)
        self.shift = torch.as_tensor(np.concatenate(ss) if ss else np.zeros(1), device=device)
        arr = (Problem * self.count)()
        zb, pb, sb = self.z.data_ptr(), self.params.data_ptr(), self.shift.data_ptr()
        for i, (fam, d, n, zo, po, so) in enumerate(descs):
            arr[i] = Problem(fam, d, n, zb + 8 * zo, pb + 8 * po, None if so is None else sb + 8 * so)
        cfg = None
        if config:
            cfg = BatchConfig(config.get("points_per_thread", 0), config.get("workgroups_per_cu", 0),
                              config.get("order", 0))
        self._plan = ctypes.c_void_p()
        with _on(self.z):  # the plan's device arrays live on the problems' device
            _check(lib().qmc_batch_plan_create(self.count, ctypes.byref(arr), precision,
                                               ctypes.byref(cfg) if cfg is not None else None,
                                               ctypes.byref(self._plan)), "qmc_batch_plan_create")
        b = ctypes.c_size_t(0)
        _check(lib().qmc_batch_workspace_size(self._plan, ctypes.byref(b)), "qmc_batch_workspace_size")
        self.ws = Workspace(int(b.value), device)

    @classmethod
    def from_batch(cls, batch, precision: int = FP32_COMPENSATED, config=None, device="cuda"):
        """Plan for a workloads.Batch (Korobov z from qmc_korobov for each problem)."""
        probs = [(p.family, korobov(p.d, p.n, p.a), p.n, p.params, p.shift) for p in batch.problems]
        return cls(probs, precision, config, device)

    @property
    def config(self) -> dict:
        c = BatchConfig()
        _check(lib().qmc_batch_plan_config(self._plan, ctypes.byref(c)), "qmc_batch_plan_config")
        return c.as_dict()

    def set_config(self, **kw):
        c = BatchConfig(kw.get("points_per_thread", 8), kw.get("workgroups_per_cu", 4), kw.get("order", 0))
        _check(lib().qmc_batch_plan_set_config(self._plan, ctypes.byref(c)), "qmc_batch_plan_set_config")

    def run(self, out=None):
        torch = _torch()
        q = out if out is not None else torch.empty(self.count, dtype=torch.float64, device=self.device)
        with _on(q):
            _check(lib().qmc_lattice_sum_batched(self._plan, _ptr(q), self.ws.ptr, self.ws.nbytes, _stream()),
                   "qmc_lattice_sum_batched")
        return q

    def autotune(self, reps: int = 2, out=None) -> dict:
        torch = _torch()
        q = out if out is not None else torch.empty(self.count, dtype=torch.float64, device=self.device)
        best = BatchConfig()
        with _on(q):
            _check(lib().qmc_batch_autotune(self._plan, _ptr(q), self.ws.ptr, self.ws.nbytes, _stream(), reps,
                                            ctypes.byref(best)), "qmc_batch_autotune")
        return best.as_dict()

    def graph(self, out):
        """A native HIP graph replaying one batched launch into `out`."""
        return Graph(self, out)

    def __del__(self):
        if getattr(self, "_plan", None) and _lib is not None:
            _lib.qmc_batch_plan_destroy(self._plan)
            self._plan = None


class Graph:
    def __init__(self, plan: BatchPlan, out):
        self._keep = (plan, out)
        self._g = ctypes.c_void_p()
        with _on(out):
            _check(lib().qmc_batch_graph_create(plan._plan, _ptr(out), plan.ws.ptr, plan.ws.nbytes,
                                                ctypes.byref(self._g)), "qmc_batch_graph_create")

    def launch(self):
        with _on(self._keep[1]):
            _check(lib().qmc_graph_launch(self._g, _stream()), "qmc_graph_launch")

    def __del__(self):
        if getattr(self, "_g", None) and _lib is not None:
            _lib.qmc_graph_destroy(self._g)
            self._g = None


# ---- adjoint -----------------------------------------------------------------
def lattice_sum_adjoint(z, n: int, family: int, params, precision: int = FP64, shift=None, gq=None,
                        ws: Workspace | None = None, device="cuda"):
    """(Q, gq * dQ/dparams) of the plain rule for each parameter row (qmc_lattice_sum_adjoint).

    params: float64 [P] or [nsets, P]; gq: float64 [nsets] or None (= 1).
    Returns (q [nsets], grad [nsets, P]) device tensors (squeezed for 1-D params)."""
    torch = _torch()
    zt = _dev(z, torch.int64, device)
    pt = _dev(params, torch.float64, device)
    squeeze = pt.dim() == 1
    if squeeze:
        pt = pt.unsqueeze(0)
    d = int(zt.numel())
    nsets, P = int(pt.shape[0]), int(pt.shape[1])
    st = None if shift is None else _dev(shift, torch.float64, device)
    gt = None if gq is None else _dev(gq, torch.float64, device).reshape(-1)
    if gt is not None and gt.numel() != nsets:
        raise QmcError(ERR_INVALID_ARG, "gq must have one value per parameter set")
    q = torch.empty(nsets, dtype=torch.float64, device=device)
    g = torch.empty((nsets, P), dtype=torch.float64, device=device)
    w = _workspace(d, n, nsets, device, ws)
    with _on(q):
        _check(lib().qmc_lattice_sum_adjoint(d, n, _ptr(zt), _ptr(st), family, _ptr(pt), nsets, precision,
                                             _ptr(gt), _ptr(q), _ptr(g), w.ptr, w.nbytes, _stream()),
               "qmc_lattice_sum_adjoint")
    if squeeze:
        return q[0], g[0]
    return q, g


def _autograd_class():
    torch = _torch()

    class LatticeSumFunction(torch.autograd.Function):
        """Q = lattice_sum(params) with dQ/dparams from the adjoint kernel.

        forward: qmc_lattice_sum;  backward(gQ): qmc_lattice_sum_adjoint with gq = gQ."""

        @staticmethod
        def forward(ctx, params, z, n, family, precision, shift):
            ctx.save_for_backward(params, z, shift if shift is not None else torch.empty(0))
            ctx.n, ctx.family, ctx.precision, ctx.has_shift = n, family, precision, shift is not None
            return lattice_sum(z, n, family, params, precision, shift=shift)

        @staticmethod
        def backward(ctx, gq):
            params, z, shift = ctx.saved_tensors
            sh = shift if ctx.has_shift else None
            one_d = params.dim() == 1
            g_in = gq.reshape(1) if one_d else gq.contiguous()
            _, grad = lattice_sum_adjoint(z, ctx.n, ctx.family, params, ctx.precision, shift=sh,
                                          gq=g_in, device=params.device)
            return grad, None, None, None, None, None

    return LatticeSumFunction


_LSF = None


def lattice_sum_autograd(params, z, n: int, family: int, precision: int = FP64, shift=None):
    """Differentiable Q (w.r.t. params) through the HIP forward and adjoint kernels."""
    global _LSF
    torch = _torch()
    if _LSF is None:
        _LSF = _autograd_class()
    zt = _dev(z, torch.int64, params.device)
    st = None if shift is None else _dev(shift, torch.float64, params.device)
    return _LSF.apply(params, zt, n, family, precision, st)
