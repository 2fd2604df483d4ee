"""Plain FP64 CPU oracle for the rank-1 lattice sum and its MDI-LR form.

TEST INFRASTRUCTURE ONLY: the checker, not the product.  Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library (``paper_2404_08867_amd``)
and neither side imports the other; the C source ``qmc_oracle.c`` is compiled
with gcc into ``liboracle.so`` next to it.

This module is argument marshalling only: every arithmetic step lives in the
C file, which cites the paper passage each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

EXP_SUM, PRODUCT_PEAK, GAUSSIAN, OSCILLATORY, EXP_QUADRATIC = 0, 1, 2, 3, 4
TEST1_F, SIN_SQ = 100, 101

_lib = None


def build(verbose: bool = False) -> str:
    """Compile ``qmc_oracle.c`` into ``liboracle.so`` (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-ffp-contract=off", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, dp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_korobov.argtypes = [i32, i64, i64, dp]
    lib.oracle_lattice_points.argtypes = [i32, i64, dp, i64, i64, dp]
    lib.oracle_param_count.argtypes = [i32, i32]
    lib.oracle_eval.argtypes = [i32, i32, dp, dp]
    lib.oracle_eval.restype = ctypes.c_double
    lib.oracle_lattice_sum.argtypes = [i32, i64, dp, dp, i32, dp, dp, dp]
    lib.oracle_lattice_partial.argtypes = [i32, i64, dp, dp, i32, dp, i64, i64, dp]
    lib.oracle_lattice_grad.argtypes = [i32, i64, dp, dp, i32, dp, dp, dp]
    lib.oracle_shift_ensemble.argtypes = [i32, i64, dp, i32, dp, dp, i32, dp, dp, dp]
    lib.oracle_bernoulli.argtypes = [i32, ctypes.c_double]
    lib.oracle_bernoulli.restype = ctypes.c_double
    lib.oracle_lattice_kernel_sum.argtypes = [i32, i64, dp, i32, dp, dp, dp]
    lib.oracle_p_alpha.argtypes = [i32, i64, dp, i32, dp]
    lib.oracle_shift_avg_wce2.argtypes = [i32, i64, dp, dp, ctypes.c_double, dp]
    lib.oracle_korobov_search.argtypes = [i32, i64, i32, i64, i64, dp, dp]
    lib.oracle_cbc.argtypes = [i32, i64, dp, ctypes.c_double, dp, dp]
    lib.oracle_mdi_sum_brute.argtypes = [i32, i64, i64, i32, dp, dp]
    lib.oracle_mdi_sum_sweep.argtypes = [i32, i64, i64, i32, dp, dp, dp]
    lib.oracle_implr_coords.argtypes = [i32, i64, dp, dp]
    lib.oracle_implr_grid.argtypes = [i32, i64, dp, dp, dp, dp]
    lib.oracle_implr_coords_at.argtypes = [i32, i64, dp, i64, dp, dp]
    lib.oracle_mdi_dims.argtypes = [i32, dp, i64, dp]
    lib.oracle_mdi_lr_brute.argtypes = [i32, dp, i32, dp, dp]
    lib.oracle_mdi_lr_sweep.argtypes = [i32, dp, i32, dp, dp]
    lib.oracle_mdi_lr_factors.argtypes = [i32, dp, i32, dp, dp, dp]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def param_count(family: int, d: int) -> int:
    return int(_load().oracle_param_count(family, d))


def korobov(d: int, n: int, a: int) -> np.ndarray:
    z = np.zeros(d, dtype=np.int64)
    _check(_load().oracle_korobov(d, n, a, _ptr(z)), "korobov")
    return z


def lattice_points(z, n: int, i0: int = 0, count: int | None = None) -> np.ndarray:
    z = _i64(z)
    d = z.size
    count = n - i0 if count is None else count
    k = np.zeros((count, d), dtype=np.int64)
    _check(_load().oracle_lattice_points(d, n, _ptr(z), i0, count, _ptr(k)), "lattice_points")
    return k


def evaluate(family: int, params, x) -> float:
    x = _f64(x)
    params = _f64(params) if params is not None else np.zeros(1)
    return float(_load().oracle_eval(family, x.size, _ptr(params), _ptr(x)))


def lattice_sum(z, n: int, family: int, params, shift=None):
    """Return (Q, A): the plain rule and the mean absolute integrand value."""
    z = _i64(z)
    params = _f64(params) if params is not None else np.zeros(1)
    shift = _f64(shift)
    q = np.zeros(1)
    a = np.zeros(1)
    _check(_load().oracle_lattice_sum(z.size, n, _ptr(z), _ptr(shift), family, _ptr(params),
                                      _ptr(q), _ptr(a)), "lattice_sum")
    return float(q[0]), float(a[0])


def lattice_partial(z, n: int, family: int, params, i0: int, count: int, shift=None) -> float:
    """Un-normalised sum of f over the lattice indices [i0, i0 + count)."""
    z = _i64(z)
    params = _f64(params)
    shift = _f64(shift)
    out = np.zeros(1)
    _check(_load().oracle_lattice_partial(z.size, n, _ptr(z), _ptr(shift), family, _ptr(params),
                                          i0, count, _ptr(out)), "lattice_partial")
    return float(out[0])


def lattice_grad(z, n: int, family: int, params, shift=None):
    """Return (Q, dQ/dparams) of the plain rule."""
    z = _i64(z)
    params = _f64(params)
    shift = _f64(shift)
    q = np.zeros(1)
    g = np.zeros(params.size)
    _check(_load().oracle_lattice_grad(z.size, n, _ptr(z), _ptr(shift), family, _ptr(params),
                                       _ptr(q), _ptr(g)), "lattice_grad")
    return float(q[0]), g


def shift_ensemble(z, n: int, family: int, params, shifts):
    """Randomly shifted rule over the rows of `shifts` (R x d): (Q[R], mean, standard error)."""
    z = _i64(z)
    params = _f64(params)
    shifts = _f64(np.atleast_2d(shifts))
    R = shifts.shape[0]
    q = np.zeros(R)
    mean = np.zeros(1)
    se = np.zeros(1)
    _check(_load().oracle_shift_ensemble(z.size, n, _ptr(z), family, _ptr(params), _ptr(shifts), R,
                                         _ptr(q), _ptr(mean), _ptr(se)), "shift_ensemble")
    return q, float(mean[0]), float(se[0])


def bernoulli(alpha: int, x: float) -> float:
    """Bernoulli polynomial B_alpha(x), alpha in {2, 4}."""
    return float(_load().oracle_bernoulli(alpha, float(x)))


def lattice_kernel_sum(z, n: int, alpha: int, a):
    """(S, A): S = (1/n) sum_k [prod_j (1 + a_j B_alpha({k z_j/n})) - 1], A its mean |term|."""
    z = _i64(z)
    a = _f64(a)
    out = np.zeros(2)
    _check(_load().oracle_lattice_kernel_sum(z.size, n, _ptr(z), alpha, _ptr(a), _ptr(out[0:]),
                                             _ptr(out[1:])), "lattice_kernel_sum")
    return float(out[0]), float(out[1])


def p_alpha(z, n: int, alpha: int) -> float:
    """P_alpha(z) by eq. 2.4."""
    z = _i64(z)
    out = np.zeros(1)
    _check(_load().oracle_p_alpha(z.size, n, _ptr(z), alpha, _ptr(out)), "p_alpha")
    return float(out[0])


def shift_avg_wce2(z, n: int, gamma, beta: float) -> float:
    """Squared shift-averaged worst-case error by eq. 2.12 (product weights)."""
    z = _i64(z)
    gamma = _f64(gamma)
    out = np.zeros(1)
    _check(_load().oracle_shift_avg_wce2(z.size, n, _ptr(z), _ptr(gamma), float(beta), _ptr(out)),
           "shift_avg_wce2")
    return float(out[0])


def korobov_search(d: int, n: int, alpha: int, a0: int = 1, count: int | None = None):
    """P_alpha(z(a)) for a = a0 .. a0+count-1 and the best a (first minimum)."""
    count = n - a0 if count is None else count
    vals = np.zeros(count)
    best = np.zeros(1, dtype=np.int64)
    _check(_load().oracle_korobov_search(d, n, alpha, a0, count, _ptr(vals), _ptr(best)),
           "korobov_search")
    return vals, int(best[0])


def cbc(d: int, n: int, gamma, beta: float):
    """CBC generating vector (z[d]) and the criterion after each component (e2[d])."""
    gamma = _f64(gamma)
    z = np.zeros(d, dtype=np.int64)
    e2 = np.zeros(d)
    _check(_load().oracle_cbc(d, n, _ptr(gamma), float(beta), _ptr(z), _ptr(e2)), "cbc")
    return z, e2


def mdi_sum_brute(d: int, N: int, N_last: int, gfam: int, gp) -> float:
    """Tensor midpoint rule of g(sum x) by brute force over the grid."""
    gp = _f64(gp)
    q = np.zeros(1)
    _check(_load().oracle_mdi_sum_brute(d, N, N_last, gfam, _ptr(gp), _ptr(q)), "mdi_sum_brute")
    return float(q[0])


def mdi_sum(d: int, N: int, N_last: int, gfam: int, gp, counts: bool = False):
    """Tensor midpoint rule of g(sum x) by the merged-state dimension iteration;
    with counts=True also the number of index tuples per state after d-1 directions."""
    gp = _f64(gp)
    q = np.zeros(1)
    c = np.zeros((d - 1) * (N - 1) + 1) if counts else None
    _check(_load().oracle_mdi_sum_sweep(d, N, N_last, gfam, _ptr(gp), _ptr(q), _ptr(c)), "mdi_sum")
    return (float(q[0]), c) if counts else float(q[0])


def implr_coords(z, n: int) -> np.ndarray:
    """Integer numerators [n, d] of the transformed coordinates of Theorem 3.1."""
    z = _i64(z)
    u = np.zeros((n, z.size), dtype=np.int64)
    _check(_load().oracle_implr_coords(z.size, n, _ptr(z), _ptr(u)), "implr_coords")
    return u


def implr_coords_at(z, n: int, js) -> np.ndarray:
    """implr_coords at the chosen lattice points js only (any n below 2^31)."""
    z = _i64(z)
    js = _i64(js)
    u = np.zeros((js.size, z.size), dtype=np.int64)
    _check(_load().oracle_implr_coords_at(z.size, n, _ptr(z), js.size, _ptr(js), _ptr(u)), "implr_coords_at")
    return u


def implr_grid(z, n: int):
    """(counts per direction, n*, distinct transformed points) of the improved rule."""
    z = _i64(z)
    counts = np.zeros(z.size, dtype=np.int64)
    out = np.zeros(2, dtype=np.int64)
    _check(_load().oracle_implr_grid(z.size, n, _ptr(z), _ptr(counts), _ptr(out[0:]), _ptr(out[1:])),
           "implr_grid")
    return counts, int(out[0]), int(out[1])


def mdi_dims(z, n: int) -> np.ndarray:
    """Per-direction node counts of eq. 3.5 for generating vector z and n points."""
    z = _i64(z)
    N = np.zeros(z.size, dtype=np.int64)
    _check(_load().oracle_mdi_dims(z.size, _ptr(z), n, _ptr(N)), "mdi_dims")
    return N


def mdi_lr_brute(N, family: int, params) -> float:
    N = _i64(N)
    params = _f64(params)
    out = np.zeros(1)
    _check(_load().oracle_mdi_lr_brute(N.size, _ptr(N), family, _ptr(params), _ptr(out)),
           "mdi_lr_brute")
    return float(out[0])


def mdi_lr(N, family: int, params) -> float:
    """MDI-LR value (dimension sweep, m = 1) of the improved tensor rule."""
    N = _i64(N)
    params = _f64(params)
    out = np.zeros(1)
    _check(_load().oracle_mdi_lr_sweep(N.size, _ptr(N), family, _ptr(params), _ptr(out)),
           "mdi_lr_sweep")
    return float(out[0])


def mdi_lr_factors(N, family: int, params):
    N = _i64(N)
    params = _f64(params)
    re = np.zeros(N.size)
    im = np.zeros(N.size)
    _check(_load().oracle_mdi_lr_factors(N.size, _ptr(N), family, _ptr(params), _ptr(re),
                                         _ptr(im)), "mdi_lr_factors")
    return re, im
