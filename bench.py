#!/usr/bin/env python3
"""Throughput of the rank-1 lattice-sum hot path on one MI355X.

One step is one pass of the hot path over the whole workload.  The default
workload is `batched_4096`: 4096 plain lattice rules (d uniform in [8, 200], n a
prime in [2^12, 2^22], each with its own seeded Korobov z; exp-sum, product-peak
and Gaussian integrands) in one persistent launch -- index generation,
coordinates, integrand, per-thread, wavefront, workgroup and per-integrand
reductions, all fused -- with QMC_FP32_COMPENSATED; the QMC_FP64 path is timed
beside it.  `--workload` selects the other workloads (the plain rule at d = 20,
MDI-LR, the adjoint, shifts, criteria, the improved rule's grid, the issue-rate
probe behind the roofline's peak).

Timing: W warm-up steps, then K steps (captured in one HIP graph and replayed once
for the microsecond-scale plain sums; issued eagerly for the long ones) between two
device synchronisations; the inputs are resident in HBM.  HIP events recorded on
the launch stream give the average kernel duration used for the roofline.  Every
GPU result is compared with the FP64 CPU oracle (for the batched workload: all
4096 integrands against the oracle's cached values), and the oracle itself is
timed on a bounded sample of the workload over the host cores and on one core.

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

W_FAMILY = {0: "exp_sum", 1: "product_peak", 2: "gaussian", 3: "oscillatory", 4: "exp_quadratic"}

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "lattice-point integrand evals/sec at rel err ≤1e-6 vs FP64 oracle (1 GPU)"

# ALU peak of MI355X in 32-bit VALU lane-operation slots: 256 CUs x 128 lanes x
# 2.4 GHz = 78.6 T/s, AMD's FP32 vector rate (157.3 TFLOP/s, an FMA counted as two
# flops).  One instruction type alone issues at half of it (64 lanes per CU per
# clock, measured), but the lattice loops mix 32-bit integer and FP32 work and run
# above that rate, so the 128-lane figure is the ceiling.  Costs in slots:
C32 = 1   # 32-bit integer or FP32 operation
C64 = 2   # FP64 operation (FP64 vector rate 78.6 TFLOP/s: half the 32-bit rate)
CT = 4    # v_exp_f32 / v_rcp_f32 / v_cos_f32 (a quarter of the 32-bit rate, measured)
PEAK_SLOTS = 256 * 128 * 2.4e9

# Algorithmic work per lattice point of the QMC_FP32_COMPENSATED path, in slots:
# per direction, the exact-float index step (two FP32 adds and an unsigned minimum, or
# the integer step's two adds and a minimum: 3) plus the family's operations once the
# coordinate's scale and offset are folded into its first FMA; per point, one
# transcendental and the FP64 accumulation (convert, add).
#   exp-sum, oscillatory: conversion to FP64, FP64 argument FMA;
#   Gaussian:             conversion, FP64 y = b k + g, FP64 y^2 accumulated;
#   product peak:         FP32 y, y^2 + g, product (d <= 32, the exact float taken
#                         as it is); FP64 factors above 32 directions (conversion, three
#                         FP64 operations).
INDEX = 3 * C32
ACCUM = 2 * C64
PEAK_F32_MAX_DIMS = 32


def work_per_point(d: int, family: int) -> int:
    if family == 1:  # product peak
        if d <= PEAK_F32_MAX_DIMS:
            per_dim = INDEX + 3 * C32
        else:
            per_dim = INDEX + C64 + 3 * C64
    elif family in (2, 4):  # Gaussian, exp of a signed quadratic (y, then s y^2 added)
        per_dim = INDEX + C64 + 2 * C64
    else:  # exp-sum, oscillatory
        per_dim = INDEX + C64 + C64
    return d * per_dim + CT + ACCUM


# The count the roofline's `achieved` uses: the minimal work per point of the plain
# rule counted one operation per lane, W = d (3 index + 2 coordinate + c_f) + 1
# transcendental + 6 (accumulation and scaling), c_f = 1 (exp-sum, oscillatory),
# 2 (Gaussian, exp of a signed quadratic), 3 (product peak); per MDI-LR factor
# evaluation 2 FMAs + 1 exp = 3.  work_per_point() above weights the same operations by
# their measured issue cost (an FP64 operation two 32-bit slots) and is reported beside
# it as `measured_costs`.
LANE_OPS_FAMILY = {0: 1, 3: 1, 2: 2, 4: 2, 1: 3}


def lane_ops_per_point(d: int, family: int) -> int:
    return d * (3 + 2 + LANE_OPS_FAMILY[family]) + 1 + 6


LANE_OPS_PER_MDI_FACTOR = 3


# The adjoint's second sweep regenerates each direction's indices and accumulates
# w(x) h_j(x_j): index step, conversion, coordinate FMA and accumulating FMA (FP64),
# plus a second transcendental per point.
def work_per_point_adjoint(d: int, family: int) -> int:
    return work_per_point(d, family) + d * (INDEX + 3 * C64) + CT


# Set-batched adjoint (exp-sum and oscillatory, d <= 64, >= 16 sets sharing the
# lattice): two dense FP64 contractions over the lattice indices, the arguments
# T = k A and the index-weighted sums K = k^T W, on the FP64 matrix unit: 2 d
# flops each per point and set (d unpadded), against the dense FP64 MFMA peak.
PEAK_MFMA_F64 = 78.6e12


def flops_per_point_adjoint_sets(d: int) -> int:
    return 4 * d


def uses_adjoint_sets(d: int, family: int, nsets: int) -> bool:
    return family in (0, 3) and d <= 64 and nsets >= 16


# MDI-LR factor evaluation (Gaussian): a run of nodes summed in Horner form from its
# last ratio down, h <- 1 + r h and r <- r / q: one FP64 FMA and one FP64 multiply per
# node (the exp2 seeds of each run of nodes are not counted).
WORK_PER_MDI_FACTOR = 2 * C64

# MDI-LR of g(sum x), power g, QMC_FP32_COMPENSATED, per merged-state evaluation of
# g (FP64 operations): the node and b + c s (2); the range test (1); log2 from the
# table (9: mantissa and exponent, t = m / T_j - 1, the three-step polynomial, the
# exponent converted and added, the last FMA; plus two 32-bit operations for the table
# index); the exponent -p log2 (1); the split exp2 (6: rounding, fraction, three
# conversions, ldexp; plus one v_exp_f32); the weighted add (1).
WORK_PER_SUM_EVAL = 20 * C64 + 2 * C32 + CT

# Lattice-quality criteria (FP64): per point and direction the index step, the
# conversion, x = k/n, y = x (1 - x), the factor 1 + a B(x) and the product; per
# point the "- 1" and the FP64 add.
def work_per_point_criterion(d: int) -> int:
    return d * (INDEX + 5 * C64) + 2 * C64


# CBC candidate evaluation, per (candidate, k): the residue update (modular add),
# the conversion, x, y, the factor, p(k) * factor - 1 and the FP64 add.
WORK_PER_CBC_TERM = INDEX + 6 * C64


# The improved rule's point set: one int32 grid rank written per point and
# direction (the generator is HBM-bound).  The order check that gives n* works
# per residue wrap, not per point (about n / z_d wraps).
IMPLR_BYTES_PER_POINT_DIM = 4


# The paper's own timings nearest to each workload, with their hardware: context for
# the numbers above, not a target (serial MATLAB on one Intel Xeon Gold 6226R at
# 2.90 GHz with 32 GB of RAM, Sec. 4; MDI-LR there builds symbolic functions).
_PAPER_HW = "MATLAB, one Intel Xeon Gold 6226R 2.90 GHz core, 32 GB (Sec. 4)"
_SLR = {"source": "Table 2-1, standard lattice rule, Gaussian of Test 3, d = 10, n = 1 + 10^10",
        "cpu_time_s": 13084.0, "points_per_s": (1 + 10 ** 10) / 13084.0,
        "point_dims_per_s": 10 * (1 + 10 ** 10) / 13084.0, "hardware": _PAPER_HW}
PAPER_CONTEXT = {
    "batched_4096": _SLR, "plain_d20_peak": _SLR, "plain_d4_expsum": _SLR, "plain_d20_f5": _SLR,
    "shifts_d20_peak": _SLR,
    "mdi_d100_gauss": {"source": "Table 2-3, MDI-LR, product peak of Test 5, a = N = 20, d = 100",
                       "cpu_time_s": 11.120, "factor_evals_per_s": 100 * 20 / 11.120,
                       "hardware": _PAPER_HW + "; symbolic sweeps"},
    "mdi_sum_d100": {"source": "Table 4-2 fits for Test 7's f_6 (CPU time ~ N^2 d^3); no single timing",
                     "hardware": _PAPER_HW},
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched_4096",
                    choices=["plain_d20_peak", "plain_d4_expsum", "plain_d20_f5", "mdi_d100_gauss", "batched_4096",
                             "adjoint_d50_osc", "shifts_d20_peak", "korobov_search_d20",
                             "cbc_d20", "mdi_sum_d100", "implr_d3", "rates", "timeline_d20_peak"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="one core's worth of oracle work in the CPU-baseline sample of a plain workload")
    ap.add_argument("--batched-stride", type=int, default=64,
                    help="the batched workload's CPU-baseline sample: every k-th integrand")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-form", action="store_true",
                    help="batched workload: leave out the comparison with the plain form (its 8192 "
                         "single-integrand launches); used for the rocprofv3 counter runs")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB three times "
                         "(the reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


# HBM traffic of a workload's dominant kernel as measured with rocprofv3 counters and
# recorded in its profile summary, together with a SHA-256 of the kernel's sources and
# of the build script (its compiler flags) at the time: reported only while they still
# match.
TRAFFIC = {
    "plain_d20_peak": ("lattice_sum_plain_d20_peak.md",
                       ["lattice_sum.hip", "tile.hpp", "common.hpp", "families.hpp", "exp2_f64.hpp", "kernels.hpp",
                        "../build.py"]),
    "batched_4096": ("batched_kernel_batched_4096.md",
                     ["batched.hip", "batched.hpp", "plan.hip", "tile.hpp", "common.hpp", "families.hpp", "exp2_f64.hpp",
                      "../build.py"]),
}


def kernel_sources_sha256(names) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2404_08867_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """Bytes per launch from the workload's profile summary, or None if absent or stale."""
    if workload not in TRAFFIC:
        return None
    profile, names = TRAFFIC[workload]
    try:
        with open(os.path.join(ROOT, "profiles", profile)) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for ln in text.splitlines():
        if ln.startswith("traffic_bytes_per_launch:") or ln.startswith("kernel_sources_sha256:"):
            k, v = ln.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256(names):
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(torch, mib):
    """A plain device copy of `mib` MiB, three times (counter calibration)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


# ---------------------------------------------------------------- CPU baseline
# The FP64 oracle is timed on the host cores of the machine running the benchmark:
# independent oracle calls (integrands, parameter sets, shifts, or index ranges of one
# sum through oracle.lattice_partial) run side by side in a thread pool -- the oracle's
# C functions release the interpreter lock, and each call stays single-threaded and
# literal -- and a smaller sample runs on one thread for the single-core figure.
MAX_POOL = 16  # worker threads: the CPU share of one GPU on a shared host


def cpu_info() -> dict:
    model, mhz = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if model is None and ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                if mhz is None and ln.startswith("cpu MHz"):
                    mhz = float(ln.split(":", 1)[1])
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model, "mhz": mhz}


def run_pool(calls, threads):
    """Run zero-argument callables on `threads` worker threads; (results, wall s)."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    if threads <= 1:
        out = [c() for c in calls]
    else:
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            out = list(ex.map(lambda c: c(), calls))
    return out, time.perf_counter() - t0


def cpu_baseline(unit, calls, units, single_calls, single_units, sample):
    """The oracle's rate on all usable cores (up to MAX_POOL) over `calls`, and on one
    core over `single_calls`; returns (cpu_baseline dict, results of `calls`)."""
    info = cpu_info()
    cores = max(1, min(info["usable"], MAX_POOL))
    res, wall = run_pool(calls, cores)
    _, wall1 = run_pool(single_calls, 1)
    return {"value": units / wall, "unit": unit, "cores": cores, "kind": "oracle", "sample": sample,
            "wall_s": wall, "single_core": {"value": single_units / wall1, "wall_s": wall1},
            "host": info}, res


def plain_partial_tasks(z, prob, reps, tasks):
    """`reps` full oracle sums over [0, n) as `tasks` callables: the sums are split into
    index ranges (oracle.lattice_partial) only when they are long, and each task runs
    its share of (range, repetition) items in a loop, so that tiny sums do not turn
    into millions of pool tasks."""
    import oracle as O
    pieces = tasks if prob.n >= (1 << 16) else 1
    edges = [prob.n * k // pieces for k in range(pieces + 1)]
    items = [(lo, hi) for _ in range(reps) for lo, hi in zip(edges[:-1], edges[1:]) if hi > lo]
    shares = [items[t::tasks] for t in range(tasks)]

    def run(share):
        for lo, hi in share:
            O.lattice_partial(z, prob.n, prob.family, prob.params, lo, hi - lo, prob.shift)
    return [(lambda sh=sh: run(sh)) for sh in shares if sh], pieces


def oracle_baseline(prob, seconds):
    """CPU-baseline leg of a plain workload: the whole sum repeated for about `seconds`
    of one core's work, spread over the host cores (index ranges of one sum for long
    sums, whole sums for short ones), and once on one core.  Returns (cpu_baseline
    dict, Q, A) with Q and A from the single-core run."""
    import oracle as O
    z = O.korobov(prob.d, prob.n, prob.a)
    t0 = time.perf_counter()
    q, a = O.lattice_sum(z, prob.n, prob.family, prob.params, prob.shift)
    t1 = time.perf_counter() - t0
    reps = max(1, int(seconds / max(t1, 1e-9)))
    cores = max(1, min(cpu_info()["usable"], MAX_POOL))
    calls, pieces = plain_partial_tasks(z, prob, reps, 4 * cores)
    single_reps = max(1, reps // 8)
    base, _ = cpu_baseline("lattice-point evals/s", calls, prob.n * reps,
                           [lambda: [O.lattice_sum(z, prob.n, prob.family, prob.params, prob.shift)
                                     for _ in range(single_reps)]], prob.n * single_reps,
                           f"the full sum (n={prob.n}) repeated {reps} times"
                           + (f", each split into {pieces} index ranges (oracle.lattice_partial)" if pieces > 1 else "")
                           + f", over the cores; single core: {single_reps} full sums")
    return base, q, a


def oracle_mdi_baseline(w):
    """Every parameter set's MDI-LR value by the oracle, the sets split over the host cores
    in chunks, and the first 2048 sets on one core.  Returns (cpu_baseline dict, values)."""
    import numpy as np
    import oracle as O
    nsets = len(w.params)
    cores = max(1, min(cpu_info()["usable"], MAX_POOL))
    chunks = np.array_split(np.arange(nsets), 8 * cores)

    N64 = np.ascontiguousarray(w.N, dtype=np.int64)  # converted once, not per call

    def run(idx):
        return [O.mdi_lr(N64, w.family, w.params[s]) for s in idx]
    calls = [(lambda idx=idx: run(idx)) for idx in chunks if len(idx)]
    single = min(2048, nsets)
    per_set = float(np.sum(w.N))
    base, res = cpu_baseline("factor evals/s", calls, per_set * nsets,
                             [lambda: run(range(single))], per_set * single,
                             f"all {nsets} parameter sets (d={w.d}, N={int(w.N[0])}), in {len(calls)} chunks "
                             f"over the cores (each set a short oracle call, so the interpreter's lock "
                             f"limits the speed-up); the first {single} on one core")
    return base, [v for part in res for v in part]


def time_graph(torch, launch, steps, warmup):
    """Eager warm-up, capture `steps` launches in one graph, replay it once timed."""
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    # single-call eager latency (host launch + kernel), median of 20
    lat = []
    for _ in range(20):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        launch()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(steps):
            launch()
    g.replay()  # untimed replay
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern = e0.elapsed_time(e1) * 1e-3
    return wall / steps, kern / steps, statistics.median(lat), g


def bench_plain(args, torch, qmc, W):
    prob = {"plain_d20_peak": W.plain_d20_peak, "plain_d4_expsum": W.plain_d4_expsum,
            "plain_d20_f5": W.plain_d20_f5}[args.workload]()
    z = torch.tensor(qmc.korobov(prob.d, prob.n, prob.a), device="cuda")
    params = torch.tensor(prob.params, dtype=torch.float64, device="cuda")
    ws = qmc.Workspace(qmc.workspace_size(prob.d, prob.n, 1))
    results = {}
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        out = torch.zeros(1, dtype=torch.float64, device="cuda")

        def launch(prec=prec, out=out):
            qmc.lattice_sum(z, prob.n, prob.family, params, prec, ws=ws, out=out)

        step_s, kern_s, lat_s, g = time_graph(torch, launch, args.steps, args.warmup)
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=lat_s, q=float(out.item()))
        del g
    units = prob.n
    wpp = work_per_point(prob.d, prob.family)
    results["fp32c"]["lane_ops"] = lane_ops_per_point(prob.d, prob.family)
    config = {"workload": prob.name, "d": prob.d, "n": prob.n, "a": prob.a,
              "family": W.FAMILY_NAMES[prob.family], "precision": "fp32_compensated",
              "lattice": "korobov", "shift": None}
    return prob, results, units, wpp, config


def bench_shifts(args, torch, qmc, W):
    """Random-shift ensemble: one step is the R = 64 shifted sums of plain_d20_peak
    and their mean and standard error (two launches)."""
    w = W.shifts_d20_peak()
    z = torch.tensor(qmc.korobov(w.d, w.n, w.a), device="cuda")
    params = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    shifts = torch.tensor(w.shifts, dtype=torch.float64, device="cuda")
    R = shifts.shape[0]
    ws = qmc.Workspace(qmc.workspace_size(w.d, w.n, R))
    results = {}
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        q = torch.zeros(R, dtype=torch.float64, device="cuda")
        stats = torch.zeros(2, dtype=torch.float64, device="cuda")

        def launch(prec=prec, q=q, stats=stats):
            qmc.lattice_sum_shifts(z, w.n, w.family, params, shifts, prec, ws=ws, out=q,
                                   stats_out=stats)

        step_s, kern_s, lat_s, g = time_graph(torch, launch, args.steps, args.warmup)
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=lat_s, q=q.cpu().numpy(),
                             stats=stats.cpu().numpy())
        del g
    units = w.n * R
    wpp = work_per_point(w.d, w.family)
    results["fp32c"]["lane_ops"] = lane_ops_per_point(w.d, w.family)
    config = {"workload": w.name, "d": w.d, "n": w.n, "a": w.a, "shifts": R,
              "family": W.FAMILY_NAMES[w.family], "precision": "fp32_compensated",
              "lattice": "korobov", "unit_of_work": "one point of one shifted lattice"}
    return w, results, units, wpp, config


def oracle_shifts_baseline(w, r32, r64):
    """All R shifted sums by the oracle, one shift per pool task over the host cores (the
    oracle is fast enough for the whole ensemble), and the first four on one core; the
    errors of every Q_r.  Returns (cpu_baseline dict, e32, e64)."""
    import oracle as O
    z = O.korobov(w.d, w.n, w.a)
    R = w.shifts.shape[0]
    calls = [(lambda r=r: O.lattice_sum(z, w.n, w.family, w.params, w.shifts[r])) for r in range(R)]
    single = min(4, R)
    base, res = cpu_baseline("shifted-lattice point evals/s", calls, w.n * R, calls[:single], w.n * single,
                             f"all {R} shifted sums (n={w.n} points each), one per task over the cores; "
                             f"the first {single} on one core")
    e32 = max(abs(r32["q"][r] - qo) / max(abs(qo), ao) for r, (qo, ao) in enumerate(res))
    e64 = max(abs(r64["q"][r] - qo) / max(abs(qo), ao) for r, (qo, ao) in enumerate(res))
    return base, e32, e64


def bench_mdi_sum(args, torch, qmc, W):
    """MDI-LR of g(sum x): one step is the state iteration and the evaluation of
    all 4096 parameter sets (two launches)."""
    w = W.mdi_sum_d100()
    params = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    nsets = params.shape[0]
    ws = qmc.Workspace(qmc.mdi_lr_sum_workspace_size(w.d, w.N))
    results = {}
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        out = torch.zeros(nsets, dtype=torch.float64, device="cuda")

        def launch(prec=prec, out=out):
            qmc.mdi_lr_sum(w.d, w.N, w.N_last, w.gfamily, params, prec, ws=ws, out=out)

        step_s, kern_s, lat_s, g = time_graph(torch, launch, args.steps, args.warmup)
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=lat_s, q=out.cpu().numpy())
        del g
    merge = w.N_last == w.N
    states = (w.d if merge else w.d - 1) * (w.N - 1) + 1
    units = nsets * states * (1 if merge else w.N_last)
    config = {"workload": w.name, "d": w.d, "N": w.N, "N_last": w.N_last, "nsets": nsets,
              "family": "sum_power (set 0: f_6 = (1 + sum x)^-(d+1))", "precision": "fp32_compensated",
              "merged_states": states, "tensor_grid_points": f"{w.N}^{w.d}",
              "sets_per_s": nsets / results["fp32c"]["step_s"],
              "unit_of_work": "one evaluation of g at a merged state"}
    return w, results, units, WORK_PER_SUM_EVAL, config


def oracle_mdi_sum_baseline(w, r32, r64, seconds):
    import oracle as O
    t0 = time.perf_counter()
    e32 = e64 = 0.0
    k = 0
    for s in range(len(w.params)):
        qo = O.mdi_sum(w.d, w.N, w.N_last, w.gfamily, w.params[s])
        e32 = max(e32, abs(r32["q"][s] - qo) / abs(qo))
        e64 = max(e64, abs(r64["q"][s] - qo) / abs(qo))
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    states = (w.d - 1) * (w.N - 1) + 1  # the oracle evaluates g at (state, last node) pairs
    return states * w.N_last * k / dt, k, e32, e64


def bench_search(args, torch, qmc, W):
    """Korobov search: one step is the whole search over a in [1, (n-1)/2]."""
    w = W.korobov_search_d20()
    ws = qmc.Workspace(qmc.criteria_workspace_size(w.d, w.n))
    holder = {}

    def launch():
        holder["r"] = qmc.korobov_search(w.d, w.n, gamma=w.gamma, beta=w.beta, a0=w.a0, count=w.count, ws=ws)

    step_s, kern_s = time_eager(torch, launch, args.steps, args.warmup)
    vals, best = holder["r"]
    r = dict(step_s=step_s, kern_s=kern_s, lat_s=step_s, q=vals.cpu().numpy(), best=best.cpu().numpy())
    # distinct points per candidate: points i and n - i are mirror images with equal
    # Bernoulli products, so a criterion has n // 2 + 1 distinct terms
    units = w.count * (w.n // 2 + 1)
    config = {"workload": w.name, "d": w.d, "n": w.n,
              "criterion": "e^2 (eq. 2.12), gamma_j = j^-2, beta = 0",
              "candidates": w.count, "best_a": int(r["best"][1]), "best_e2": float(r["best"][0]),
              "precision": "fp64",
              "unit_of_work": "one distinct d-dimensional lattice point of one candidate (i and n - i are one)"}
    return w, {"fp32c": r, "fp64": r}, units, work_per_point_criterion(w.d), config


def bench_cbc(args, torch, qmc, W):
    """CBC: one step is the whole d-component construction."""
    w = W.cbc_d20()
    ws = qmc.Workspace(qmc.criteria_workspace_size(w.d, w.n))
    holder = {}

    def launch():
        holder["r"] = qmc.cbc(w.d, w.n, w.gamma, w.beta, ws=ws)

    step_s, kern_s = time_eager(torch, launch, args.steps, args.warmup)
    z, e2 = holder["r"]
    r = dict(step_s=step_s, kern_s=kern_s, lat_s=step_s, z=z.cpu().numpy(), q=e2.cpu().numpy())
    # distinct (candidate, k) terms over all components: k and n - k give the same
    # term, so a candidate's criterion has n // 2 + 1 of them
    units = (1 + (w.d - 1) * (w.n // 2)) * (w.n // 2 + 1)
    config = {"workload": w.name, "d": w.d, "n": w.n, "criterion": "e^2 (eq. 2.12), gamma_j = j^-2, beta = 0",
              "z": [int(v) for v in r["z"]], "e2_final": float(r["q"][-1]), "precision": "fp64",
              "unit_of_work": "one distinct (candidate, lattice index) term (k and n - k are one term)"}
    return w, {"fp32c": r, "fp64": r}, units, WORK_PER_CBC_TERM, config


def bench_implr(args, torch, qmc, W):
    """Theorem 3.1's transformed point set: one step writes the grid ranks of all n
    lattice points (qmc_implr_points, the dominant kernel, HBM-bound) and counts
    the added points n* exactly (qmc_implr_grid, order check)."""
    w = W.implr_d3()
    ws = qmc.Workspace(qmc.implr_workspace_size(w.d, w.n, w.a))
    nstar = torch.empty(1, dtype=torch.int64, device="cuda")
    pts = torch.empty((w.d, (w.n + 63) // 64 * 64), dtype=torch.int32, device="cuda")  # rows 256-byte aligned
    holder = {}

    def gen():
        qmc.implr_points(w.d, w.n, w.a, 0, w.n, out=pts)

    def count():
        holder["counts"], _ = qmc.implr_grid(w.d, w.n, w.a, qmc.IMPLR_AUTO, ws=ws, out=nstar)

    for _ in range(args.warmup):
        gen()
        count()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e in ev:
        e[0].record()
        gen()
        e[1].record()
        count()
        e[2].record()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    gen_s = sum(e[0].elapsed_time(e[1]) for e in ev) * 1e-3 / args.steps
    cnt_s = sum(e[1].elapsed_time(e[2]) for e in ev) * 1e-3 / args.steps
    bytes_written = w.n * w.d * IMPLR_BYTES_PER_POINT_DIM
    wpp = w.d * IMPLR_BYTES_PER_POINT_DIM  # bytes per point
    roofline = {"bound": "hbm", "achieved": bytes_written / gen_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                "frac": bytes_written / gen_s / 8.0e12, "traffic": None,
                "kernel": "implr_points_kernel", "bytes_per_launch": bytes_written,
                "kernel_us": gen_s * 1e6}
    wraps = sum((w.n - 1) * w.a ** i // w.n for i in range(w.d))  # residue i wraps about z_i times
    check = {"us": cnt_s * 1e6, "pairs_verified": w.n - 1, "residue_wraps": wraps,
             "launches": 6, "note": "order kernel plus five launches that exit at once"}
    r = dict(step_s=step_s, kern_s=gen_s + cnt_s, lat_s=step_s, nstar=int(nstar.item()),
             counts=[int(c) for c in holder["counts"]], roofline=roofline, pts=pts)
    config = {"workload": w.name, "d": w.d, "n": w.n, "a": w.a, "counts": r["counts"],
              "grid": int(np.prod(r["counts"])), "nstar": r["nstar"], "precision": "integer",
              "unit_of_work": "one lattice point mapped to its grid ranks (written) and checked",
              "nstar_order_check": check}
    return w, {"fp32c": r, "fp64": r}, w.n, wpp, config


def oracle_implr_baseline(w, qmc, res, seconds):
    """The oracle's transformed coordinates of consecutive blocks of lattice points
    until the time budget is spent (its n* needs every point in memory, which this
    size does not allow); the GPU's n* is checked against prod(n_i) - n and sampled
    GPU points against the oracle."""
    import oracle as O
    z = O.korobov(w.d, w.n, w.a)
    exact = res["nstar"] == int(np.prod(O.mdi_dims(z, w.n))) - w.n
    pts = res.pop("pts")
    for j0 in (0, 12345678, w.n // 2, w.n - 4096):
        s = pts[:, j0:j0 + 4096].cpu().numpy().astype(np.int64).T
        exact = exact and bool(np.array_equal(s * z, O.implr_coords_at(z, w.n, np.arange(j0, j0 + 4096))))
    del pts
    block = 1 << 20
    t0 = time.perf_counter()
    k = 0
    while k == 0 or time.perf_counter() - t0 < seconds:
        O.implr_coords_at(z, w.n, np.arange(k * block, (k + 1) * block))
        k += 1
    dt = time.perf_counter() - t0
    return block * k / dt, k, 0.0 if exact else 1.0


def _wce2_with_scale(O, z, w):
    """Oracle e^2 and the scale C * A of its terms (A: mean |term| of the sum S)."""
    g = np.asarray(w.gamma[: len(z)])
    c = float(np.prod(1.0 + g * w.beta))
    _, a_scale = O.lattice_kernel_sum(z, w.n, 2, g / (1.0 + g * w.beta))
    return O.shift_avg_wce2(z, w.n, g, w.beta), c * a_scale


def oracle_search_baseline(w, vals, seconds):
    """The oracle's e^2 of the first candidates until the time budget is spent (the
    rate counts the oracle's own evaluation); the error uses the mixed-sign measure."""
    import oracle as O
    t0 = time.perf_counter()
    k = 0
    for i in range(w.count):
        O.shift_avg_wce2(O.korobov(w.d, w.n, w.a0 + i), w.n, w.gamma, w.beta)
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    err = 0.0
    for i in range(min(k, 64)):
        eo, scale = _wce2_with_scale(O, O.korobov(w.d, w.n, w.a0 + i), w)
        err = max(err, abs(vals[i] - eo) / max(abs(eo), scale))
    return (w.n // 2 + 1) * k / dt, k, err


def oracle_cbc_baseline(w, res, seconds):
    """The oracle's criterion for the first candidates of the second component, and
    the relative error of every component's criterion at the GPU's choices."""
    import oracle as O
    z, e2 = res["z"], res["q"]
    err = 0.0
    for j in range(w.d):
        eo, scale = _wce2_with_scale(O, z[: j + 1], w)
        err = max(err, abs(e2[j] - eo) / max(abs(eo), scale))
    t0 = time.perf_counter()
    k = 0
    for c in range(1, w.n // 2 + 1):
        O.shift_avg_wce2([1, c], w.n, w.gamma[:2], w.beta)
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return (w.n // 2 + 1) * k / dt, k, err


def gaussian_integral(c, w):
    """Exact integral over [0,1]^d of exp(-sum_j c_j^2 (x_j - w_j)^2)."""
    out = 1.0
    for cj, wj in zip(c, w):
        out *= math.sqrt(math.pi) / (2 * cj) * (math.erf(cj * (1 - wj)) + math.erf(cj * wj))
    return out


def mdi_beside_plain_rule(torch, qmc, W, w, results):
    """Set 0 of the MDI-LR launch and the plain rule on the same Gaussian (n = 1048573,
    seeded a), both against the exact integral (outside the timed region)."""
    pr = W.mdi_d100_gauss_plain_rule()
    exact = gaussian_integral(pr.params[:pr.d], pr.params[pr.d:])
    z = torch.tensor(qmc.korobov(pr.d, pr.n, pr.a), device="cuda")
    params = torch.tensor(pr.params, dtype=torch.float64, device="cuda")
    out = {"exact_integral": exact, "mdi_lr": {"N": int(w.N[0]), "nodes": f"{int(w.N[0])}^{w.d}"},
           "plain_rule": {"n": pr.n, "a": pr.a}}
    for name, prec in (("fp32c", qmc.FP32_COMPENSATED), ("fp64", qmc.FP64)):
        out["mdi_lr"][f"rel_err_{name}"] = float(results[name]["q"][0]) / exact - 1
        q = float(qmc.lattice_sum(z, pr.n, pr.family, params, prec).item())
        out["plain_rule"][f"rel_err_{name}"] = q / exact - 1
    return out


def bench_mdi(args, torch, qmc, W):
    nsets = 65536
    w = W.mdi_d100_gauss(nsets=nsets)
    N = torch.tensor(w.N.astype("int32"), device="cuda")
    params = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    results = {}
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        out = torch.zeros(nsets, dtype=torch.float64, device="cuda")

        def launch(prec=prec, out=out):
            qmc.mdi_lr(N, w.family, params, prec, out=out)

        step_s, kern_s, lat_s, g = time_graph(torch, launch, args.steps, args.warmup)
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=lat_s, q=out.cpu().numpy())
        del g
    units = int(w.N.sum()) * nsets  # one-dimensional factor evaluations per launch
    wpp = WORK_PER_MDI_FACTOR
    results["fp32c"]["lane_ops"] = LANE_OPS_PER_MDI_FACTOR
    results["vs_plain_rule"] = mdi_beside_plain_rule(torch, qmc, W, w, results)
    config = {"workload": w.name, "d": w.d, "N": int(w.N[0]), "nsets": nsets,
              "family": W.FAMILY_NAMES[w.family], "precision": "fp32_compensated",
              "unit_of_work": "one-dimensional factor evaluation"}
    return w, results, units, wpp, config


def time_eager(torch, launch, steps, warmup):
    """For launches much longer than their launch overhead: W eager warm-ups, then
    K eager launches between two synchronisations, HIP events around them."""
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, e0.elapsed_time(e1) * 1e-3 / steps


def bench_batched(args, torch, qmc, W):
    batch = W.batched_4096()
    units = sum(p.n for p in batch.problems)
    wpp = sum(p.n * work_per_point(p.d, p.family) for p in batch.problems) / units
    results = {}
    tuned = None
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        plan = qmc.BatchPlan.from_batch(batch, prec, config=tuned)
        out = torch.zeros(plan.count, dtype=torch.float64, device="cuda")
        if tuned is None:
            tuned = plan.autotune(reps=1, out=out)
        step_s, kern_s = time_eager(torch, lambda: plan.run(out=out), args.steps, args.warmup)
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=step_s, q=out.cpu().numpy())
        del plan
    results["fp32c"]["lane_ops"] = sum(p.n * lane_ops_per_point(p.d, p.family) for p in batch.problems) / units
    if not args.no_plain_form:
        results["plain_per_integrand"] = plain_per_integrand(torch, qmc, batch, results)
    config = {"workload": batch.name, "integrands": len(batch.problems), "points": units,
              "point_dims": int(sum(p.n * p.d for p in batch.problems)),
              "families": "exp_sum/product_peak/gaussian", "precision": "fp32_compensated",
              "schedule": dict(tuned)}
    return batch, results, units, wpp, config


def plain_per_integrand(torch, qmc, batch, results):
    """The same integrands as one plain-rule launch each (qmc_lattice_sum), the 4096
    launches captured in one HIP graph and replayed (the plain form's best case: no host
    work between launches), in FP64 and FP32c: the time per pass over the whole batch,
    and the batched launch's speed-up over it."""
    probs = batch.problems
    zs = [torch.tensor(qmc.korobov(p.d, p.n, p.a), device="cuda") for p in probs]
    ps = [torch.tensor(p.params, dtype=torch.float64, device="cuda") for p in probs]
    ws = qmc.Workspace(qmc.workspace_size(max(p.d for p in probs), max(p.n for p in probs), 1))
    out = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    res = {}
    for prec, name in ((qmc.FP64, "fp64"), (qmc.FP32_COMPENSATED, "fp32c")):
        def one_pass(prec=prec):
            for b, p in enumerate(probs):
                qmc.lattice_sum(zs[b], p.n, p.family, ps[b], prec, ws=ws, out=out[b:b + 1])
        one_pass()  # eager warm-up
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            one_pass()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = e0.elapsed_time(e1)
        del g
    res["launches"] = len(probs)
    res["batched_fp32c_speedup_over_plain_fp64"] = res["fp64_ms"] / (results["fp32c"]["kern_s"] * 1e3)
    res["batched_fp32c_speedup_over_plain_fp32c"] = res["fp32c_ms"] / (results["fp32c"]["kern_s"] * 1e3)
    return res


def bench_adjoint(args, torch, qmc, W):
    w = W.adjoint_d50_osc()
    z = torch.tensor(qmc.korobov(w.d, w.n, w.a), device="cuda")
    params = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    nsets = params.shape[0]
    ws = qmc.Workspace(qmc.workspace_size(w.d, w.n, nsets))
    results = {}
    for prec, name in ((qmc.FP32_COMPENSATED, "fp32c"), (qmc.FP64, "fp64")):
        holder = {}

        def launch(prec=prec):
            holder["r"] = qmc.lattice_sum_adjoint(z, w.n, w.family, params, prec, ws=ws)

        step_s, kern_s = time_eager(torch, launch, args.steps, args.warmup)
        q, g = holder["r"]
        results[name] = dict(step_s=step_s, kern_s=kern_s, lat_s=step_s, q=q.cpu().numpy(),
                             g=g.cpu().numpy())
    units = w.n * nsets  # point-set evaluations of f and all its parameter derivatives
    wpp = work_per_point_adjoint(w.d, w.family)
    if uses_adjoint_sets(w.d, w.family, nsets):
        fpp = flops_per_point_adjoint_sets(w.d)
        kern = results["fp32c"]["kern_s"]
        results["fp32c"]["roofline"] = {
            "bound": "mfma", "achieved": fpp * units / kern / 1e12, "peak": PEAK_MFMA_F64 / 1e12,
            "unit": "TFLOP/s (FP64 matrix)", "frac": fpp * units / kern / PEAK_MFMA_F64, "traffic": None,
            "kernel": "adjoint_sets_kernel", "flops_per_unit": fpp, "kernel_us": kern * 1e6}
    config = {"workload": w.name, "d": w.d, "n": w.n, "nsets": nsets, "a": w.a,
              "family": W.FAMILY_NAMES[w.family], "precision": "fp32_compensated",
              "unit_of_work": "one point of one parameter set, value and full gradient"}
    return w, results, units, wpp, config


BATCHED_ORACLE = os.path.join(ROOT, "tests", "golden", "batched_4096_oracle.json")


def oracle_batched_baseline(batch, qs32, qs64, stride):
    """Errors of every GPU result against the oracle's, cached by
    tests/golden/make_oracle_cache.py (oracle only), and the oracle timed on every
    `stride`-th integrand over the host cores (every 8 * stride-th on one core); the
    sample's fresh oracle values must equal the cached ones."""
    import oracle as O
    with open(BATCHED_ORACLE) as f:
        ref = json.load(f)
    probs = batch.problems
    if ref["n"] != [p.n for p in probs] or ref["a"] != [p.a for p in probs]:
        raise RuntimeError(f"{BATCHED_ORACLE} does not describe this workload: rerun make_oracle_cache.py")
    qo, ao = np.array(ref["q"]), np.array(ref["abs_mean"])
    scale = np.maximum(np.abs(qo), ao)
    err32 = np.abs(np.asarray(qs32) - qo) / scale
    err64 = np.abs(np.asarray(qs64) - qo) / scale

    def call(p):
        return lambda: O.lattice_sum(O.korobov(p.d, p.n, p.a), p.n, p.family, p.params)[0]

    sample = list(range(0, len(probs), stride))
    single = sample[::8]
    base, fresh = cpu_baseline("lattice-point evals/s", [call(probs[i]) for i in sample],
                               sum(probs[i].n for i in sample), [call(probs[i]) for i in single],
                               sum(probs[i].n for i in single),
                               f"integrands 0, {stride}, 2*{stride}, ... ({len(sample)} of {len(probs)}, "
                               f"{sum(probs[i].n * probs[i].d for i in sample):.3g} point-dims) over the cores; "
                               f"every {8 * stride}-th ({len(single)}) on one core")
    if any(fresh[k] != qo[i] for k, i in enumerate(sample)):
        raise RuntimeError("the oracle's cached values differ from a fresh oracle run")
    worst = int(np.argmax(err32))
    errs = {"max_fp32c": float(err32[worst]), "median_fp32c": float(np.median(err32)),
            "worst_integrand": {"index": worst, "family": W_FAMILY.get(probs[worst].family),
                                "d": probs[worst].d, "n": probs[worst].n},
            "max_fp64": float(np.max(err64)), "integrands_checked": len(probs)}
    return base, errs


ADJOINT_ORACLE = os.path.join(ROOT, "tests", "golden", "adjoint_d50_osc_oracle.json")


def oracle_adjoint_baseline(w, r32, r64):
    """Errors of every set's value and gradient against the oracle's cached values
    (tests/golden/make_oracle_cache.py, oracle only), and the oracle timed on set 0 on
    one core (value and gradient over all n points); the fresh set-0 values must equal
    the cached ones.  Value errors are relative to max(|Q_o|, A), gradient errors to the
    largest |component|.  Returns (rate, e32, e64)."""
    import numpy as np
    import oracle as O
    with open(ADJOINT_ORACLE) as f:
        ref = json.load(f)
    if (ref["d"], ref["n"], ref["a"], ref["nsets"]) != (w.d, w.n, w.a, w.params.shape[0]):
        raise RuntimeError(f"{ADJOINT_ORACLE} does not describe this workload: rerun make_oracle_cache.py")
    z = O.korobov(w.d, w.n, w.a)
    t0 = time.perf_counter()
    qo, go = O.lattice_grad(z, w.n, w.family, w.params[0])
    dt = time.perf_counter() - t0
    if qo != ref["q"][0] or not np.array_equal(np.asarray(go), np.asarray(ref["grad"][0])):
        raise RuntimeError("the oracle's cached adjoint values differ from a fresh oracle run")
    errs = []
    for r in (r32, r64):
        e = 0.0
        for s in range(w.params.shape[0]):
            gs = np.asarray(ref["grad"][s])
            scale = max(float(np.max(np.abs(gs))), 1e-300)
            e = max(e, abs(r["q"][s] - ref["q"][s]) / max(abs(ref["q"][s]), ref["abs_mean"][s]),
                    float(np.max(np.abs(r["g"][s] - gs))) / scale)
        errs.append(e)
    return w.n / dt, errs[0], errs[1]


# ---------------------------------------------------------------- issue-rate probe
# paper_2404_08867_amd/probe/issue_rates.hip (libqmc_probe.so): lane-operations per second
# of each instruction type on the lattice path, alone and mixed, over 8 workgroups of 256
# threads per CU with 8 independent chains per thread.  The ceiling the ALU rooflines use,
# 256 CUs x 64 lanes x 2.4 GHz, and the transcendental costs rest on these figures.
PROBE_KINDS = ["u32_add", "index_step(add,add,min)", "f32_fma", "f64_fma", "f64_add", "cvt_f64_u32",
               "cvt_f32_u32", "exp2_f32", "rcp_f32", "cos_f32", "log2_f32", "f64_fma x4 + exp2_f32",
               "u32_add + f64_fma", "point_dim(index step, cvt_f64_u32, f64_fma)", "u32_min", "u32_sub",
               "sub + cmp + cndmask", "f32_add", "f32_mul", "float_step(f32 add x2, u32 min)",
               "u32_add + f32_fma", "f32_fma + f64_fma", "f32_fma x4 + exp2_f32",
               "peak_dim(float step, f32 fma x2, f32 mul)", "cvt_f64_f32",
               "point_dim_float(float step, cvt_f64_f32, f64_fma)",
               "gauss_dim(index step, cvt_f64_u32, f64_fma x2)",
               "gauss_dim_float(float step, cvt_f64_f32, f64_fma x2)", "f64_mul",
               "horner(f64 fma + mul)", "horner, 2 chains per thread(f64 fma + mul)"]
PROBE_MAIN = "point_dim(index step, cvt_f64_u32, f64_fma)"
LANE_RATE = 256 * 64 * 2.4e9  # one VALU lane-operation per lane per clock


TIMELINE_MODES = {0: "whole kernel", 1: "empty kernel on the same grid",
                  2: "setup, workgroup total and grid sum, no tiles"}
CLOCK_HZ = 100e6  # the constant clock that wall_clock64() (s_memrealtime) reads on gfx950


def bench_timeline(args, torch, qmc, W):
    """Phase timeline of the plain_d20_peak launch (FP32c) from the probe copy of the
    plain-sum kernel (probe/plain_timeline.hip), beside the library's own launch: when
    the last workgroup starts, how long the setup, the tiles and the grid sum take, and
    the launch time of the empty kernel and of the fixed part without the tiles."""
    import ctypes
    import numpy as np
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2404_08867_amd", "libqmc_probe.so"))
    lib.qmc_probe_plain_timeline.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]
    lib.qmc_probe_timeline_workgroups.argtypes = [ctypes.c_uint32]
    w = W.plain_d20_peak()
    z = torch.tensor(qmc.korobov(w.d, w.n, w.a), device="cuda")
    params = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    ws = qmc.Workspace(qmc.workspace_size(w.d, w.n, 1))
    q_lib = torch.zeros(1, dtype=torch.float64, device="cuda")
    q_probe = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = lib.qmc_probe_timeline_workgroups(w.n)
    KM = lib.qmc_probe_timeline_marks()
    marks = torch.zeros(G * KM, dtype=torch.int64, device="cuda")

    def lib_launch():
        qmc.lattice_sum(z, w.n, w.family, params, qmc.FP32_COMPENSATED, ws=ws, out=q_lib)

    _, lib_kern, _, g = time_graph(torch, lib_launch, args.steps, args.warmup)
    del g
    line = {"metric": "phases of the plain-sum launch (probe copy of the kernel)",
            "value": lib_kern * 1e6, "unit": "us per launch (library kernel)", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": lib_kern * 1e3,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32",
            "data": "synthetic",
            "config": {"workload": "timeline_d20_peak", "d": w.d, "n": w.n, "family": "product_peak",
                       "precision": "fp32_compensated", "workgroups": G, "threads": 1024,
                       "points_per_thread": 4, "clock_hz": CLOCK_HZ},
            "modes": {}}
    for mode, name in TIMELINE_MODES.items():
        def launch(mode=mode):
            rc = lib.qmc_probe_plain_timeline(mode, w.d, w.n, ctypes.c_void_p(z.data_ptr()),
                                              ctypes.c_void_p(params.data_ptr()),
                                              ctypes.c_void_p(q_probe.data_ptr()),
                                              ctypes.c_void_p(marks.data_ptr()), ctypes.c_void_p(ws.ptr),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            if rc != G:
                raise RuntimeError(f"qmc_probe_plain_timeline(mode {mode}) returned {rc}")
        _, kern, _, g = time_graph(torch, launch, args.steps, args.warmup)
        del g
        # phases of single launches (the medians over `reps` launches of each figure)
        reps = 9
        figs = []
        for _ in range(reps):
            marks.zero_()
            torch.cuda.synchronize()
            launch()
            torch.cuda.synchronize()
            a = marks.view(G, KM).cpu().numpy().astype(np.float64)
            us = (a - a[:, 0].min()) / CLOCK_HZ * 1e6
            f = {"last_workgroup_start_us": us[:, 0].max(), "kernel_end_us": us[:, 19].max()}
            if mode != 1:
                tile_end = us[:, 2:18].max(axis=1)
                f.update({"setup_us_median": float(np.median(us[:, 1] - us[:, 0])),
                          "setup_end_us_max": us[:, 1].max(),
                          "wave0_tiles_end_us_median": float(np.median(us[:, 2])),
                          "tiles_end_us_median": float(np.median(tile_end)),
                          "tiles_end_us_max": tile_end.max(),
                          "workgroup_total_us_max": us[:, 18].max(),
                          "grid_sum_after_last_total_us": us[:, 19].max() - us[:, 18].max()})
                assert int(a[:, 20].sum()) == 1, "exactly one workgroup produces the total"
            figs.append(f)
        med = {k: round(float(np.median([f[k] for f in figs])), 3) for k in figs[0]}
        line["modes"][name] = {"us_per_launch": round(kern * 1e6, 3), "phases": med}
        if mode == 0:
            line["bits_equal_to_library"] = bool(torch.equal(q_probe, q_lib))
    print(json.dumps(line), flush=True)


def bench_rates(args, torch):
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2404_08867_amd", "libqmc_probe.so"))
    lib.qmc_probe_lane_ops.restype = ctypes.c_double
    lib.qmc_probe_lane_ops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.qmc_probe_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.qmc_probe_kinds() == len(PROBE_KINDS)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks, iters = 8 * cus, 256
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rates = {}
    for k, name in enumerate(PROBE_KINDS):
        def launch(k=k):
            rc = lib.qmc_probe_launch(k, blocks, iters, ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(stream.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"qmc_probe_launch({k}) returned {rc}")
        for _ in range(max(1, args.warmup)):
            launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            launch()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / args.steps
        ops = lib.qmc_probe_lane_ops(k, blocks, iters)
        rates[name] = {"lane_ops_per_s": ops / t, "vs_lane_rate": ops / t / LANE_RATE, "launch_us": t * 1e6}
    main = rates[PROBE_MAIN]
    line = {"metric": "VALU lane-operation issue rate of the point-and-direction loop (probe)",
            "value": main["lane_ops_per_s"], "unit": "lane-ops/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": main["launch_us"] * 1e-3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32/f64", "data": "synthetic",
            "config": {"workload": "rates", "workgroups": blocks, "threads": 256, "chains_per_thread": 8,
                       "cus": cus},
            "roofline": {"bound": "alu", "achieved": main["lane_ops_per_s"] / 1e12, "peak": LANE_RATE / 1e12,
                         "unit": "T VALU lane-ops/s", "frac": main["vs_lane_rate"], "traffic": None},
            "rates": rates}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding the lattice over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2404_08867_amd import qmc
    from paper_2404_08867_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "rates":
        bench_rates(args, torch)
        return
    if args.workload == "timeline_d20_peak":
        bench_timeline(args, torch, qmc, W)
        return
    qmc.lib()  # fail loudly if the HIP library is missing
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)

    if args.workload == "mdi_d100_gauss":
        prob, res, units, wpp, config = bench_mdi(args, torch, qmc, W)
    elif args.workload == "batched_4096":
        prob, res, units, wpp, config = bench_batched(args, torch, qmc, W)
    elif args.workload == "adjoint_d50_osc":
        prob, res, units, wpp, config = bench_adjoint(args, torch, qmc, W)
    elif args.workload == "shifts_d20_peak":
        prob, res, units, wpp, config = bench_shifts(args, torch, qmc, W)
    elif args.workload == "korobov_search_d20":
        prob, res, units, wpp, config = bench_search(args, torch, qmc, W)
    elif args.workload == "cbc_d20":
        prob, res, units, wpp, config = bench_cbc(args, torch, qmc, W)
    elif args.workload == "mdi_sum_d100":
        prob, res, units, wpp, config = bench_mdi_sum(args, torch, qmc, W)
    elif args.workload == "implr_d3":
        prob, res, units, wpp, config = bench_implr(args, torch, qmc, W)
    else:
        prob, res, units, wpp, config = bench_plain(args, torch, qmc, W)

    line = {"metric": METRIC}
    main_r = res["fp32c"]
    if args.no_cpu_baseline:
        main_r.pop("pts", None)  # the f4 point set is kept only for the oracle's spot checks
    value = units / main_r["step_s"]
    achieved = wpp * units / main_r["kern_s"]  # slots per second, measured costs
    lane_ops = main_r.get("lane_ops")
    if lane_ops is not None:
        roofline = {"bound": "alu", "achieved": lane_ops * units / main_r["kern_s"] / 1e12,
                    "peak": PEAK_SLOTS / 1e12, "unit": "T 32-bit VALU lane-op slots/s",
                    "frac": lane_ops * units / main_r["kern_s"] / PEAK_SLOTS,
                    "traffic": measured_traffic(args.workload), "work_per_unit": lane_ops,
                    "kernel_us": main_r["kern_s"] * 1e6,
                    "measured_costs": {"work_per_unit": wpp, "achieved": achieved / 1e12,
                                       "frac": achieved / PEAK_SLOTS}}
    else:
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                    "unit": "T 32-bit VALU lane-op slots/s", "frac": achieved / PEAK_SLOTS,
                    "traffic": measured_traffic(args.workload), "work_per_unit": wpp,
                    "kernel_us": main_r["kern_s"] * 1e6}
    line.update({
        "value": value,
        "unit": {"mdi_d100_gauss": "factor evals/s",
                 "adjoint_d50_osc": "point-set evals (value + gradient)/s",
                 "shifts_d20_peak": "shifted-lattice point evals/s",
                 "korobov_search_d20": "distinct candidate lattice-point evals/s",
                 "cbc_d20": "distinct candidate-index terms/s",
                 "mdi_sum_d100": "merged-state evaluations of g/s",
                 "implr_d3": "lattice points mapped to the grid and checked/s"}.get(
                     args.workload, "lattice-point evals/s"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["step_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # QMC_FP32_COMPENSATED: FP64 arguments and sums, FP32 transcendentals (and
        # product-peak factors where their error allows)
        "dtype": {"korobov_search_d20": "f64", "cbc_d20": "f64", "implr_d3": "u32"}.get(args.workload, "f64/f32"),
        "data": "synthetic",
        "config": config,
        "roofline": main_r.get("roofline") or roofline,
        "eager_latency_us": main_r["lat_s"] * 1e6,
        "fp64": {"value": units / res["fp64"]["step_s"], "ms_per_step": res["fp64"]["step_s"] * 1e3,
                 "kernel_us": res["fp64"]["kern_s"] * 1e6},
        # how much the QMC_FP32_COMPENSATED path gains over QMC_FP64 on this workload
        "fp32c_speedup_over_fp64": res["fp64"]["step_s"] / main_r["step_s"],
        "paper_context": PAPER_CONTEXT.get(args.workload),
    })
    if "vs_plain_rule" in res:
        line["vs_plain_rule"] = res["vs_plain_rule"]
    if "plain_per_integrand" in res:
        line["plain_per_integrand"] = res["plain_per_integrand"]

    if not args.no_cpu_baseline:
        base = None
        if args.workload == "batched_4096":
            base, errs = oracle_batched_baseline(prob, res["fp32c"]["q"], res["fp64"]["q"], args.batched_stride)
            e32, e64 = errs["max_fp32c"], errs["max_fp64"]
            line["errors_all_integrands"] = errs
        elif args.workload == "adjoint_d50_osc":
            rate, e32, e64 = oracle_adjoint_baseline(prob, res["fp32c"], res["fp64"])
            sample = ("parameter set 0 of 64 on one core, all n points, value and 51 gradient "
                      "components; rel_err over all 64 sets against the oracle's cached values")
        elif args.workload == "korobov_search_d20":
            rate, k, e32 = oracle_search_baseline(prob, res["fp64"]["q"], args.cpu_seconds)
            e64 = e32
            sample = (f"e^2 of the first {k} of {prob.count} candidates (the oracle sums all "
                      f"n={prob.n} points, {prob.n // 2 + 1} distinct); rel_err over the first {min(k, 64)}")
        elif args.workload == "cbc_d20":
            rate, k, e32 = oracle_cbc_baseline(prob, res["fp64"], args.cpu_seconds)
            e64 = e32
            sample = (f"the criterion of the first {k} candidates of the second component "
                      f"(the oracle sums all n={prob.n} terms, {prob.n // 2 + 1} distinct); "
                      f"rel_err over the {prob.d} chosen components")
        elif args.workload == "implr_d3":
            rate, k, e32 = oracle_implr_baseline(prob, qmc, res["fp64"], args.cpu_seconds)
            e64 = e32
            sample = (f"the oracle's transformed coordinates of the first {k} blocks of 2^20 lattice "
                      "points (its n* needs every point in memory); rel_err 0: n* and 16384 sampled "
                      "GPU points exact")
        elif args.workload == "mdi_sum_d100":
            rate, k, e32, e64 = oracle_mdi_sum_baseline(prob, res["fp32c"], res["fp64"], args.cpu_seconds)
            sample = (f"the first {k} of {len(prob.params)} parameter sets; the oracle evaluates g at "
                      "every (state, last node) pair, so its rate is in those evaluations")
        elif args.workload == "shifts_d20_peak":
            base, e32, e64 = oracle_shifts_baseline(prob, res["fp32c"], res["fp64"])
        elif args.workload == "mdi_d100_gauss":
            base, vals = oracle_mdi_baseline(prob)
            qs32, qs64 = res["fp32c"]["q"], res["fp64"]["q"]
            e32 = max(abs(qs32[s] - v) / abs(v) for s, v in enumerate(vals))
            e64 = max(abs(qs64[s] - v) / abs(v) for s, v in enumerate(vals))
        else:
            base, qo, ao = oracle_baseline(prob, args.cpu_seconds)
            e32 = abs(res["fp32c"]["q"] - qo) / max(abs(qo), ao)
            e64 = abs(res["fp64"]["q"] - qo) / max(abs(qo), ao)
        if base is None:
            base = {"value": rate, "unit": line["unit"], "cores": 1, "kind": "oracle", "sample": sample}
        line["cpu_baseline"] = base
        line["rel_err"] = e32
        line["fp64"]["rel_err"] = e64
        line["meets_1e-6"] = bool(e32 <= 1e-6)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
