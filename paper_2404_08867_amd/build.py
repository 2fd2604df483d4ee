"""Build libqmc.so (the HIP library behind include/qmc.h) for gfx950.

Every source in csrc/ is compiled with hipcc into _build/, then linked into
paper_2404_08867_amd/libqmc.so (in-tree, so it travels with the repository).
Packed-FP32 instruction forms are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqmc.so")
# The probes behind the benchmark's measurements, a library of their own, not part of
# the C ABI: the issue-rate probe behind the ALU roofline (bench.py --workload rates)
# and the phase timeline of the plain-sum launch (--workload timeline_d20_peak).
PROBE_DIR = os.path.join(PKG, "probe")
PROBE_SRCS = ["issue_rates.hip", "plain_timeline.hip"]
PROBE_LIB = os.path.join(PKG, "libqmc_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

DEVICE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


# Per-source additions.  The plain-sum kernels take scalar arguments, the
# prologue's ten first: preloaded into scalar registers at wave start (gfx950
# supports kernel-argument preloading; the code object keeps a fallback
# prologue that loads them for firmware without it).
SOURCE_FLAGS = {
    "lattice_sum.hip": ["-mllvm", "-amdgpu-kernarg-preload-count=10"],
    # the timeline copy of the plain-sum kernel is built as the kernel itself is
    "plain_timeline.hip": ["-mllvm", "-amdgpu-kernarg-preload-count=10"],
    # The set-batched adjoint keeps its FP64 matrix accumulators in ordinary
    # VGPRs: in the AGPR form the compiler moved them between the two register
    # files every block of points.
    "adjoint.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    # The batched kernel's persistent loop: machine-level loop-invariant code motion
    # hoisted constants and per-thread addresses of every family's tile code out of it
    # and kept them live across the whole loop, which set the register count (150
    # vector registers in single precision, three waves per SIMD).  Without it: 125 and
    # 117, four waves per SIMD, no spills; the direction loops are unchanged.
    "batched.hip": ["-mllvm", "-disable-machine-licm"],
    # The same for the MDI-LR sum evaluation: the hoisted series constants of its log2
    # and exp2 held 85 registers in FP64 (63 without), and the step takes 2.5 % less.
    "mdi_sum.hip": ["-mllvm", "-disable-machine-licm"],
}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, verbose: bool, src_dir: str = CSRC, prefix: str = "") -> str:
    obj = os.path.join(BUILD, prefix + src.replace(".hip", ".o"))
    cmd = [HIPCC, "-c", *DEVICE_FLAGS, *SOURCE_FLAGS.get(src, []), os.path.join(src_dir, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build_probe(verbose: bool = False) -> str:
    """Compile the probes into libqmc_probe.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = [_compile(src, verbose, PROBE_DIR, "probe_") for src in PROBE_SRCS]
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    """Compile every csrc/*.hip and link libqmc.so (and the probe library); returns the
    path of libqmc.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + 1)) as ex:
        probe = ex.submit(build_probe, verbose)
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
        probe.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
