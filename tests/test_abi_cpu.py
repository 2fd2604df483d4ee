"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, its host helpers are right, and invalid calls fail cleanly
before anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_08867_amd import qmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = qmc.lib()
    names = _declared()
    assert "qmc_lattice_sum" in names and "qmc_mdi_lr" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings():
    assert "gfx950" in qmc.version()
    L = qmc.lib()
    for s in range(6):
        assert L.qmc_status_string(s)
    assert L.qmc_status_string(99) == b"unknown status"


@pytest.mark.parametrize("d,n,a", [(4, 1009, 77), (20, 1048573, 123457), (50, 16777213, 9999991),
                                   (7, 1000, 3), (1, 1, 5), (1024, 2147483647, 16807)])
def test_korobov_is_modular_power(d, n, a):
    assert [int(v) for v in qmc.korobov(d, n, a)] == [pow(a, j, n) for j in range(d)]


def test_mdi_dims_paper_cases():
    # Lemma 3.2 (n = a^d), Table 2-1 header (n = 1 + 10^d), Fig. 5 (n = 81, z = (1, 7)).
    assert list(qmc.mdi_lr_dims(100, 64, qmc.N_A_POW_D)) == [64] * 100
    assert list(qmc.mdi_lr_dims(6, 10, qmc.N_ONE_PLUS_A_POW_D)) == [10] * 5 + [11]
    assert list(qmc.mdi_lr_dims(2, 7, qmc.N_EXPLICIT, 81)) == [7, 12]
    assert list(qmc.mdi_lr_dims(3, 4, qmc.N_EXPLICIT, 161)) == [4, 4, 11]
    for d in range(2, 7):
        N = qmc.mdi_lr_dims(d, 10, qmc.N_EXPLICIT, 1 + 10 ** d)
        assert int(np.prod(N.astype(np.int64))) == 11 * 10 ** (d - 1)


def test_param_count_and_workspace():
    assert [qmc.param_count(f, 7) for f in range(5)] == [7, 14, 14, 8, 14]
    assert qmc.workspace_size(20, 1 << 20, 1) >= 8 * 2048
    assert qmc.workspace_size(50, 1 << 24, 64) >= 64 * 8


def _status(fn, *args):
    return fn(*args)


def test_invalid_arguments_fail_before_launch():
    L = qmc.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ws = ctypes.c_void_p(0x100000)
    # d out of range
    assert L.qmc_lattice_sum(0, 100, fake, None, 0, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    assert b"d = 0" in L.qmc_last_error()
    assert L.qmc_lattice_sum(1025, 100, fake, None, 0, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    # n out of range
    assert L.qmc_lattice_sum(4, 0, fake, None, 0, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum(4, 1 << 31, fake, None, 0, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    # family, precision, nsets
    assert L.qmc_lattice_sum(4, 100, fake, None, 7, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum(4, 100, fake, None, 0, fake, 1, 5, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum(4, 100, fake, None, 0, fake, 0, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    # null pointers
    assert L.qmc_lattice_sum(4, 100, None, None, 0, fake, 1, 0, fake, ws, 1 << 20, None) == qmc.ERR_INVALID_ARG
    # workspace: null, misaligned, too small
    assert L.qmc_lattice_sum(4, 100, fake, None, 0, fake, 1, 0, fake, None, 1 << 20, None) == qmc.ERR_WORKSPACE
    assert L.qmc_lattice_sum(4, 100, fake, None, 0, fake, 1, 0, fake, ctypes.c_void_p(0x100008), 1 << 20,
                             None) == qmc.ERR_WORKSPACE
    assert L.qmc_lattice_sum(4, 100, fake, None, 0, fake, 1, 0, fake, ws, 16, None) == qmc.ERR_WORKSPACE
    assert b"needed" in L.qmc_last_error()
    # shift ensembles: R out of range, null shifts or params, short workspace
    big = 1 << 23
    assert L.qmc_lattice_sum_shifts(4, 100, fake, fake, 0, 0, fake, 0, fake, None, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum_shifts(4, 100, fake, fake, 4097, 0, fake, 0, fake, None, ws, big,
                                    None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum_shifts(4, 100, fake, None, 3, 0, fake, 0, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum_shifts(4, 100, fake, fake, 3, 0, None, 0, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum_shifts(4, 100, fake, fake, 3, 0, fake, 0, fake, fake, ws, 16, None) == qmc.ERR_WORKSPACE
    # lattice criteria: alpha, n, candidate range, CBC size limit, workspace
    assert L.qmc_bernoulli_sum(4, 100, fake, 1, 3, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_bernoulli_sum(4, 1, fake, 1, 2, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_bernoulli_sum(4, 100, fake, 0, 2, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_bernoulli_sum(4, 100, fake, 1, 2, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    p2 = ctypes.byref(qmc.Criterion(qmc.CRIT_P_ALPHA, 2, None, 0.0))
    assert L.qmc_korobov_search(4, 100, p2, 0, 10, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_korobov_search(4, 100, p2, 95, 10, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_korobov_search(4, 100, p2, 1, 10, fake, fake, ws, 16, None) == qmc.ERR_WORKSPACE
    assert L.qmc_korobov_search(4, 100, None, 1, 10, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_cbc(4, (1 << 26) + 1, p2, fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_cbc(4, 100, p2, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    # criterion descriptors: unknown kind, alpha, missing gamma, negative or infinite beta
    for crit in (qmc.Criterion(7, 2, None, 0.0), qmc.Criterion(qmc.CRIT_P_ALPHA, 3, None, 0.0),
                 qmc.Criterion(qmc.CRIT_WCE2, 2, None, 0.0), qmc.Criterion(qmc.CRIT_WCE2, 2, fake.value, -1.0),
                 qmc.Criterion(qmc.CRIT_WCE2, 2, fake.value, float("inf"))):
        assert L.qmc_cbc(4, 100, ctypes.byref(crit), fake, fake, ws, big, None) == qmc.ERR_INVALID_ARG
        assert L.qmc_korobov_search(4, 100, ctypes.byref(crit), 1, 10, fake, fake, ws, big,
                                    None) == qmc.ERR_INVALID_ARG
    assert L.qmc_p_alpha(4, 100, fake, 1, 3, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_p_alpha(4, 100, fake, 0, 2, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_p_alpha(4, 100, fake, 1, 2, None, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_p_alpha(4, 100, fake, 1, 2, fake, ws, 16, None) == qmc.ERR_WORKSPACE
    assert L.qmc_shift_avg_wce2(4, 100, fake, 1, None, 0.0, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_shift_avg_wce2(4, 100, fake, 1, fake, -0.1, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_shift_avg_wce2(4, 1, fake, 1, fake, 0.0, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    # the improved rule's grid: d, a, a^{d-1} < n, null output, workspace
    assert L.qmc_implr_grid(0, 101, 3, 0, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_grid(3, 101, 0, 0, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_grid(3, 100, 10, 0, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert b"below n" in L.qmc_last_error()
    assert L.qmc_implr_grid(4, 101, 5, 0, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_grid(3, 101, 3, 2, None, fake, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_grid(3, 101, 3, 0, None, None, ws, big, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_grid(3, 101, 3, 1, None, fake, ws, 16, None) == qmc.ERR_WORKSPACE
    assert L.qmc_implr_points(3, 101, 3, 100, 2, fake, 4, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 3, -1, 2, fake, 4, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 3, 0, 2, None, 4, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 11, 0, 2, fake, 4, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 3, 0, 8, fake, 7, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 3, 0, 8, fake, (1 << 40) + 1, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_implr_points(3, 101, 3, 0, 8, ctypes.c_void_p(0x1002), 8, None) == qmc.ERR_INVALID_ARG
    # MDI-LR and the index export
    assert L.qmc_mdi_lr(0, fake, 0, fake, 1, 0, fake, None, 0, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_mdi_lr(4, None, 0, fake, 1, 0, fake, None, 0, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_points(4, 100, fake, -1, 10, fake, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_points(4, 100, fake, 0, (1 << 26) + 1, fake, None) == qmc.ERR_INVALID_ARG
    # host helpers
    z = np.zeros(4, dtype=np.int64)
    assert L.qmc_korobov(4, 0, 3, z.ctypes.data) == qmc.ERR_INVALID_ARG
    N = np.zeros(3, dtype=np.int32)
    assert L.qmc_mdi_lr_dims(3, 3, 9, 0, N.ctypes.data) == qmc.ERR_INVALID_ARG
    assert L.qmc_mdi_lr_dims(3, 1 << 21, 0, 0, N.ctypes.data) == qmc.ERR_INVALID_ARG
    # z(a) with a = n: z_2 = 0 makes eq. 3.5 undefined
    assert L.qmc_mdi_lr_dims(3, 7, qmc.N_EXPLICIT, 7, N.ctypes.data) == qmc.ERR_INVALID_ARG


def test_criteria_workspace_size():
    # zero region, the weights (2 d + 1 doubles), then the larger of (4096 generating
    # vectors + n mask bytes) and n + n/2 doubles, each part 256-byte aligned
    def expect(d, n):
        weights = ((2 * d + 1) * 8 + 255) // 256 * 256
        return (4 << 20) + weights + (max(4096 * d * 8 + n, (n + n // 2 + 2) * 8) + 255) // 256 * 256
    for d, n in [(20, 65521), (200, 1009), (2, 1 << 24), (1024, 3)]:
        assert qmc.criteria_workspace_size(d, n) == expect(d, n)


@pytest.mark.parametrize("d,n,a", [(3, 101, 3), (3, 1290**3 + 1, 1290), (1, 97, 5), (5, 1 << 30, 181),
                                   (2, 2147483647, 16807)])
def test_implr_workspace_size(d, n, a):
    # the shared 4 MiB zero region, a counter, then one bit per point of the
    # a^{d-1} ceil(n / a^{d-1}) grid (eq. 3.5)
    zd = a ** (d - 1)
    grid = zd * -(-n // zd)
    assert qmc.implr_workspace_size(d, n, a) == (4 << 20) + 256 + ((grid + 31) // 32 * 4 + 255) // 256 * 256


@pytest.mark.parametrize("d,N", [(1, 1), (7, 2), (100, 64), (300, 64)])
def test_mdi_lr_sum_workspace_size(d, N):
    # the shared 4 MiB zero region, then 35 vectors of d (N - 1) + 1 doubles
    L = d * (N - 1) + 1
    assert qmc.mdi_lr_sum_workspace_size(d, N) == (4 << 20) + (35 * L * 8 + 255) // 256 * 256


def test_last_error_is_cleared_by_success():
    L = qmc.lib()
    z = np.zeros(4, dtype=np.int64)
    assert L.qmc_korobov(4, 0, 3, z.ctypes.data) == qmc.ERR_INVALID_ARG
    assert L.qmc_last_error() != b""
    assert L.qmc_korobov(4, 11, 3, z.ctypes.data) == qmc.OK
    assert L.qmc_last_error() == b""


def test_python_binding_raises_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(qmc, "_lib", None)
    monkeypatch.setattr(qmc, "LIB_PATH", str(tmp_path / "libqmc.so"))
    with pytest.raises(qmc.QmcError):
        qmc.lib()


def test_batch_plan_rejects_invalid_problems():
    L = qmc.lib()
    fake = 0x1000
    plan = ctypes.c_void_p()

    def create(probs, precision=0, cfg=None):
        arr = (qmc.Problem * len(probs))(*probs)
        return L.qmc_batch_plan_create(len(probs), ctypes.byref(arr), precision,
                                       ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(plan))

    good = qmc.Problem(0, 4, 1009, fake, fake, None)
    assert L.qmc_batch_plan_create(0, None, 0, None, ctypes.byref(plan)) == qmc.ERR_INVALID_ARG
    assert create([good, qmc.Problem(9, 4, 1009, fake, fake, None)]) == qmc.ERR_INVALID_ARG
    assert b"problem 1" in L.qmc_last_error()
    assert create([qmc.Problem(0, 0, 1009, fake, fake, None)]) == qmc.ERR_INVALID_ARG
    assert create([qmc.Problem(0, 4, 0, fake, fake, None)]) == qmc.ERR_INVALID_ARG
    assert create([qmc.Problem(0, 4, 1 << 31, fake, fake, None)]) == qmc.ERR_INVALID_ARG
    assert create([qmc.Problem(0, 4, 1009, None, fake, None)]) == qmc.ERR_INVALID_ARG
    assert create([good], precision=7) == qmc.ERR_INVALID_ARG
    assert create([good], cfg=qmc.BatchConfig(5, 4, 0)) == qmc.ERR_INVALID_ARG
    assert create([good], cfg=qmc.BatchConfig(8, 9, 0)) == qmc.ERR_INVALID_ARG
    assert create([good], cfg=qmc.BatchConfig(8, 4, 2)) == qmc.ERR_INVALID_ARG
    assert L.qmc_lattice_sum_batched(None, fake, fake, 0, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_graph_launch(None, None) == qmc.ERR_INVALID_ARG
    assert L.qmc_batch_plan_destroy(None) == qmc.OK


def test_probe_library_host_side():
    """The measurement probes (libqmc_probe.so, not part of the C ABI) load without a GPU:
    the issue-rate kinds and the timeline's layout are host arithmetic, and the timeline
    entry point rejects bad arguments before any HIP call."""
    path = os.path.join(ROOT, "paper_2404_08867_amd", "libqmc_probe.so")
    if not os.path.exists(path):
        pytest.skip("libqmc_probe.so not built")
    P = ctypes.CDLL(path)
    P.qmc_probe_lane_ops.restype = ctypes.c_double
    P.qmc_probe_lane_ops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    kinds = P.qmc_probe_kinds()
    assert kinds == 31
    # two chains of two operations per step out of eight chains: half an operation each
    assert P.qmc_probe_lane_ops(30, 2, 3) == 2 * 256 * 3 * 16 * 8 * 0.5
    assert P.qmc_probe_lane_ops(kinds, 2, 3) == -1.0
    P.qmc_probe_timeline_workgroups.argtypes = [ctypes.c_uint32]
    assert P.qmc_probe_timeline_marks() == 24
    # 1024 threads x 4 points per tile, one workgroup per tile up to 512
    assert P.qmc_probe_timeline_workgroups(1048573) == 256
    assert P.qmc_probe_timeline_workgroups(4096) == 1
    assert P.qmc_probe_timeline_workgroups(1 << 24) == 512
    P.qmc_probe_plain_timeline.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32] + [ctypes.c_void_p] * 6
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below fails its argument check
    for mode, d, n in [(3, 20, 1000), (0, 0, 1000), (0, 33, 1000), (0, 20, 0), (0, 20, (1 << 24) + 1)]:
        assert P.qmc_probe_plain_timeline(mode, d, n, fake, fake, fake, fake, fake, None) == -1
    assert P.qmc_probe_plain_timeline(0, 20, 1000, None, fake, fake, fake, fake, None) == -1
