"""The measurement probes against the library: the phase-timeline copy of the plain-sum
kernel (probe/plain_timeline.hip) must compute the library's own bits, or its phase
times would describe another kernel; and every workgroup must leave exactly one total."""
import ctypes
import os

import numpy as np
import pytest

from paper_2404_08867_amd import qmc
from paper_2404_08867_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def probe():
    path = os.path.join(ROOT, "paper_2404_08867_amd", "libqmc_probe.so")
    if not os.path.exists(path):
        pytest.fail("libqmc_probe.so is not built")
    P = ctypes.CDLL(path)
    P.qmc_probe_plain_timeline.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32] + [ctypes.c_void_p] * 6
    P.qmc_probe_timeline_workgroups.argtypes = [ctypes.c_uint32]
    return P


@pytest.mark.parametrize("d,n,seed", [(20, 1048573, None), (5, 4097, 3), (32, 65521, 4), (1, 8191, 5)])
def test_timeline_copy_returns_library_bits(probe, d, n, seed):
    import torch
    if seed is None:
        w = W.plain_d20_peak()
        a, params = w.a, w.params
    else:
        rng = np.random.default_rng(seed)
        a = int(rng.integers(2, n))
        params = W.draw_params(rng, qmc.PRODUCT_PEAK, d)
    z = torch.tensor(qmc.korobov(d, n, a), device="cuda")
    p = torch.tensor(params, dtype=torch.float64, device="cuda")
    ws = qmc.Workspace(qmc.workspace_size(d, n, 1))
    q_lib = torch.zeros(1, dtype=torch.float64, device="cuda")
    qmc.lattice_sum(z, n, qmc.PRODUCT_PEAK, p, qmc.FP32_COMPENSATED, ws=ws, out=q_lib)
    G = probe.qmc_probe_timeline_workgroups(n)
    KM = probe.qmc_probe_timeline_marks()
    marks = torch.zeros(G * KM, dtype=torch.int64, device="cuda")
    q = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for mode in (0, 2, 1, 0):
        marks.zero_()
        rc = probe.qmc_probe_plain_timeline(mode, d, n, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                            ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(marks.data_ptr()),
                                            ctypes.c_void_p(ws.ptr), ctypes.c_void_p(stream))
        assert rc == G, rc
        torch.cuda.synchronize()
        a_marks = marks.view(G, KM).cpu().numpy()
        assert (a_marks[:, 0] > 0).all() and (a_marks[:, 19] >= a_marks[:, 0]).all()
        if mode != 1:
            assert int(a_marks[:, 20].sum()) == 1
            assert (a_marks[:, 1] >= a_marks[:, 0]).all() and (a_marks[:, 18] >= a_marks[:, 1]).all()
        if mode == 0:
            assert torch.equal(q, q_lib), (q.item(), q_lib.item())
    # the zero region is left zero: the library still gives the same bits afterwards
    q_again = torch.zeros(1, dtype=torch.float64, device="cuda")
    qmc.lattice_sum(z, n, qmc.PRODUCT_PEAK, p, qmc.FP32_COMPENSATED, ws=ws, out=q_again)
    assert torch.equal(q_again, q_lib)
