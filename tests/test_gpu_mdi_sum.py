"""Parity of MDI-LR for integrands of the coordinate sum (qmc_mdi_lr_sum) with the
FP64 oracle.  Every term is positive, so the bar is relative: 1e-12 (QMC_FP64)
and 1e-6 (QMC_FP32_COMPENSATED)."""
import numpy as np
import pytest

import oracle as O
from paper_2404_08867_amd import qmc
from paper_2404_08867_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {qmc.FP64: 1e-12, qmc.FP32_COMPENSATED: 1e-6}
PRECS = [qmc.FP64, qmc.FP32_COMPENSATED]


# (d, N, N_last): one direction; N = 1 (every state merges); a last count of
# a + 1 (eq. 3.5 with n = 1 + a^d); states past one pass of the window loop;
# Test 7's shape; more states than LDS holds (workspace buffers); long windows
# (N = 128, 600, 1500) with few directions, odd and even step counts.  The launcher
# counts the powers of up to 8 directions exactly (fewer where N^k or the binomials
# would leave 64-bit integers: 4 for N = 128 and 300, 2 for N = 1500 at two steps)
# and squares on from there: (64, 8, 8) is a pure power (no remainder), (2, 1500, 1500)
# needs no convolution at all, (5, 1500, 1500) counts four directions with N^4 near 5e12.
SHAPES = [(1, 1, 17), (5, 1, 3), (4, 10, 11), (12, 9, 9), (100, 64, 64), (300, 64, 65),
          (9, 128, 128), (3, 600, 600), (2, 1500, 1500), (2, 1500, 7),
          (64, 8, 8), (40, 2, 2), (5, 1500, 1500), (20, 300, 300)]
PARAMS = {qmc.SUM_POWER: [[1.0, 1.0, 5.0], [0.7, 1.3, 2.5], [2.0, 0.4, 0.5]],
          qmc.SUM_GAUSS: [[0.9, 0.3], [0.2, 1.7], [1.5, 4.0]]}


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("gfam", [qmc.SUM_POWER, qmc.SUM_GAUSS])
@pytest.mark.parametrize("d,N,N_last", SHAPES)
def test_mdi_sum_matches_oracle(precision, gfam, d, N, N_last):
    params = np.array(PARAMS[gfam], dtype=np.float64)
    if gfam == qmc.SUM_GAUSS:
        params[:, 1] *= d / 2  # centre the Gaussians where the sum lives
    q = qmc.mdi_lr_sum(d, N, N_last, gfam, params, precision).cpu().numpy()
    for s in range(len(params)):
        qo = O.mdi_sum(d, N, N_last, gfam, params[s])
        assert abs(q[s] - qo) <= TOL[precision] * abs(qo), (s, q[s], qo)


@pytest.mark.parametrize("precision", PRECS)
def test_mdi_sum_d100_full_size_sampled(precision):
    """The benchmark's workload (4096 sets, set 0 = f_6): sampled sets."""
    w = W.mdi_sum_d100()
    q = qmc.mdi_lr_sum(w.d, w.N, w.N_last, w.gfamily, w.params, precision).cpu().numpy()
    assert q.size == len(w.params) and np.all(q > 0) and np.all(np.isfinite(q))
    for s in (0, 1, 2047, 4095):
        qo = O.mdi_sum(w.d, w.N, w.N_last, w.gfamily, w.params[s])
        assert abs(q[s] - qo) <= TOL[precision] * abs(qo), (s, q[s], qo)


def test_mdi_sum_graph_replays_match_eager():
    """The state convolutions and the evaluation captured in one graph through the
    C ABI replay bit for bit, with eager calls of other shapes on the same
    workspace in between."""
    import torch
    L = qmc.lib()
    d, N, N_last = 100, 64, 64
    w = W.mdi_sum_d100()
    params = torch.tensor(w.params[:64], dtype=torch.float64, device="cuda")
    ws = qmc.Workspace(qmc.mdi_lr_sum_workspace_size(300, 64))
    for prec in PRECS:
        q = torch.zeros(64, dtype=torch.float64, device="cuda")

        def call():
            qmc._check(L.qmc_mdi_lr_sum(d, N, N_last, w.gfamily, qmc._ptr(params), 64, prec, qmc._ptr(q),
                                        ws.ptr, ws.nbytes, qmc._stream()), "qmc_mdi_lr_sum")

        call()
        torch.cuda.synchronize()
        ref = q.clone()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g):
                call()
        torch.cuda.current_stream().wait_stream(side)
        for rep in range(3):
            q.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(q, ref), (prec, rep)
            qmc.mdi_lr_sum(300, 64, 65, w.gfamily, w.params[:3], prec, ws=ws)  # another shape
            torch.cuda.synchronize()
        qo = O.mdi_sum(d, N, N_last, w.gfamily, w.params[0])
        assert abs(float(ref[0]) - qo) <= TOL[prec] * abs(qo)
