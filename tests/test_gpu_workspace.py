"""One workspace shared by every entry point that takes one.  Its first 4 MiB
(completion counters and reduction slots) must be zero again after every call,
so that any sequence of calls may use one workspace without clearing it: each
call here runs on the shared workspace and on a fresh one, and the two must
agree bit for bit."""
import numpy as np
import pytest

from paper_2404_08867_amd import qmc

pytestmark = pytest.mark.gpu

ZERO_REGION = 4 << 20


def _region_is_zero(ws):
    import torch
    torch.cuda.synchronize()
    return int(torch.count_nonzero(ws.buf[:ZERO_REGION]).item()) == 0


def test_one_workspace_serves_every_entry_point():
    import torch
    d, n = 20, 65521
    z = qmc.korobov(d, n, 17)
    rng = np.random.default_rng(2404)
    peak = np.concatenate([rng.uniform(0.5, 1.5, d), rng.uniform(0.0, 1.0, d)])
    sums = np.array([[1.0, 1.0, 5.0], [0.7, 1.3, 2.5]])
    need = max(qmc.workspace_size(d, n, 1), qmc.mdi_lr_sum_workspace_size(100, 64),
               qmc.implr_workspace_size(4, 1048573, 100), qmc.criteria_workspace_size(d, n))
    ws = qmc.Workspace(need)
    assert _region_is_zero(ws)

    def fresh():
        return qmc.Workspace(need)

    steps = [
        ("lattice_sum", lambda w: qmc.lattice_sum(z, n, qmc.PRODUCT_PEAK, peak, qmc.FP32_COMPENSATED, ws=w)),
        ("mdi_lr_sum", lambda w: qmc.mdi_lr_sum(100, 64, 64, qmc.SUM_POWER, sums, qmc.FP64, ws=w)),
        ("implr_grid", lambda w: qmc.implr_grid(4, 1048573, 100, qmc.IMPLR_AUTO, ws=w)[1]),
        ("implr_grid bitmap", lambda w: qmc.implr_grid(4, 1048573, 100, qmc.IMPLR_BITMAP, ws=w)[1]),
        ("p_alpha", lambda w: qmc.p_alpha(z, n, 2, ws=w)),
        ("mdi_lr_sum fp32c", lambda w: qmc.mdi_lr_sum(100, 64, 64, qmc.SUM_POWER, sums,
                                                     qmc.FP32_COMPENSATED, ws=w)),
        ("lattice_sum again", lambda w: qmc.lattice_sum(z, n, qmc.PRODUCT_PEAK, peak,
                                                        qmc.FP32_COMPENSATED, ws=w)),
    ]
    for name, call in steps:
        got = call(ws).clone()
        assert _region_is_zero(ws), name
        want = call(fresh())
        torch.cuda.synchronize()
        assert torch.equal(got, want), (name, got, want)
