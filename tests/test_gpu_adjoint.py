"""Adjoint kernel and autograd Function against the oracle, finite differences and
an exact derivative.  Gradient errors are measured componentwise against the
largest oracle gradient component of the set (mixed signs make a per-component
relative error meaningless near zero)."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_08867_amd import qmc
from paper_2404_08867_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {qmc.FP64: 1e-12, qmc.FP32_COMPENSATED: 1e-6}


def _torch():
    import torch
    return torch


def _check_set(q, g, qo, ao, go, tol):
    assert abs(q - qo) <= tol * max(abs(qo), ao)
    scale = max(float(np.max(np.abs(go))), 1e-300)
    err = float(np.max(np.abs(g - go)))
    assert err <= tol * scale, (err / scale, np.argmax(np.abs(g - go)))


@pytest.mark.parametrize("precision", [qmc.FP64, qmc.FP32_COMPENSATED])
@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("d,n", [(3, 10007), (20, 65537), (65, 3001), (130, 1009), (1, 997)])
def test_adjoint_matches_oracle(precision, family, d, n):
    rng = np.random.default_rng(7 * d + n + family)
    z = qmc.korobov(d, n, W.draw_coprime(rng, n))
    shift = rng.uniform(0, 1, d) if (d + family) % 2 else None
    params = np.stack([W.draw_params(rng, family, d) for _ in range(2)])
    q, g = qmc.lattice_sum_adjoint(z, n, family, params, precision, shift=shift)
    q, g = q.cpu().numpy(), g.cpu().numpy()
    for s in range(2):
        qo, go = O.lattice_grad(z, n, family, params[s], shift)
        _, ao = O.lattice_sum(z, n, family, params[s], shift)
        _check_set(q[s], g[s], qo, ao, go, TOL[precision])


def test_adjoint_value_equals_forward_and_gq_scales():
    rng = np.random.default_rng(3)
    d, n = 12, 50021
    z = qmc.korobov(d, n, 4321)
    for family in range(5):
        params = np.stack([W.draw_params(rng, family, d) for _ in range(3)])
        q, g = qmc.lattice_sum_adjoint(z, n, family, params, qmc.FP64)
        qf = qmc.lattice_sum(z, n, family, params, qmc.FP64)
        assert np.allclose(q.cpu().numpy(), qf.cpu().numpy(), rtol=1e-13, atol=0)
        gq = np.array([2.5, -1.0, 0.0])
        _, g2 = qmc.lattice_sum_adjoint(z, n, family, params, qmc.FP64, gq=gq)
        assert np.allclose(g2.cpu().numpy(), gq[:, None] * g.cpu().numpy(), rtol=1e-15, atol=0)


@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
def test_adjoint_matches_finite_differences_of_device_forward(family):
    rng = np.random.default_rng(40 + family)
    d, n = 4, 4099
    z = qmc.korobov(d, n, 1234)
    shift = rng.uniform(0, 1, d)
    p = W.draw_params(rng, family, d)
    _, g = qmc.lattice_sum_adjoint(z, n, family, p, qmc.FP64, shift=shift)
    g = g.cpu().numpy()
    for k in range(p.size):
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (float(qmc.lattice_sum(z, n, family, pp, qmc.FP64, shift=shift).item())
              - float(qmc.lattice_sum(z, n, family, pm, qmc.FP64, shift=shift).item())) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9), k


def test_adjoint_exact_u_derivative_of_character_sum():
    """d/du (1/n) sum cos(2 pi u + 2 pi h.(x_i + Delta)) = -2 pi sin(2 pi u + 2 pi h.Delta)
    for h in the dual lattice (eq. 2.3)."""
    n, d = 10007, 4
    z = qmc.korobov(d, n, 1234)
    rng = np.random.default_rng(9)
    shift = rng.uniform(0, 1, d)
    h = [int(v) for v in rng.integers(-5, 6, d - 1)]
    s = sum(hj * int(zj) for hj, zj in zip(h, z[:-1]))
    hd = (-s * pow(int(z[-1]), -1, n)) % n
    h = np.array(h + [hd - n if hd > n // 2 else hd])
    u = 0.37
    params = np.concatenate([[u], 2 * math.pi * h.astype(float)])
    q, g = qmc.lattice_sum_adjoint(z, n, qmc.OSCILLATORY, params, qmc.FP64, shift=shift)
    arg = 2 * math.pi * u + 2 * math.pi * float(np.dot(h, shift))
    assert float(q.item()) == pytest.approx(math.cos(arg), abs=1e-12)
    assert float(g[0].item()) == pytest.approx(-2 * math.pi * math.sin(arg), abs=2 * math.pi * 1e-12)


def test_adjoint_character_identity_at_largest_n():
    """The adjoint at n = 2^31 - 1, z = (1, 2, 4), h = (-2, 1, 0) in the dual lattice: the
    value is cos(2 pi u + 2 pi h.Delta) and its u-derivative -2 pi sin(...) exactly."""
    n, d = 2147483647, 3
    z = qmc.korobov(d, n, 2)
    shift = np.random.default_rng(6).uniform(0, 1, d)
    u = 0.37
    h = np.array([-2.0, 1.0, 0.0])
    params = np.concatenate([[u], 2 * math.pi * h])
    arg = 2 * math.pi * u + 2 * math.pi * float(np.dot(h, shift))
    for precision, tol in ((qmc.FP64, 1e-12), (qmc.FP32_COMPENSATED, 1e-6)):
        q, g = qmc.lattice_sum_adjoint(z, n, qmc.OSCILLATORY, params, precision, shift=shift)
        assert float(q.item()) == pytest.approx(math.cos(arg), abs=tol)
        assert float(g[0].item()) == pytest.approx(-2 * math.pi * math.sin(arg), abs=2 * math.pi * tol)


@pytest.mark.parametrize("precision", [qmc.FP32_COMPENSATED, qmc.FP64])
def test_adjoint_workload_d50_every_set(precision):
    """64 oscillatory sets, d = 50, n = 16777213 in one adjoint launch: the value and all
    51 gradient components of every set against the FP64 oracle's (cached)."""
    w = W.adjoint_d50_osc()
    with open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_d50_osc_oracle.json")) as f:
        ref = json.load(f)
    assert (ref["d"], ref["n"], ref["a"], ref["nsets"]) == (w.d, w.n, w.a, w.params.shape[0])
    z = qmc.korobov(w.d, w.n, w.a)
    q, g = qmc.lattice_sum_adjoint(z, w.n, w.family, w.params, precision)
    q, g = q.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(q)) and np.all(np.isfinite(g))
    for s in range(w.params.shape[0]):
        _check_set(q[s], g[s], ref["q"][s], ref["abs_mean"][s], np.array(ref["grad"][s]), TOL[precision])


def test_autograd_function_gradcheck_and_chain_rule():
    torch = _torch()
    d, n = 3, 2003
    z = qmc.korobov(d, n, 561)
    rng = np.random.default_rng(5)
    for family in range(5):
        p = torch.tensor(np.stack([W.draw_params(rng, family, d) for _ in range(2)]), device="cuda",
                         requires_grad=True)
        f = lambda x: qmc.lattice_sum_autograd(x, z, n, family, qmc.FP64)
        assert torch.autograd.gradcheck(f, (p,), eps=1e-6, atol=1e-7, rtol=1e-5)
        q = f(p)
        loss = (q ** 2).sum()
        loss.backward()
        _, g = qmc.lattice_sum_adjoint(z, n, family, p.detach(), qmc.FP64)
        expect = 2 * q.detach()[:, None] * g
        assert torch.allclose(p.grad, expect, rtol=1e-12, atol=1e-14)


def test_adjoint_rejects_large_d():
    z = np.zeros(513, dtype=np.int64)
    with pytest.raises(qmc.QmcError) as e:
        qmc.lattice_sum_adjoint(z, 7, qmc.EXP_SUM, np.ones(513), qmc.FP64)
    assert e.value.status == qmc.ERR_UNSUPPORTED


# The set-batched form (exp-sum and oscillatory, d <= 64, at least 16 sets: FP64
# matrix instructions over 32 sets per wave) against the oracle set by set, and
# against the per-set form.  Direction buckets 16, 32, 48, 52, 56, 64.
@pytest.mark.parametrize("precision", [qmc.FP64, qmc.FP32_COMPENSATED])
@pytest.mark.parametrize("family", [0, 3])
@pytest.mark.parametrize("d,n,nsets", [(3, 10007, 16), (20, 65537, 64), (56, 3001, 70), (1, 997, 130),
                                       (9, 1009, 17), (64, 4099, 65), (57, 2003, 128), (33, 101, 20),
                                       (49, 2011, 33), (52, 4001, 47)])
def test_adjoint_set_batched_matches_oracle(precision, family, d, n, nsets):
    rng = np.random.default_rng(11 * d + n + family + nsets)
    z = qmc.korobov(d, n, W.draw_coprime(rng, n))
    shift = rng.uniform(0, 1, d) if (d + nsets) % 2 else None
    params = np.stack([W.draw_params(rng, family, d) for _ in range(nsets)])
    gq = rng.uniform(-2.0, 2.0, nsets)
    q, g = qmc.lattice_sum_adjoint(z, n, family, params, precision, shift=shift, gq=gq)
    q, g = q.cpu().numpy(), g.cpu().numpy()
    for s in sorted({0, 1, nsets // 2, nsets - 1, min(63, nsets - 1), min(64, nsets - 1)}):
        qo, go = O.lattice_grad(z, n, family, params[s], shift)
        _, ao = O.lattice_sum(z, n, family, params[s], shift)
        _check_set(q[s], g[s], qo, ao, gq[s] * go, TOL[precision])


@pytest.mark.parametrize("family", [0, 3])
def test_adjoint_set_batched_agrees_with_per_set_form(family):
    rng = np.random.default_rng(42 + family)
    d, n, nsets = 24, 50021, 40
    z = qmc.korobov(d, n, 20011)
    shift = rng.uniform(0, 1, d)
    params = np.stack([W.draw_params(rng, family, d) for _ in range(nsets)])
    q, g = qmc.lattice_sum_adjoint(z, n, family, params, qmc.FP64, shift=shift)
    q, g = q.cpu().numpy(), g.cpu().numpy()
    for s in (0, 7, 39):
        q1, g1 = qmc.lattice_sum_adjoint(z, n, family, params[s:s + 1], qmc.FP64, shift=shift)
        q1, g1 = q1.cpu().numpy()[0], g1.cpu().numpy()[0]
        assert abs(q[s] - q1) <= 1e-12 * max(abs(q1), 1e-3)
        assert np.max(np.abs(g[s] - g1)) <= 1e-12 * max(np.max(np.abs(g1)), 1e-300)


def test_adjoint_set_batched_workspace_from_workspace_size():
    # a workspace sized by qmc_workspace_size serves the set-batched form
    d, n, nsets = 50, 4099, 64
    rng = np.random.default_rng(9)
    z = qmc.korobov(d, n, 1234)
    params = np.stack([W.draw_params(rng, 3, d) for _ in range(nsets)])
    ws = qmc.Workspace(qmc.workspace_size(d, n, nsets))
    q, g = qmc.lattice_sum_adjoint(z, n, 3, params, qmc.FP64, ws=ws)
    qo, go = O.lattice_grad(z, n, 3, params[5])
    _, ao = O.lattice_sum(z, n, 3, params[5])
    _check_set(q.cpu().numpy()[5], g.cpu().numpy()[5], qo, ao, go, TOL[qmc.FP64])


def test_adjoint_set_batched_replays_in_a_graph():
    # the set-batched form's tickets reset themselves: every replay of a captured
    # call matches the eager result bit for bit, with eager calls in between
    torch = _torch()
    rng = np.random.default_rng(77)
    d, n, nsets = 30, 50021, 64
    z = torch.tensor(qmc.korobov(d, n, 4321), device="cuda")
    params = torch.tensor(np.stack([W.draw_params(rng, 3, d) for _ in range(nsets)]), device="cuda")
    ws = qmc.Workspace(qmc.workspace_size(d, n, nsets))
    q0, g0 = qmc.lattice_sum_adjoint(z, n, 3, params, qmc.FP32_COMPENSATED, ws=ws)
    q0, g0 = q0.clone(), g0.clone()
    holder = {}
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            holder["r"] = qmc.lattice_sum_adjoint(z, n, 3, params, qmc.FP32_COMPENSATED, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        holder["r"][0].fill_(0.0)
        holder["r"][1].fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(holder["r"][0], q0) and torch.equal(holder["r"][1], g0), rep
        qmc.lattice_sum_adjoint(z, n, 0, params[:20, :d], qmc.FP64, ws=ws)  # other work in between
        torch.cuda.synchronize()
