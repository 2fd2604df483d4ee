"""Batched plain sums (one persistent launch for many integrands) against the oracle."""
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


def _mixed_problems(seed, count, dmax=130, nmax=60000):
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        fam = b % 5
        d = int(rng.integers(1, dmax + 1))
        n = int(rng.choice([1, 2, 63, 1025, int(rng.integers(3, nmax))])) if b % 7 == 0 else int(rng.integers(3, nmax))
        a = W.draw_coprime(rng, n)
        p = W.draw_params(rng, fam, d)
        shift = rng.uniform(0, 1, d) if b % 3 == 0 else None
        probs.append((fam, qmc.korobov(d, n, a), n, p, shift))
    return probs


def _oracle(probs):
    out = []
    for fam, z, n, p, shift in probs:
        out.append(O.lattice_sum(z, n, fam, p, shift))
    return out


def _check(q, ref, precision):
    for i, (qo, ao) in enumerate(ref):
        assert abs(q[i] - qo) / max(abs(qo), ao, 1e-300) <= TOL[precision], (i, q[i], qo)


@pytest.mark.parametrize("precision", [qmc.FP64, qmc.FP32_COMPENSATED])
def test_batched_matches_oracle(precision):
    probs = _mixed_problems(1, 41)
    plan = qmc.BatchPlan(probs, precision)
    q = plan.run().cpu().numpy()
    _check(q, _oracle(probs), precision)


def test_batched_every_configuration_is_exact_and_reproducible():
    probs = _mixed_problems(2, 23, dmax=70, nmax=30000)
    ref = _oracle(probs)
    for precision in (qmc.FP64, qmc.FP32_COMPENSATED):
        plan = qmc.BatchPlan(probs, precision)
        for M in (4, 8, 16):
            for wpc in (1, 8):
                for order in (0, 1):
                    plan.set_config(points_per_thread=M, workgroups_per_cu=wpc, order=order)
                    assert plan.config == {"points_per_thread": M, "workgroups_per_cu": wpc, "order": order}
                    q1 = plan.run().cpu().numpy()
                    q2 = plan.run().cpu().numpy()
                    assert np.array_equal(q1.view(np.int64), q2.view(np.int64))
                    _check(q1, ref, precision)


def test_batched_with_a_largest_n_problem():
    """A batch holding one n = 2^31 - 1 problem (z = (1, 2, 4), oscillatory with h =
    (-2, 1, 0) in the dual lattice: exactly cos(2 pi u + 2 pi h.Delta), eq. 2.3) among small
    random ones, which are checked against the oracle."""
    n, d = 2147483647, 3
    shift = np.random.default_rng(12).uniform(0, 1, d)
    u = 0.3125
    h = np.array([-2.0, 1.0, 0.0])
    big = (qmc.OSCILLATORY, qmc.korobov(d, n, 2), n, np.concatenate([[u], 2 * math.pi * h]), shift)
    small = _mixed_problems(9, 6, dmax=20, nmax=20000)
    probs = small[:3] + [big] + small[3:]
    expect = math.cos(2 * math.pi * u + 2 * math.pi * float(np.dot(h, shift)))
    ref = _oracle(small[:3]) + [None] + _oracle(small[3:])
    for precision, tol in ((qmc.FP64, 1e-12), (qmc.FP32_COMPENSATED, 1e-6)):
        q = qmc.BatchPlan(probs, precision).run().cpu().numpy()
        assert abs(q[3] - expect) < tol, (precision, q[3], expect)
        _check(np.delete(q, 3), ref[:3] + ref[4:], precision)


def test_batched_agrees_with_single_problem_kernel():
    probs = _mixed_problems(3, 12, dmax=40, nmax=200000)
    q = qmc.BatchPlan(probs, qmc.FP64).run().cpu().numpy()
    for i, (fam, z, n, p, shift) in enumerate(probs):
        qs = float(qmc.lattice_sum(z, n, fam, p, qmc.FP64, shift=shift).item())
        assert abs(q[i] - qs) <= 1e-13 * max(abs(qs), 1.0), i


def test_batched_graph_replays_match_eager():
    """A captured batched launch replayed several times, with eager work in between,
    returns the eager result every time (no memset nodes; counters self-reset)."""
    torch = _torch()
    probs = _mixed_problems(4, 17, dmax=50, nmax=40000)
    plan = qmc.BatchPlan(probs, qmc.FP32_COMPENSATED)
    eager = plan.run().cpu().numpy()
    out = torch.full((len(probs),), -1.0, dtype=torch.float64, device="cuda")
    g = plan.graph(out)
    other = _mixed_problems(5, 1, dmax=10, nmax=5000)[0]
    for r in range(4):
        out.fill_(-1.0)
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.int64), eager.view(np.int64)), r
        # eager work between replays: torch ops and a plain sum on the default workspace
        _ = (torch.arange(1000, device="cuda", dtype=torch.float64) ** 2).sum().item()
        fam, z, n, p, sh = other
        qmc.lattice_sum(z, n, fam, p, qmc.FP64, shift=sh)
        torch.cuda.synchronize()
    del g


def test_batched_autotune_picks_a_valid_config(tmp_path, monkeypatch):
    monkeypatch.setenv("QMC_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    probs = _mixed_problems(6, 30, dmax=60, nmax=100000)
    ref = _oracle(probs)
    plan = qmc.BatchPlan(probs, qmc.FP32_COMPENSATED)
    best = plan.autotune(reps=1)
    assert best["points_per_thread"] in (4, 8, 16) and 1 <= best["workgroups_per_cu"] <= 8
    assert plan.config == best
    _check(plan.run().cpu().numpy(), ref, qmc.FP32_COMPENSATED)
    # the cached entry is reused by a new plan of the same batch
    plan2 = qmc.BatchPlan(probs, qmc.FP32_COMPENSATED)
    assert plan2.autotune(reps=1) == best
    assert (tmp_path / "tune.txt").read_text().strip()


def _cached(name):
    """Oracle results written by tests/golden/make_oracle_cache.py (oracle/ only)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


@pytest.mark.parametrize("precision", [qmc.FP32_COMPENSATED, qmc.FP64])
def test_batched_workload_4096_every_integrand(precision):
    """The 4096-integrand workload in one persistent launch: every Q against the FP64
    oracle's (cached), element by element."""
    batch = W.batched_4096()
    ref = _cached("batched_4096_oracle.json")
    assert ref["count"] == len(batch.problems)
    assert ref["d"] == [p.d for p in batch.problems] and ref["n"] == [p.n for p in batch.problems]
    assert ref["a"] == [p.a for p in batch.problems] and ref["family"] == [p.family for p in batch.problems]
    plan = qmc.BatchPlan.from_batch(batch, precision)
    q = plan.run().cpu().numpy()
    qo = np.array(ref["q"])
    ao = np.array(ref["abs_mean"])
    err = np.abs(q - qo) / np.maximum(np.abs(qo), ao)
    worst = int(np.argmax(err))
    p = batch.problems[worst]
    print(f"batched_4096 precision={precision}: max rel err {err[worst]:.3e} at integrand {worst} "
          f"(family {p.family}, d={p.d}, n={p.n}); median {np.median(err):.3e}")
    assert np.all(np.isfinite(q))
    assert err[worst] <= TOL[precision], (worst, p.family, p.d, p.n, q[worst], qo[worst])
