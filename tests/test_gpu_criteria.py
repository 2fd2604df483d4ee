"""Parity of the lattice-quality criteria and constructions (qmc_bernoulli_sum,
qmc_p_alpha, qmc_shift_avg_wce2, qmc_korobov_search, qmc_cbc) with the FP64 oracle.

Tolerance: criteria are FP64 sums of O(1) terms of both signs whose result is
small, so |S - S_oracle| <= 1e-12 * max(|S_oracle|, A), A the oracle's mean |term|
(the measure used for every mixed-sign sum).  The chosen generating vectors are
integers decided by floating point: for e^2 both sides apply the same rule
(smallest candidate within 1e-10 relative of the minimum) and are compared
exactly; for P_alpha, whose minimum can sit many orders of magnitude below its
terms and tie exactly between candidates, the GPU's choice is checked to attain
the oracle's minimum within the tolerance above.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle as O
from paper_2404_08867_amd import qmc
from paper_2404_08867_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _close(s, so, ao):
    return abs(s - so) <= TOL * max(abs(so), ao)


@pytest.mark.parametrize("alpha", [2, 4])
@pytest.mark.parametrize("d,n", [(3, 1009), (20, 4099), (65, 2003), (1, 997), (8, 64)])
def test_bernoulli_sum_matches_oracle(alpha, d, n):
    rng = np.random.default_rng(100 * d + n + alpha)
    rows = [O.korobov(d, n, int(rng.integers(1, n))) for _ in range(5)]
    a = rng.uniform(-2.0, 20.0, d) if alpha == 2 else rng.uniform(-20.0, 2.0, d)
    s = qmc.bernoulli_sum(np.stack(rows), n, alpha, a).cpu().numpy()
    for r, z in enumerate(rows):
        so, ao = O.lattice_kernel_sum(z, n, alpha, a)
        assert _close(s[r], so, ao), (r, s[r], so)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 64, 65, 4096, 4097, 65521, 65536, 1048573])
def test_bernoulli_sum_mirrored_half_for_any_z(n):
    """The device sums Bernoulli products over i <= n/2 only, with weight 2 for the
    mirrored pairs (i, n - i); odd and even n, generating vectors with any entries
    (zeros and repeats included), against the oracle's sums over all n points."""
    rng = np.random.default_rng(n)
    d = 6
    rows = [rng.integers(0, n, d) for _ in range(3)] + [np.zeros(d, dtype=np.int64),
                                                          np.full(d, n // 2, dtype=np.int64)]
    for alpha in (2, 4):
        a = rng.uniform(-2.0, 5.0, d)
        s = qmc.bernoulli_sum(np.stack(rows), n, alpha, a).cpu().numpy()
        for r, z in enumerate(rows):
            so, ao = O.lattice_kernel_sum(z, n, alpha, a)
            assert _close(s[r], so, ao), (n, alpha, r, s[r], so)


# The weights that make the Bernoulli sum S equal each criterion (eq. 2.4; eq. 2.12 with
# product weights): used here only to take the oracle's mean |term| as the scale of
# the mixed-sign sums.
P_ALPHA_WEIGHT = {2: 2 * math.pi ** 2, 4: -2 * math.pi ** 4 / 3}


def _p_alpha_scale(z, n, alpha):
    return O.lattice_kernel_sum(z, n, alpha, np.full(len(z), P_ALPHA_WEIGHT[alpha]))[1]


def _wce2_scale(z, n, gamma, beta):
    g = np.asarray(gamma, dtype=np.float64)[: len(z)]
    return float(np.prod(1 + g * beta)) * O.lattice_kernel_sum(z, n, 2, g / (1 + g * beta))[1]


@pytest.mark.parametrize("z,n", [([1, 3, 9, 27, 81], 1009), ([1, 40, 33, 19], 97), ([1, 1], 2)])
def test_criteria_entry_points(z, n):
    """qmc_p_alpha and qmc_shift_avg_wce2 return eq. 2.4's and eq. 2.12's values."""
    rows = np.stack([np.array(z), (np.array(z) * 7) % n])
    for alpha in (2, 4):
        p = qmc.p_alpha(rows, n, alpha).cpu().numpy()
        for r in range(2):
            assert _close(p[r], O.p_alpha(rows[r], n, alpha), _p_alpha_scale(rows[r], n, alpha)), (alpha, r)
    for gamma, beta in (([1.0, 0.5, 0.25, 0.125, 0.0625][: len(z)], 0.3), ([2.0] * len(z), 0.0),
                        ([0.7] * len(z), 1.0 / 12.0)):
        e2 = qmc.shift_avg_wce2(rows, n, gamma, beta).cpu().numpy()
        for r in range(2):
            eo = O.shift_avg_wce2(rows[r], n, gamma, beta)
            assert _close(e2[r], eo, _wce2_scale(rows[r], n, gamma, beta)), (gamma, beta, r)


def test_criteria_reject_bad_descriptors():
    z = np.array([[1, 3, 9]])
    with pytest.raises(qmc.QmcError):
        qmc.p_alpha(z, 101, 3)
    with pytest.raises(qmc.QmcError):
        qmc.shift_avg_wce2(z, 101, [1.0, 1.0, 1.0], -0.5)
    with pytest.raises(qmc.QmcError):
        qmc.shift_avg_wce2(z, 101, [1.0, 1.0], 0.0)


@pytest.mark.parametrize("d,n,alpha", [(8, 1009, 2), (5, 2003, 4), (4, 1000, 2), (4, 8191, 2)])
def test_korobov_search_matches_oracle(d, n, alpha):
    vals, best = qmc.korobov_search(d, n, alpha)
    vals = vals.cpu().numpy()
    best = best.cpu().numpy()
    ov, ob = O.korobov_search(d, n, alpha)
    assert np.array_equal(np.isinf(vals), np.isinf(ov))
    for a in range(1, n):
        if np.isfinite(ov[a - 1]):
            ao = _p_alpha_scale(O.korobov(d, n, a), n, alpha)
            assert _close(vals[a - 1], ov[a - 1], ao), (a, vals[a - 1], ov[a - 1])
    assert int(best[1]) == ob
    assert best[0] == vals[ob - 1]


@pytest.mark.parametrize("d,n,gamma,beta", [(5, 1009, [1.0, 0.5, 0.3, 0.2, 0.1], 0.0),
                                            (3, 997, [0.9, 0.9, 0.9], 0.25)])
def test_korobov_search_wce2_matches_oracle(d, n, gamma, beta):
    """The search minimising e^2 of eq. 2.12: every candidate's e^2 against the oracle's
    and the chosen a against the same selection rule on the oracle's values."""
    vals, best = qmc.korobov_search(d, n, gamma=gamma, beta=beta)
    vals = vals.cpu().numpy()
    best = best.cpu().numpy()
    ov = np.full(n - 1, np.inf)
    for a in range(1, n):
        if math.gcd(a, n) == 1:
            z = O.korobov(d, n, a)
            ov[a - 1] = O.shift_avg_wce2(z, n, gamma, beta)
            assert _close(vals[a - 1], ov[a - 1], _wce2_scale(z, n, gamma, beta)), a
        else:
            assert np.isinf(vals[a - 1])
    m = np.min(ov)
    pick = 1 + int(np.argmax(ov <= m + 1e-10 * abs(m)))
    assert int(best[1]) == pick and best[0] == vals[pick - 1]


@pytest.mark.parametrize("d,n,gamma,beta", [
    (5, 1009, [1.0, 0.8, 0.64, 0.512, 0.41], 0.0),
    (4, 2003, [0.5, 0.5, 0.5, 0.5], 0.25),
    (6, 251, [1.0, 1.0, 0.5, 0.5, 0.25, 0.25], 1.0 / 3.0),
    (3, 64, [0.9, 0.9, 0.9], 0.0),
])
def test_cbc_matches_oracle(d, n, gamma, beta):
    z, e2 = qmc.cbc(d, n, gamma, beta)
    z = z.cpu().numpy()
    e2 = e2.cpu().numpy()
    oz, oe2 = O.cbc(d, n, gamma, beta)
    assert np.array_equal(z, oz), (z, oz)
    for j in range(d):
        assert _close(e2[j], oe2[j], _wce2_scale(oz[: j + 1], n, gamma, beta)), j


def _check_p_alpha_cbc(z, s, n, alpha):
    """A P_alpha CBC result is valid when, at every component j, the chosen z_j is
    coprime to n, lies in [1, n/2], and its oracle P_alpha(z_1..z_j) attains the oracle's
    minimum over all such candidates given the same z_1..z_{j-1}, within the
    tolerance of the mixed-sign sums; and s_j is the oracle's P_alpha of z_1..z_j.
    Where the minimum is isolated this fixes z_j; exact ties (c and its inverse
    mod n at d = 2, where P_alpha sits many orders of magnitude below its terms)
    leave either choice valid."""
    assert z[0] == 1
    for j in range(len(z)):
        if j > 0:
            assert 1 <= z[j] <= n // 2 and math.gcd(int(z[j]), n) == 1, (j, z[j])
            prefix = [int(c) for c in z[:j]]
            m = min(O.p_alpha(prefix + [c], n, alpha)
                    for c in range(1, n // 2 + 1) if math.gcd(c, n) == 1)
        got = O.p_alpha(z[: j + 1], n, alpha)
        scale = _p_alpha_scale(z[: j + 1], n, alpha)
        if j > 0:
            assert got - m <= TOL * max(abs(m), scale), (n, j, z[j], got, m)
        assert _close(s[j], got, scale), (n, j, s[j], got)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 8, 30, 1024, 1025])
@pytest.mark.parametrize("alpha", [2, 4])
def test_cbc_small_and_even_n(n, alpha):
    """The device sums each criterion over the mirrored half of the indices (k and
    n - k give mirrored points); odd and even n, down to n = 2, against the oracle's
    full sums: e^2 (alpha = 2) and P_4."""
    d = 3
    if alpha == 2:
        gamma = np.array([1.0, 0.7, 0.3])
        z, e2 = qmc.cbc(d, n, gamma, 0.2)
        oz, oe2 = O.cbc(d, n, gamma, 0.2)
        assert np.array_equal(z.cpu().numpy(), oz)
        for j in range(d):
            assert _close(e2.cpu().numpy()[j], oe2[j], _wce2_scale(oz[: j + 1], n, gamma, 0.2)), j
    else:
        z, s = qmc.cbc(d, n, alpha=4)
        _check_p_alpha_cbc(z.cpu().numpy(), s.cpu().numpy(), n, 4)


@pytest.mark.parametrize("alpha", [2, 4])
def test_cbc_p_alpha_against_exhaustive_oracle_search(alpha):
    d, n = 3, 101
    z, s = qmc.cbc(d, n, alpha=alpha)
    _check_p_alpha_cbc(z.cpu().numpy(), s.cpu().numpy(), n, alpha)


@pytest.mark.parametrize("n", [(1 << 24) - 3, 1 << 24, (1 << 24) + 1, (1 << 24) + 43])
def test_cbc_either_side_of_the_float_index_limit(n):
    """Up to n = 2^24 the candidate sums step their residues as exact floats, above it
    as integers.  At d = 1 the one candidate z_1 = 1 is summed over all n/2 paired
    indices: its criterion against the oracle on either side of the limit."""
    gamma = np.array([0.8])
    z, e2 = qmc.cbc(1, n, gamma, 0.3)
    assert z.cpu().numpy().tolist() == [1]
    eo = O.shift_avg_wce2([1], n, gamma, 0.3)
    assert _close(e2.cpu().numpy()[0], eo, _wce2_scale([1], n, gamma, 0.3)), (n, e2, eo)


def test_korobov_search_d20_full_size_sampled():
    """The benchmark's search (n = 65521, d = 20, e^2 with gamma_j = j^-2, a in
    [1, n/2]): sampled candidates against the oracle, the chosen a's value, and the
    selection rule on the GPU's own values."""
    w = W.korobov_search_d20()
    vals, best = qmc.korobov_search(w.d, w.n, gamma=w.gamma, beta=w.beta, a0=w.a0, count=w.count)
    vals = vals.cpu().numpy()
    best = best.cpu().numpy()
    assert np.all(np.isfinite(vals)) and vals.size == w.count
    for cand in (1, 2, 17, 4099, w.a0 + w.count - 1, int(best[1])):
        z = O.korobov(w.d, w.n, cand)
        eo = O.shift_avg_wce2(z, w.n, w.gamma, w.beta)
        assert _close(vals[cand - w.a0], eo, _wce2_scale(z, w.n, w.gamma, w.beta)), cand
    m = np.min(vals)
    assert best[0] <= m * (1 + 1e-10) and np.all(vals[: int(best[1]) - w.a0] > m * (1 + 1e-10))


def test_cbc_d20_full_size_components():
    """The benchmark's CBC (n = 65521, d = 20): each component's criterion at the
    GPU's choices against the oracle; each choice beats the sampled alternatives."""
    w = W.cbc_d20()
    z, e2 = qmc.cbc(w.d, w.n, w.gamma, w.beta)
    z = z.cpu().numpy()
    e2 = e2.cpu().numpy()
    assert z[0] == 1 and np.all((z >= 1) & (z <= w.n // 2))
    for j in (0, 1, 2, 9, 19):
        eo = O.shift_avg_wce2(z[: j + 1], w.n, w.gamma[: j + 1], w.beta)
        assert _close(e2[j], eo, _wce2_scale(z[: j + 1], w.n, w.gamma, w.beta)), j
    for c in (1, 2, 1000, 20000, w.n // 2):
        alt = O.shift_avg_wce2(np.concatenate([z[:1], [c]]), w.n, w.gamma[:2], w.beta)
        assert e2[1] <= alt * (1 + 1e-10)


def test_criteria_graph_replays_match_eager():
    """The Korobov search (weights, table, mirrored Bernoulli sums, selection) and CBC
    (weights, init, then evaluation, selection and product update per component)
    captured in one graph through the C ABI: every replay reproduces the eager results
    bit for bit, with eager calls of other sizes on the same workspace in between."""
    import torch
    L = qmc.lib()
    d, n, count = 6, 1031, 515
    gamma_np = np.array([1.0, 0.8, 0.6, 0.4, 0.3, 0.2])
    gamma = torch.tensor(gamma_np, dtype=torch.float64, device="cuda")
    crit = qmc.Criterion(qmc.CRIT_WCE2, 2, qmc._ptr(gamma), 0.1)
    ws = qmc.Workspace(qmc.criteria_workspace_size(d, 4099))
    vals = torch.zeros(count, dtype=torch.float64, device="cuda")
    best = torch.zeros(2, dtype=torch.float64, device="cuda")
    z = torch.zeros(d, dtype=torch.int64, device="cuda")
    s = torch.zeros(d, dtype=torch.float64, device="cuda")

    def calls():
        qmc._check(L.qmc_korobov_search(d, n, ctypes.byref(crit), 1, count, qmc._ptr(vals), qmc._ptr(best),
                                        ws.ptr, ws.nbytes, qmc._stream()), "qmc_korobov_search")
        qmc._check(L.qmc_cbc(d, n, ctypes.byref(crit), qmc._ptr(z), qmc._ptr(s), ws.ptr, ws.nbytes,
                             qmc._stream()), "qmc_cbc")

    calls()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (vals, best, z, s)]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            calls()
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for t in (vals, best, z, s):
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        for t, r in zip((vals, best, z, s), ref):
            assert torch.equal(t, r), rep
        qmc.cbc(4, 4099, gamma_np[:4], 0.0, ws=ws)  # other sizes on the same workspace
        qmc.korobov_search(3, 2048, 2, a0=1, count=100, ws=ws)
        torch.cuda.synchronize()
    # the eager results themselves against the oracle
    oz, oe2 = O.cbc(d, n, gamma_np, 0.1)
    assert np.array_equal(z.cpu().numpy(), oz)
