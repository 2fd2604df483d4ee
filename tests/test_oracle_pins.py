"""Pins of the FP64 CPU oracle against facts the paper and mathematics fix.

Nothing here re-types the oracle's formulas.  Each test pins the oracle to an
independent fact:
  * relative errors printed in the paper's tables (tests/golden/paper_tables.csv);
  * node counts the paper states for eq. 3.5 (Fig. 5, Lemma 3.2, Table 2-1 header);
  * the rank-1 character identity behind eq. 2.3 (exact);
  * closed forms of one-dimensional left-rectangle and midpoint sums;
  * brute force over tiny tensor grids for the MDI-LR sweep;
  * central finite differences for the gradients;
  * Python's built-in modular power for the Korobov vector.
"""
import csv
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle as O
from paper_2404_08867_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.csv")


def _rows():
    with open(GOLDEN) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    return list(csv.DictReader(lines))


# ---- exact integrals of the paper's test integrands (textbook closed forms) ----
_S = float(mp.quad(lambda t: mp.sin(t * t), [0, 1]))  # int_0^1 sin(t^2) dt
_C = float(mp.quad(lambda t: mp.cos(t * t), [0, 1]))  # int_0^1 cos(t^2) dt


def _exact(name, d):
    if name == "gauss":  # the constant (2 pi)^-1/2 cancels in a relative error
        return (math.sqrt(math.pi / 2) * math.erf(1 / math.sqrt(2))) ** d
    if name == "expalt":
        return math.prod((math.exp(s) - 1) / s for s in [(-1.0) ** j for j in range(d)])
    if name == "peak":
        c, w = 1 / 0.9, 0.6
        return (c * (math.atan(c * (1 - w)) + math.atan(c * w))) ** d
    if name == "cos2":  # Re prod_j int e^{2 i x} dx = cos(d) sin(1)^d
        return math.cos(d) * math.sin(1.0) ** d
    if name == "test1f":
        return 1.0
    if name == "exp3":  # normalisation (e-1)^-3 cancels
        return (math.e - 1) ** 3
    if name == "sinsq":  # sin of a sum of squares, expanded
        return 2 * _S * _C if d == 2 else 3 * _S * _C * _C - _S ** 3
    raise KeyError(name)


def _family(name, d):
    if name == "gauss":
        return O.GAUSSIAN, np.concatenate([np.full(d, 1 / math.sqrt(2)), np.zeros(d)])
    if name == "expalt":
        return O.EXP_SUM, np.array([(-1.0) ** j for j in range(d)])
    if name == "peak":
        return O.PRODUCT_PEAK, np.concatenate([np.full(d, 1 / 0.9), np.full(d, 0.6)])
    if name == "cos2":
        return O.OSCILLATORY, np.concatenate([[1.0], np.full(d, 2.0)])
    if name == "exp3":
        return O.EXP_SUM, np.ones(d)
    if name == "test1f":
        return O.TEST1_F, np.zeros(1)
    if name == "sinsq":
        return O.SIN_SQ, np.zeros(1)
    raise KeyError(name)


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"{r['table']}-{r['method']}-{r['integrand']}-"
                         f"d{r['d']}-n{r['n']}-a{r['a']}-N{r['n_common']}")
def test_paper_table_value(row):
    """The oracle reproduces each printed relative error to its printed digits
    (within one unit of the last digit: the paper both rounds and truncates)."""
    d = int(row["d"])
    fam, p = _family(row["integrand"], d)
    if row["method"] == "SLR":
        n, a = int(row["n"]), int(row["a"])
        q, _ = O.lattice_sum(O.korobov(d, n, a), n, fam, p)
    else:
        N = [int(row["n_common"])] * (d - 1) + [int(row["n_last"])]
        q = O.mdi_lr_brute(N, fam, p) if fam >= 100 else O.mdi_lr(N, fam, p)
    exact = _exact(row["integrand"], d)
    err = abs(q - exact) / abs(exact)
    printed = float(row["printed"])
    unit = 10.0 ** (math.floor(math.log10(printed)) - int(row["digits"]) + 1)
    assert abs(err - printed) <= 1.0001 * unit, (err, printed)


def test_mdi_sweep_matches_brute_force_on_printed_families():
    """Sweep and brute force agree on the Table 3-x integrands at d = 4 (ragged N)."""
    for name in ("gauss", "cos2", "peak", "expalt"):
        fam, p = _family(name, 4)
        N = [3, 5, 4, 6]
        assert O.mdi_lr(N, fam, p) == pytest.approx(O.mdi_lr_brute(N, fam, p), rel=1e-13)


# ---- eq. 3.5 node counts ---------------------------------------------------------
def test_eq35_figure5_example():
    """Fig. 5: n = 81, z = (1, 7) needs n* = 3 added points for a tensor grid."""
    N = O.mdi_dims([1, 7], 81)
    assert list(N) == [7, 12]
    assert int(np.prod(N)) - 81 == 3


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_eq35_table21_header(d):
    """Table 2-1 header: n = 1 + 10^d with a = 10 gives 1.1 x 10^d tensor nodes."""
    n = 1 + 10 ** d
    N = O.mdi_dims(O.korobov(d, n, 10), n)
    assert int(np.prod(N)) == 11 * 10 ** (d - 1)


@pytest.mark.parametrize("a,d", [(3, 5), (8, 6), (10, 4), (64, 4)])
def test_eq35_lemma32_equal_counts(a, d):
    """Lemma 3.2: with n = a^d every direction has a nodes."""
    n = a ** d
    N = O.mdi_dims(O.korobov(d, n, a), n)
    assert list(N) == [a] * d


# ---- the Korobov vector and the lattice indices --------------------------------
@pytest.mark.parametrize("d,n,a", [(4, 1009, 77), (20, 1048573, 123457), (50, 16777213, 9999991),
                                   (7, 1000, 3), (3, 2, 1)])
def test_korobov_is_modular_power(d, n, a):
    z = O.korobov(d, n, a)
    assert [int(v) for v in z] == [pow(a, j, n) for j in range(d)]


@pytest.mark.parametrize("n,a", [(1009, 77), (1000, 7), (97, 5)])
def test_lattice_indices_are_permutations(n, a):
    """With gcd(z_j, n) = 1 each coordinate index runs over all residues, and
    consecutive points differ by z_j (mod n)."""
    z = O.korobov(3, n, a)
    k = O.lattice_points(z, n)
    for j in range(3):
        assert sorted(k[:, j].tolist()) == list(range(n))
        assert np.all((k[1:, j] - k[:-1, j]) % n == z[j] % n)
    assert np.all(k[0] == 0)


# ---- the character identity (eq. 2.3) -------------------------------------------
def _dual_vector(rng, z, n):
    """h with h . z = 0 (mod n): free h_1..h_{d-1}, h_d solved with z_d^-1 mod n."""
    d = len(z)
    h = [int(v) for v in rng.integers(-6, 7, d - 1)]
    s = sum(hj * int(zj) for hj, zj in zip(h, z[:-1]))
    hd = (-s * pow(int(z[-1]), -1, n)) % n
    if hd > n // 2:
        hd -= n
    return np.array(h + [hd])


@pytest.mark.parametrize("n,a,d,shifted", [(1009, 331, 3, False), (1009, 331, 4, True),
                                           (10007, 1234, 5, True), (4099, 17, 2, False)])
def test_character_identity(n, a, d, shifted):
    """(1/n) sum_i cos(2 pi u + 2 pi h.(x_i + Delta)) = cos(2 pi u + 2 pi h.Delta) if h.z = 0
    (mod n), else 0 -- exactly, for every h (the rank-1 lattice dual, eq. 2.3)."""
    rng = np.random.default_rng(n + d)
    z = O.korobov(d, n, a)
    shift = rng.uniform(0, 1, d) if shifted else None
    delta = shift if shifted else np.zeros(d)
    u = 0.3125
    for trial in range(4):
        if trial % 2 == 0:
            h = _dual_vector(rng, z, n)
        else:
            h = rng.integers(-6, 7, d)
            if int(np.dot(h, z)) % n == 0:
                h[0] += 1
        params = np.concatenate([[u], 2 * math.pi * h.astype(float)])
        q, _ = O.lattice_sum(z, n, O.OSCILLATORY, params, shift)
        in_dual = int(np.dot(h.astype(object), z.astype(object))) % n == 0
        expect = math.cos(2 * math.pi * u + 2 * math.pi * float(np.dot(h, delta))) if in_dual else 0.0
        assert abs(q - expect) < 1e-9, (h, q, expect)


# ---- one-dimensional closed forms ------------------------------------------------
@pytest.mark.parametrize("n,c", [(1, 0.7), (7, 1.3), (1009, 0.25), (65537, -2.0)])
def test_left_rectangle_geometric_sum(n, c):
    """d = 1, z = 1: (1/n) sum_k e^{c k/n} = (e^c - 1) / (n (e^{c/n} - 1))."""
    q, _ = O.lattice_sum([1 % n], n, O.EXP_SUM, [c])
    expect = math.expm1(c) / (n * math.expm1(c / n))
    assert q == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("n,c,i0,m", [(1, 0.7, 0, 1), (7, 1.3, 2, 4), (1009, 0.25, 0, 1009),
                                       (1009, -0.8, 500, 1), (65537, -2.0, 1234, 40000)])
def test_partial_sum_geometric_closed_form(n, c, i0, m):
    """d = 1, z = 1: the indices i0 .. i0+m-1 (< n) are their own residues, so the
    partial sum of e^{c k/n} is e^{c i0/n} (e^{c m/n} - 1) / (e^{c/n} - 1)."""
    s = O.lattice_partial([1 % n], n, O.EXP_SUM, [c], i0, m)
    expect = math.exp(c * i0 / n) * math.expm1(c * m / n) / math.expm1(c / n)
    assert s == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("shifted", [False, True])
def test_partial_sums_over_a_split_add_up(family, shifted):
    """Partial sums over any split of [0, n) add up to n Q of the full rule; the
    whole range is the full rule's own sum (the same additions in the same order)."""
    p = W.random_plain(40 + family, family, 5, 4099, shift=shifted)
    z = O.korobov(p.d, p.n, p.a)
    q, a = O.lattice_sum(z, p.n, p.family, p.params, p.shift)
    cuts = np.sort(np.random.default_rng(family).choice(np.arange(1, p.n), 6, replace=False))
    edges = [0, *cuts.tolist(), p.n]
    parts = [O.lattice_partial(z, p.n, p.family, p.params, lo, hi - lo, p.shift)
             for lo, hi in zip(edges[:-1], edges[1:])]
    assert math.fsum(parts) == pytest.approx(p.n * q, abs=1e-14 * p.n * a)
    assert O.lattice_partial(z, p.n, p.family, p.params, 0, p.n, p.shift) / p.n == q
    assert O.lattice_partial(z, p.n, p.family, p.params, 17, 0, p.shift) == 0.0
    with pytest.raises(ValueError):
        O.lattice_partial(z, p.n, p.family, p.params, p.n - 3, 4, p.shift)


@pytest.mark.parametrize("N", [1, 2, 5, 64, 1000])
def test_midpoint_closed_forms(N):
    """M = (1/N) sum_s e^{c (s+1/2)/N} = (e^c - 1) / (2 N sinh(c / 2N)); the complex
    analogue gives e^{i c/2} sin(c/2) / (N sin(c / 2N)).  Products over d = 3."""
    cs = [0.4, -1.7, 2.9]
    expect = math.prod(math.expm1(c) / (2 * N * math.sinh(c / (2 * N))) for c in cs)
    assert O.mdi_lr([N] * 3, O.EXP_SUM, cs) == pytest.approx(expect, rel=1e-13)
    u = 0.17
    z = complex(math.cos(2 * math.pi * u), math.sin(2 * math.pi * u))
    for c in cs:
        z *= complex(math.cos(c / 2), math.sin(c / 2)) * math.sin(c / 2) / (N * math.sin(c / (2 * N)))
    got = O.mdi_lr([N] * 3, O.OSCILLATORY, [u] + cs)
    assert got == pytest.approx(z.real, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
def test_half_shifted_1d_lattice_is_midpoint_rule(family):
    """d = 1, z = 1, Delta = 1/(2n): the lattice points are the midpoints (k + 1/2)/n,
    so the plain rule equals the MDI-LR tensor rule with N_1 = n."""
    rng = np.random.default_rng(family)
    p = W.draw_params(rng, family, 1)
    n = 997
    q, _ = O.lattice_sum([1], n, family, p, shift=[0.5 / n])
    assert q == pytest.approx(O.mdi_lr([n], family, p), rel=1e-13, abs=1e-15)


# ---- brute force for the MDI-LR sweep --------------------------------------------
@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("N", [[7], [4, 9], [3, 1, 6], [5, 4, 3, 7], [12, 12, 12, 12]])
def test_mdi_sweep_matches_brute_force(family, N):
    rng = np.random.default_rng(len(N) * 10 + family)
    p = W.draw_params(rng, family, len(N))
    brute = O.mdi_lr_brute(N, family, p)
    scale = max(abs(brute), 1e-3)
    assert abs(O.mdi_lr(N, family, p) - brute) <= 1e-13 * scale


def test_mdi_sweep_survives_d1000_underflow_range():
    """d = 1000 Gaussian factors ~ e^-0.3 each: the product ~ 1e-130 stays exact
    in the exponent-tracked sweep and equals the product of the 1-D factors."""
    d = 1000
    p = np.concatenate([np.full(d, 1.0), np.full(d, 0.9)])
    re, _ = O.mdi_lr_factors(np.full(d, 16), O.GAUSSIAN, p)
    lg = float(np.sum(np.log(re)))
    got = O.mdi_lr(np.full(d, 16), O.GAUSSIAN, p)
    assert math.log(got) == pytest.approx(lg, rel=1e-13)


def _gauss_integral_and_midpoint_error(c, w, N):
    """Closed form of int_[0,1]^d exp(-sum c_j^2 (x_j - w_j)^2) dx and the relative error
    of the tensor midpoint rule predicted by the first Euler-Maclaurin term of each
    direction, -(h^2/24) (phi'(1) - phi'(0)) / I_j with phi'(x) = -2 c^2 (x - w) phi(x)."""
    h = 1.0 / N
    exact, pred = 1.0, 1.0
    for cj, wj in zip(c, w):
        Ij = math.sqrt(math.pi) / (2 * cj) * (math.erf(cj * (1 - wj)) + math.erf(cj * wj))
        dphi = -2 * cj * cj * ((1 - wj) * math.exp(-cj * cj * (1 - wj) ** 2) + wj * math.exp(-cj * cj * wj * wj))
        exact *= Ij
        pred *= 1 - h * h / 24 * dphi / Ij
    return exact, pred - 1


def test_mdi_lr_d100_gaussian_against_closed_form():
    """The MDI-LR workload's set 0 (d = 100, N = 64): the oracle's relative error against
    the exact integral is the midpoint rule's Euler-Maclaurin prediction to 1e-4 of itself
    (the next term is O(h^4))."""
    m = W.mdi_d100_gauss(nsets=1)
    d = m.d
    exact, pred = _gauss_integral_and_midpoint_error(m.params[0][:d], m.params[0][d:], 64)
    err = O.mdi_lr(m.N, m.family, m.params[0]) / exact - 1
    assert abs(err / pred - 1) < 1e-4, (err, pred)


# ---- exp of a signed quadratic (Test 7's f_5) ------------------------------------
def test_exp_quadratic_with_negative_weights_is_the_gaussian():
    """c_j = -g_j^2 makes exp(sum_j c_j (x_j - w_j)^2) the Gaussian family with widths g."""
    rng = np.random.default_rng(11)
    d, n = 5, 1009
    g, w = rng.uniform(0.2, 1.5, d), rng.uniform(0, 1, d)
    z, shift = O.korobov(d, n, 389), rng.uniform(0, 1, d)
    pq, pg = np.concatenate([-g * g, w]), np.concatenate([g, w])
    q = O.lattice_sum(z, n, O.EXP_QUADRATIC, pq, shift)[0]
    assert q == pytest.approx(O.lattice_sum(z, n, O.GAUSSIAN, pg, shift)[0], rel=1e-14)
    N = [5, 8, 3, 7, 6]
    assert O.mdi_lr(N, O.EXP_QUADRATIC, pq) == pytest.approx(O.mdi_lr(N, O.GAUSSIAN, pg), rel=1e-14)


@pytest.mark.parametrize("N", [16, 64, 256])
def test_f5_mdi_lr_against_erf_erfi_closed_form(N):
    """f_5 = exp(sum_j (-1)^{j+1} x_j^2): MDI-LR is the tensor midpoint rule, a product of
    1-D midpoint sums of exp(s x^2), s = +-1, whose integrals are (sqrt(pi)/2) erfi(1) and
    (sqrt(pi)/2) erf(1).  The midpoint rule's Euler-Maclaurin expansion gives each factor
    as I - (h^2/24) D1 + (7 h^4/5760) D3 + O(h^6), with h = 1/N and the end-point
    differences D1 = f'(1) - f'(0) = 2 s e^s, D3 = f'''(1) - f'''(0) = (12 + 8 s) e^s."""
    d = 6
    s = np.array([(-1.0) ** j for j in range(d)])
    p = np.concatenate([s, np.zeros(d)])
    h = 1.0 / N
    fac = []
    for sj in s:
        exact = math.sqrt(math.pi) / 2 * (float(mp.erfi(1)) if sj > 0 else math.erf(1.0))
        e = math.exp(sj)
        fac.append(exact - h * h / 24 * 2 * sj * e + 7 * h ** 4 / 5760 * (12 + 8 * sj) * e)
    q = O.mdi_lr([N] * d, O.EXP_QUADRATIC, p)
    assert q == pytest.approx(math.prod(fac), rel=max(d * h ** 6, 1e-13))
    # the h^4 term is resolved: dropping it misses by more than the tolerance
    if N == 16:
        lead = math.prod(f - 7 * h ** 4 / 5760 * (12 + 8 * sj) * math.exp(sj) for f, sj in zip(fac, s))
        assert abs(q - lead) > d * h ** 6 * abs(q)


# ---- gradients --------------------------------------------------------------------
@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
def test_gradient_matches_central_differences(family):
    rng = np.random.default_rng(100 + family)
    d, n = 3, 257
    z = O.korobov(d, n, 76)
    p = W.draw_params(rng, family, d)
    shift = rng.uniform(0, 1, d)
    q, g = O.lattice_grad(z, n, family, p, shift)
    q2, _ = O.lattice_sum(z, n, family, p, shift)
    assert q == q2
    for k in range(p.size):
        h = 1e-5 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (O.lattice_sum(z, n, family, pp, shift)[0] - O.lattice_sum(z, n, family, pm, shift)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-8), k


def test_gradient_character_identity_u():
    """d/du of the character sum is -2 pi sin(2 pi u + 2 pi h.Delta) for h in the dual."""
    n, d = 1009, 3
    z = O.korobov(d, n, 331)
    rng = np.random.default_rng(5)
    h = _dual_vector(rng, z, n)
    shift = rng.uniform(0, 1, d)
    u = 0.41
    params = np.concatenate([[u], 2 * math.pi * h.astype(float)])
    _, g = O.lattice_grad(z, n, O.OSCILLATORY, params, shift)
    expect = -2 * math.pi * math.sin(2 * math.pi * u + 2 * math.pi * float(np.dot(h, shift)))
    assert g[0] == pytest.approx(expect, abs=1e-9)


# ---- sanity of the workloads against their exact integrals ----------------------
def test_workload_plain_d4_expsum_near_integral():
    w = W.plain_d4_expsum()
    z = O.korobov(w.d, w.n, w.a)
    q, _ = O.lattice_sum(z, w.n, w.family, w.params)
    exact = math.prod(math.expm1(c) / c for c in w.params)
    assert abs(q - exact) / exact < 2e-2


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        O.lattice_sum([5], 5, O.EXP_SUM, [1.0])  # z_j must be < n
    with pytest.raises(ValueError):
        O.lattice_sum([1], 5, O.EXP_SUM, [1.0], shift=[1.0])  # shift in [0, 1)
    with pytest.raises(ValueError):
        O.mdi_lr([0], O.EXP_SUM, [1.0])


# ---- the shifted lattice: wrap into [0, 1) -----------------------------------------
@pytest.mark.parametrize("family", [0, 1, 2])
def test_shift_by_own_point_permutes_lattice(family):
    """Shifting a rank-1 lattice by one of its own points maps the point set onto
    itself ({x_i + x_s} = x_{i+s}), so the rule is unchanged -- for integrands that
    are not periodic this only holds if the shift wraps into [0, 1)."""
    n, d = 1009, 4
    z = O.korobov(d, n, 331)
    rng = np.random.default_rng(7 + family)
    p = W.draw_params(rng, family, d)
    q0, _ = O.lattice_sum(z, n, family, p)
    for s in (1, 500, 1008):
        shift = O.lattice_points(z, n, s, 1)[0] / n
        qs, _ = O.lattice_sum(z, n, family, p, shift)
        assert qs == pytest.approx(q0, rel=1e-13)


@pytest.mark.parametrize("m", [0, 137, 996])
def test_rotated_midpoint_shift(m):
    """d = 1, z = 1, Delta = (m + 1/2)/n: the shifted points are the midpoints in
    rotated order, so the rule equals the midpoint rule for a non-periodic f."""
    n = 997
    q, _ = O.lattice_sum([1], n, O.EXP_SUM, [1.7], shift=[(m + 0.5) / n])
    assert q == pytest.approx(O.mdi_lr([n], O.EXP_SUM, [1.7]), rel=1e-13)
