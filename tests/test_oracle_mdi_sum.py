"""Pins of the oracle's MDI-LR for integrands of the coordinate sum (Test 7's
f_6 = (1 + sum x)^-(d+1)) on the improved tensor midpoint rule.

  * the merged-state dimension iteration against brute force over the grid;
  * the number of index tuples per merged state against the inclusion-exclusion
    count of compositions of T into k parts in [0, N-1];
  * exact moments of the midpoint grid: g(s) = b + c s (power -1) integrates to
    b + c d/2, g(s) = (b + c s)^2 (power -2) to b^2 + b c d + c^2 (Var + d^2/4) with
    Var = sum_k (1 - 1/N_k^2)/12;
  * a Gaussian of the sum with c = 0 integrates to 1.
"""
from __future__ import annotations

from math import comb

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("gfam,gp", [(0, [1.0, 1.0, 5.0]), (0, [0.5, 2.0, 1.5]), (1, [1.3, 1.1])])
@pytest.mark.parametrize("d,N,N_last", [(1, 7, 7), (2, 5, 6), (3, 4, 4), (4, 3, 5), (3, 8, 2)])
def test_sweep_matches_brute_force(gfam, gp, d, N, N_last):
    if d == 1:
        N = N_last
    assert O.mdi_sum(d, N, N_last, gfam, gp) == pytest.approx(O.mdi_sum_brute(d, N, N_last, gfam, gp),
                                                             rel=1e-13)


def _compositions(T, k, N):
    return sum((-1) ** i * comb(k, i) * comb(T - i * N + k - 1, k - 1)
               for i in range(0, k + 1) if T - i * N >= 0)


@pytest.mark.parametrize("k,N", [(1, 5), (4, 4), (7, 3), (3, 10), (12, 2)])
def test_state_counts_are_bounded_compositions(k, N):
    _, counts = O.mdi_sum(k + 1, N, 3, 0, [1.0, 1.0, 1.0], counts=True)
    expect = np.array([_compositions(T, k, N) for T in range(k * (N - 1) + 1)], dtype=np.float64)
    # the iteration carries fractions (divided by N each step); scaled back by N^k
    # they are the integers to rounding
    assert np.max(np.abs(counts - expect) / expect) <= 1e-13
    assert counts.sum() == pytest.approx(N ** k, rel=1e-13)


@pytest.mark.parametrize("d,N,N_last", [(1, 9, 9), (5, 7, 8), (20, 16, 17), (100, 64, 64)])
def test_exact_moments_of_the_midpoint_grid(d, N, N_last):
    b, c = 0.75, 1.25
    q1 = O.mdi_sum(d, N, N_last, 0, [b, c, -1.0])
    assert q1 == pytest.approx(b + c * d / 2, rel=1e-13)
    var = (d - 1) * (1 - 1 / N ** 2) / 12 + (1 - 1 / N_last ** 2) / 12
    q2 = O.mdi_sum(d, N, N_last, 0, [b, c, -2.0])
    assert q2 == pytest.approx(b * b + b * c * d + c * c * (var + d * d / 4), rel=1e-12)


def test_flat_gaussian_integrates_to_one():
    assert O.mdi_sum(30, 10, 11, 1, [0.0, 3.0]) == pytest.approx(1.0, rel=1e-14)


def test_rejects_bad_arguments():
    with pytest.raises(Exception):
        O.mdi_sum(0, 4, 4, 0, [1.0, 1.0, 1.0])
    with pytest.raises(Exception):
        O.mdi_sum(3, 4, 4, 2, [1.0, 1.0, 1.0])


# One direction with N = 2^14 nodes: the midpoint rule is I - (g'(1) - g'(0)) / (24 N^2)
# up to O(N^-4) (Euler-Maclaurin), so the leading correction is included.
NN = 1 << 14


@pytest.mark.parametrize("c,w", [(1.3, 0.4), (3.0, 0.9)])
def test_one_dimensional_gaussian_of_the_sum_converges_to_its_integral(c, w):
    from math import erf, exp, pi, sqrt
    exact = sqrt(pi) / (2 * c) * (erf(c * (1 - w)) + erf(c * w))
    dg = lambda s: -2 * c * c * (s - w) * exp(-c * c * (s - w) ** 2)
    mid = exact - (dg(1.0) - dg(0.0)) / (24 * NN * NN)
    assert O.mdi_sum(1, NN, NN, 1, [c, w]) == pytest.approx(mid, rel=1e-12)


@pytest.mark.parametrize("b,c,p", [(1.0, 1.0, 2.0), (0.5, 2.0, 3.5), (2.0, 0.5, 0.25)])
def test_one_dimensional_power_of_the_sum_converges_to_its_integral(b, c, p):
    exact = ((b + c) ** (1 - p) - b ** (1 - p)) / (c * (1 - p))
    dg = lambda s: -p * c * (b + c * s) ** (-p - 1)
    mid = exact - (dg(1.0) - dg(0.0)) / (24 * NN * NN)
    assert O.mdi_sum(1, NN, NN, 0, [b, c, p]) == pytest.approx(mid, rel=1e-12)
