"""Pins of the oracle's randomly shifted lattice rule (Sec. 2.1: the shifted lattice
P + Delta, averaged over random shifts).

The oracle is checked against closed forms, not against a retyped copy of itself:
  * a one-dimensional lattice {i/n} shifted by r/(R n), r = 0..R-1, is the
    left-rectangle rule with n R points, so the mean over the R shifts of the
    exp-sum rule is a geometric series;
  * the same grid reached through shifts that wrap past 1;
  * two shifts 0 and 1/(2n): left-endpoint and midpoint rules, whose standard
    error of the mean is half their difference;
  * identical shifts give a standard error of exactly zero.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
import pytest

import oracle as O

mp.mp.dps = 40


def _geometric_mean_rule(c: float, m: int) -> float:
    """(1/m) sum_{k=0}^{m-1} exp(c k / m) in high precision."""
    c = mp.mpf(c)
    return float((mp.e ** c - 1) / (m * (mp.e ** (c / m) - 1))) if c != 0 else 1.0


@pytest.mark.parametrize("n,R,c", [(7, 1, 0.7), (7, 3, 0.7), (101, 8, -1.3), (1009, 5, 2.0)])
def test_fine_grid_of_shifts_is_the_refined_rectangle_rule(n, R, c):
    shifts = np.array([[r / (R * n)] for r in range(R)])
    q, mean, se = O.shift_ensemble([1], n, 0, [c], shifts)
    assert mean == pytest.approx(_geometric_mean_rule(c, n * R), rel=1e-14)
    # each shifted rule is itself the n-point rectangle rule moved by r/(Rn)
    for r in range(R):
        assert q[r] == pytest.approx(_geometric_mean_rule(c, n) * np.exp(c * r / (R * n)), rel=1e-14)


@pytest.mark.parametrize("n,R,c", [(7, 4, 0.9), (211, 6, -0.4)])
def test_wrapped_shifts_cover_the_same_grid(n, R, c):
    # Delta_r = 1 - (r+1)/(Rn): every point but i = 0 wraps past 1, and the union of
    # the R shifted lattices is again the grid {m / (nR)}.
    shifts = np.array([[1.0 - (r + 1) / (R * n)] for r in range(R)])
    _, mean, _ = O.shift_ensemble([1], n, 0, [c], shifts)
    assert mean == pytest.approx(_geometric_mean_rule(c, n * R), rel=1e-14)


@pytest.mark.parametrize("n,c", [(5, 1.1), (97, -2.5)])
def test_two_shift_standard_error(n, c):
    q0 = _geometric_mean_rule(c, n)
    q1 = float(mp.e ** (mp.mpf(c) / (2 * n))) * q0  # midpoint rule
    q, mean, se = O.shift_ensemble([1], n, 0, [c], [[0.0], [0.5 / n]])
    assert q[0] == pytest.approx(q0, rel=1e-14)
    assert q[1] == pytest.approx(q1, rel=1e-14)
    assert mean == pytest.approx(0.5 * (q0 + q1), rel=1e-14)
    assert se == pytest.approx(0.5 * abs(q1 - q0), rel=1e-10)


@pytest.mark.parametrize("family", [0, 1, 2, 3, 4])
def test_identical_shifts_have_zero_standard_error(family):
    d, n = 3, 211
    z = O.korobov(d, n, 17)
    rng = np.random.default_rng(5)
    params = rng.random(O.param_count(family, d)) + 0.5
    shift = rng.random(d)
    q, mean, se = O.shift_ensemble(z, n, family, params, np.tile(shift, (4, 1)))
    assert np.all(q == q[0]) and mean == q[0] and se == 0.0
    q1, m1, se1 = O.shift_ensemble(z, n, family, params, shift[None, :])
    assert q1[0] == q[0] and m1 == q[0] and se1 == 0.0


def test_shift_ensemble_rejects_bad_arguments():
    with pytest.raises(Exception):
        O.shift_ensemble([1], 7, 0, [1.0], np.zeros((0, 1)))
    with pytest.raises(Exception):
        O.shift_ensemble([1], 7, 0, [1.0], [[1.5]])
