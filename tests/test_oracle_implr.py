"""Pins of the oracle's affine transformation (Theorem 3.1, eq. 3.1) and of the
improved rule's point count (Sec. 3.2).

  * the integer numerators of the transformed coordinates against the definition
    y = abs(A x + b), eq. 3.1, evaluated in exact rational arithmetic;
  * Fig. 5: the 81-point lattice with z = (1, 7) needs 3 added points;
  * the per-direction counts are those of eq. 3.5 (Theorem 3.1);
  * Lemma 3.2: for a Korobov lattice with n = a^d every direction has a values and
    the transformation is one-to-one onto the grid (no added point);
  * for a Korobov lattice with a^{d-1} < n the grid ranks (s_1, ..., s_d),
    s_i = u_i / z_i, grow strictly in lexicographic order with j (so the map is
    one-to-one and n* = prod(n_i) - n), brute force over every point.
"""
from __future__ import annotations

from fractions import Fraction
from math import floor

import numpy as np
import pytest

import oracle as O


def _frac(q: Fraction) -> Fraction:
    return q - floor(q)


def _transform_exact(z, n, j):
    """y_j = abs(A x_j + b) with x_j = {j z / n}, A and b of eq. 3.1."""
    d = len(z)
    x = [_frac(Fraction(j * zi, n)) for zi in z]
    y = []
    for i in range(d - 1):
        y.append(abs(x[i] / z[i] - x[i + 1] / z[i + 1]))
    b = -_frac(n * x[d - 1] / z[d - 1]) * Fraction(z[d - 1], n)
    y.append(abs(x[d - 1] + b))
    return y


@pytest.mark.parametrize("z,n", [([1, 7], 81), ([1, 4], 81), ([1, 4, 16], 161), ([1, 3, 9, 27], 100),
                                 ([1, 5], 37), ([2, 3, 11], 50)])
def test_coordinates_match_the_affine_definition(z, n):
    u = O.implr_coords(z, n)
    d = len(z)
    for j in range(n):
        y = _transform_exact(z, n, j)
        for i in range(d - 1):
            assert y[i] * z[i] * z[i + 1] == u[j, i], (j, i)
        assert y[d - 1] * n == u[j, d - 1], j


def test_figure5_needs_three_added_points():
    counts, nstar, distinct = O.implr_grid([1, 7], 81)
    assert nstar == 3 and distinct == 81
    assert list(counts) == [7, 12]


@pytest.mark.parametrize("d,n,a", [(2, 81, 4), (3, 161, 4), (4, 626, 5), (3, 1001, 10), (2, 1000, 31),
                                   (5, 244, 3)])
def test_counts_are_those_of_eq35(d, n, a):
    z = O.korobov(d, n, a)
    counts, nstar, distinct = O.implr_grid(z, n)
    assert np.array_equal(counts, O.mdi_dims(z, n))
    assert distinct == n and nstar == int(np.prod(counts)) - n


@pytest.mark.parametrize("d,a", [(2, 9), (3, 4), (4, 5), (6, 3)])
def test_lemma32_grid_is_exact_for_n_equal_a_to_the_d(d, a):
    n = a ** d
    counts, nstar, distinct = O.implr_grid(O.korobov(d, n, a), n)
    assert list(counts) == [a] * d and nstar == 0 and distinct == n


@pytest.mark.parametrize("z,n", [([3, 5, 7], 64), ([4, 6], 25), ([2, 3, 11], 50), ([1, 4, 16], 161)])
def test_grid_counts_by_brute_force_sets(z, n):
    # outside the Korobov setting the transformation can fold points together
    u = O.implr_coords(z, n)
    counts, nstar, distinct = O.implr_grid(z, n)
    assert distinct == len(set(map(tuple, u)))
    assert list(counts) == [len(set(u[:, i])) for i in range(len(z))]
    assert nstar == int(np.prod(counts)) - distinct


@pytest.mark.parametrize("d,n,a", [(2, 81, 7), (3, 1200, 6), (3, 1000, 10), (4, 10007, 21), (5, 1025, 4),
                                   (2, 4099, 64), (1, 97, 5), (6, 733, 3)])
def test_korobov_grid_ranks_increase_lexicographically(d, n, a):
    z = O.korobov(d, n, a)
    s = O.implr_coords(z, n) // z
    assert np.array_equal(s * z, O.implr_coords(z, n))
    for j in range(1, n):
        assert tuple(s[j - 1]) < tuple(s[j]), j
    counts, nstar, distinct = O.implr_grid(z, n)
    assert distinct == n and nstar == int(np.prod(counts)) - n


def test_coords_at_matches_the_full_table():
    z, n = O.korobov(4, 10007, 21), 10007
    u = O.implr_coords(z, n)
    js = np.array([0, 1, 5000, 9999, 10006, 17])
    assert np.array_equal(O.implr_coords_at(z, n, js), u[js])
