"""Parity of the improved rule's tensor grid (qmc_implr_grid, qmc_implr_points)
with the oracle (Theorem 3.1, eq. 3.5, Lemma 3.2, Fig. 5).

Integer work only, so every comparison is exact: the grid ranks s against the
oracle's numerators u (u_i = z_i s_i for the Korobov z), the per-direction counts
against eq. 3.5, and n* -- by both methods, the order check and the bitmap --
against the grid size minus the oracle's number of distinct transformed points.
At the full sizes (up to 2^31 - 1 points) sampled points are compared one by
one, and n* against the closed form prod(n_i) - n that the oracle's
lexicographic-order pin establishes.
"""
import numpy as np
import pytest

import oracle as O
from paper_2404_08867_amd import qmc

pytestmark = pytest.mark.gpu

# (d, n, a): Fig. 5, gcd(a, n) > 1, n = a^d (Lemma 3.2), d = 1, a = 1, several
# thousand threads with a ragged last run, n = a^d + 1
SMALL = [(2, 81, 7), (3, 1200, 6), (3, 1000, 10), (1, 997, 5), (64, 1000, 1), (4, 1048573, 100),
         (5, 1025, 4), (2, 65537, 256), (3, 1332, 11), (6, 733, 3), (2, 3, 2)]


@pytest.mark.parametrize("d,n,a", SMALL)
def test_points_match_oracle(d, n, a):
    z = O.korobov(d, n, a)
    s = qmc.implr_points(d, n, a, 0, n).cpu().numpy().astype(np.int64).T
    assert np.array_equal(s * z, O.implr_coords(z, n))


METHODS = [qmc.IMPLR_AUTO, qmc.IMPLR_BITMAP]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("d,n,a", SMALL)
def test_grid_matches_oracle(d, n, a, method):
    z = O.korobov(d, n, a)
    counts, nstar = qmc.implr_grid(d, n, a, method)
    eq35 = O.mdi_dims(z, n)
    assert np.array_equal(counts, eq35)
    _, _, distinct = O.implr_grid(z, n)
    assert int(nstar.item()) == int(np.prod(eq35)) - distinct


@pytest.mark.parametrize("method", METHODS)
def test_figure5(method):
    counts, nstar = qmc.implr_grid(2, 81, 7, method)
    assert list(counts) == [7, 12] and int(nstar.item()) == 3


def test_repeated_calls_reuse_the_workspace():
    # the workspace is not zero-filled and keeps the previous call's bitmap
    ws = qmc.Workspace(qmc.implr_workspace_size(4, 1048573, 100))
    ws.buf.fill_(0xA5)
    for (d, n, a), m in zip([(4, 1048573, 100), (2, 81, 7), (4, 1048573, 100), (5, 1025, 4)],
                            [qmc.IMPLR_BITMAP, qmc.IMPLR_AUTO, qmc.IMPLR_BITMAP, qmc.IMPLR_BITMAP]):
        _, nstar = qmc.implr_grid(d, n, a, m, ws=ws)
        z = O.korobov(d, n, a)
        assert int(nstar.item()) == int(np.prod(O.mdi_dims(z, n))) - n


def test_points_subrange_and_empty():
    d, n, a = 4, 1048573, 100
    z = O.korobov(d, n, a)
    s = qmc.implr_points(d, n, a, 1000, 777).cpu().numpy().astype(np.int64).T
    assert np.array_equal(s * z, O.implr_coords_at(z, n, np.arange(1000, 1777)))
    assert qmc.implr_points(d, n, a, n, 0).numel() == 0


@pytest.mark.parametrize("d,a,extra,method", [(3, 1290, 1, qmc.IMPLR_AUTO), (3, 1290, 1, qmc.IMPLR_BITMAP),
                                              (3, 1290, 0, qmc.IMPLR_AUTO), (2, 46340, None, qmc.IMPLR_AUTO),
                                              (30, 2, None, qmc.IMPLR_AUTO)])
def test_full_size(d, a, extra, method):
    n = a ** d + extra if extra is not None else 2147483647
    z = O.korobov(d, n, a)
    counts, nstar = qmc.implr_grid(d, n, a, method)
    eq35 = O.mdi_dims(z, n)
    assert np.array_equal(counts, eq35)
    assert int(nstar.item()) == int(np.prod(eq35)) - n
    if extra == 1:
        assert int(nstar.item()) == a ** (d - 1) - 1
    if extra == 0:
        assert int(nstar.item()) == 0
    rng = np.random.default_rng(d * 7919 + a)
    for j0 in [0, n // 2 - 5, n - 4096] + list(rng.integers(0, n - 4096, 3)):
        j0 = int(j0)
        s = qmc.implr_points(d, n, a, j0, 4096).cpu().numpy().astype(np.int64).T
        assert np.array_equal(s * z, O.implr_coords_at(z, n, np.arange(j0, j0 + 4096))), j0


def test_points_ragged_and_unaligned_ranges():
    # ranges that start inside a wave's block and end inside a step
    d, n, a = 3, 1000003, 97
    z = O.korobov(d, n, a)
    for j0, count in [(1, 1), (63, 65), (4095, 4098), (n - 1, 1), (n - 4097, 4097), (12345, 100000)]:
        s = qmc.implr_points(d, n, a, j0, count).cpu().numpy().astype(np.int64).T
        assert np.array_equal(s * z, O.implr_coords_at(z, n, np.arange(j0, j0 + count))), (j0, count)


def test_points_unaligned_output_rows():
    # ld not a multiple of 4, and a base 4 bytes past a 16-byte boundary
    import torch
    d, n, a = 3, 1000003, 97
    z = O.korobov(d, n, a)
    count = 70001
    want = O.implr_coords_at(z, n, np.arange(500, 500 + count))
    for ld, off in [(count + 1, 0), (count + 4, 1)]:
        big = torch.full((d, ld + off), -1, dtype=torch.int32, device="cuda")
        out = big[:, off:]
        s = qmc.implr_points(d, n, a, 500, count, out=out).cpu().numpy().astype(np.int64).T
        assert np.array_equal(s * z, want), (ld, off)
        rest = big[:, off + count:].cpu().numpy()
        assert np.all(rest == -1)  # nothing written past count


def test_grid_count_replays_in_a_graph():
    # all counters are reset by the launches themselves (no memset): a captured
    # call gives the same n* on every replay, with eager calls in between
    import torch
    d, n, a = 4, 1048573, 100
    ws = qmc.Workspace(qmc.implr_workspace_size(d, n, a))
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    want = int(np.prod(O.mdi_dims(O.korobov(d, n, a), n))) - n
    for method in METHODS:
        qmc.implr_grid(d, n, a, method, ws=ws, out=out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g):
                qmc.implr_grid(d, n, a, method, ws=ws, out=out)
        torch.cuda.current_stream().wait_stream(side)
        for rep in range(3):
            out.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            assert int(out.item()) == want, (method, rep)
            _, eager = qmc.implr_grid(3, 1332, 11, method, ws=ws)  # other work in between
            assert int(eager.item()) == 11 * 11 * 12 - 1332
