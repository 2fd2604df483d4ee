"""The exact-float index step of the FP32 product-peak kernels, checked on the host.

For n <= 2^24 the kernels hold a lattice index k in [0, n) as a float and step it
by D = 64 z mod n as the unsigned minimum of the bit patterns of k + D and
k + (D - n): when k + D < n both sums are exact and the negative one has the larger
pattern; otherwise k + D - n is exact and k + D, rounded or not, is not smaller.  IEEE single precision with round-to-nearest is the same
here as on the device, so numpy float32 reproduces the step bit for bit.
"""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _step(k, dp, dm):
    a = (k + dp).view(np.uint32)
    b = (k + dm).view(np.uint32)
    return np.minimum(a, b).view(np.float32)


def _check(n, k, D, steps=1):
    kf = k.astype(np.float32)
    dp = D.astype(np.float32)
    dm = dp - np.float32(n)
    ki = k.copy()
    for _ in range(steps):
        kf = _step(kf, dp, dm)
        ki = (ki + D) % n
    return np.array_equal(kf.view(np.uint32), ki.astype(np.float32).view(np.uint32))


def test_bound_in_the_kernel_source():
    src = open(os.path.join(ROOT, "paper_2404_08867_amd", "csrc", "common.hpp")).read()
    m = re.search(r"kFloatIndexMaxN\s*=\s*1u\s*<<\s*(\d+)", src)
    assert m and int(m.group(1)) == 24


def test_every_pair_for_small_n():
    for n in (1, 2, 3, 7, 64, 257, 1009):
        k, D = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        assert _check(n, k.ravel(), D.ravel()), n


def test_random_and_edge_pairs_up_to_the_bound():
    rng = np.random.default_rng(7)
    for n in (65521, 1048573, 8388593, 1 << 23, 16777213, (1 << 24) - 1, 1 << 24):
        k = rng.integers(0, n, 400_000)
        D = rng.integers(0, n, 400_000)
        edges = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (0, 1), (n - 1, 1), (1, n - 1)]
        k[:len(edges)] = [e[0] for e in edges]
        D[:len(edges)] = [e[1] for e in edges]
        assert _check(n, k, D, steps=16), n


def test_the_bound_is_needed():
    # Above 2^24, n and the residues themselves lose their last bit.
    assert not _check((1 << 24) + 1, np.array([16155603]), np.array([2478351]))
    assert not _check((1 << 24) + 1, np.array([1 << 24]), np.array([0]))
