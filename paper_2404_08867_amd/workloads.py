"""Seeded synthetic inputs for the lattice-sum workloads.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no generating vector, no lattice index, no integrand
value).  It is the only module shared by the HIP path's tests/benchmark and the
CPU oracle's tests.

The paper (Zhong & Feng, arXiv 2404.08867) uses no dataset; its experiments are
closed-form integrands on Korobov lattices (Sec. 4-6).  The workloads below keep
those shapes -- Korobov parameter a, dimension d, prime point counts n, product
or additive integrands with per-direction parameters -- with parameters drawn
from fixed seeds:

  * generator: ``numpy.random.default_rng(seed)`` (PCG64);
  * seed of workload k: ``2404088670 + k``;
  * draw order: a, then c, then w, then u.

Workloads (k = 0..7):
  0 plain_d4_expsum      d=4,   n=1009,      exp-sum, c ~ U[0,1]
  1 plain_d20_peak       d=20,  n=1048573,   product-peak, c ~ U[0.5,2], w ~ U[0,1]
  2 mdi_d100_gauss       d=100, N=64 nodes per direction (a = N), Gaussian,
                         c ~ U[0.1,1], w ~ U[0,1]; extra sets for throughput
  3 batched_4096         4096 integrands, d ~ U{8..200}, n uniform over the primes
                         in [2^12, 2^22], a ~ U{2..n-1}, family uniform over
                         {exp-sum, product-peak, Gaussian} with the parameter laws above
  4 adjoint_d50_osc      d=50, n=16777213, one a shared by 64 oscillatory sets,
                         u ~ U[0,1], c ~ U[0,2]
  5 shifts_d20_peak      the plain_d20_peak problem (its own seed) with R = 64
                         shifts Delta_r ~ U[0,1)^20 (random-shift ensemble)
  6 mdi_sum_d100         MDI-LR of g(sum x), d=100, N=64 nodes in every direction,
                         power g(s) = (b + c s)^-p; set 0 is Test 7's f_6
                         (b = c = 1, p = d + 1), sets s >= 1 draw b ~ U[0.5,2],
                         c ~ U[0.5,1.5], p ~ U[1, d+1]
  7 plain_d20_f5         d=20, n=1048573, Test 7's f_5 (exp of a signed quadratic,
                         c = +-1 alternating, w = 0); only a is drawn
Lattice constructions (no random draws):
    korobov_search_d20   e^2 of eq. 2.12 for z(a), d=20, n=65521 (the largest
                         prime below 2^16), product weights gamma_j = j^-2,
                         unanchored (beta = 0), every a in [1, (n-1)/2] (a and
                         n-a tie).  (Unit weights would make every candidate's
                         P_2 about (1 + pi^2/3)^20 / n: the k = 0 term.)
    cbc_d20              CBC for the same e^2, d=20, n=65521
    implr_d3             Theorem 3.1's grid for a = 1290, d = 3,
                         n = a^3 + 1 = 2146689001 (largest 1 + a^3 below 2^31)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2404088670

# Family ids (the same numbering as the C ABI and the oracle).
EXP_SUM, PRODUCT_PEAK, GAUSSIAN, OSCILLATORY, EXP_QUADRATIC = 0, 1, 2, 3, 4
FAMILY_NAMES = {EXP_SUM: "exp_sum", PRODUCT_PEAK: "product_peak", GAUSSIAN: "gaussian",
                OSCILLATORY: "oscillatory", EXP_QUADRATIC: "exp_quadratic"}


def param_count(family: int, d: int) -> int:
    """Length of the FP64 parameter vector: c | c,w | c,w | u,c | c,w."""
    return {EXP_SUM: d, PRODUCT_PEAK: 2 * d, GAUSSIAN: 2 * d, OSCILLATORY: d + 1,
            EXP_QUADRATIC: 2 * d}[family]


def draw_params(rng: np.random.Generator, family: int, d: int) -> np.ndarray:
    """One parameter vector with the paper-style laws used by the workloads."""
    if family == EXP_SUM:
        return rng.uniform(0.0, 1.0, d)
    if family == PRODUCT_PEAK:
        c = rng.uniform(0.5, 2.0, d)
        w = rng.uniform(0.0, 1.0, d)
        return np.concatenate([c, w])
    if family == GAUSSIAN:
        c = rng.uniform(0.1, 1.0, d)
        w = rng.uniform(0.0, 1.0, d)
        return np.concatenate([c, w])
    if family == OSCILLATORY:
        c = rng.uniform(0.0, 2.0, d)
        u = rng.uniform(0.0, 1.0, 1)
        return np.concatenate([u, c])
    if family == EXP_QUADRATIC:
        # signed weights, as in Test 7's f_5 (alternating +-1, w = 0)
        c = rng.uniform(-1.0, 1.0, d)
        w = rng.uniform(0.0, 1.0, d)
        return np.concatenate([c, w])
    raise ValueError(f"unknown family {family}")


def draw_coprime(rng: np.random.Generator, n: int) -> int:
    """A Korobov parameter a in [2, n-1] with gcd(a, n) = 1 (a = 1 when n <= 2)."""
    if n <= 2:
        return 1
    while True:
        a = int(rng.integers(2, n))
        if math.gcd(a, n) == 1:
            return a


def primes_between(lo: int, hi: int) -> np.ndarray:
    """All primes p with lo <= p <= hi (sieve of Eratosthenes)."""
    sieve = np.ones(hi + 1, dtype=bool)
    sieve[:2] = False
    for p in range(2, int(hi ** 0.5) + 1):
        if sieve[p]:
            sieve[p * p::p] = False
    idx = np.nonzero(sieve)[0]
    return idx[idx >= lo]


@dataclass
class Plain:
    """One plain lattice-sum problem: Korobov parameter a, not the vector z."""
    name: str
    d: int
    n: int
    a: int
    family: int
    params: np.ndarray
    shift: np.ndarray | None = None


@dataclass
class MdiSets:
    """MDI-LR problem: node counts per direction and nsets parameter vectors."""
    name: str
    d: int
    N: np.ndarray
    family: int
    params: np.ndarray  # [nsets, P]


@dataclass
class Batch:
    name: str
    problems: list = field(default_factory=list)


@dataclass
class ShiftEnsemble:
    """A plain problem evaluated on R shifted copies of its lattice."""
    name: str
    d: int
    n: int
    a: int
    family: int
    params: np.ndarray
    shifts: np.ndarray  # [R, d]


@dataclass
class AdjointSets:
    name: str
    d: int
    n: int
    a: int
    family: int
    params: np.ndarray  # [nsets, P]


def plain_d4_expsum() -> Plain:
    rng = np.random.default_rng(SEED_BASE + 0)
    n, d = 1009, 4
    a = int(rng.integers(2, n))
    c = rng.uniform(0.0, 1.0, d)
    return Plain("plain_d4_expsum", d, n, a, EXP_SUM, c)


def plain_d20_peak() -> Plain:
    rng = np.random.default_rng(SEED_BASE + 1)
    n, d = 1048573, 20
    a = int(rng.integers(2, n))
    c = rng.uniform(0.5, 2.0, d)
    w = rng.uniform(0.0, 1.0, d)
    return Plain("plain_d20_peak", d, n, a, PRODUCT_PEAK, np.concatenate([c, w]))


def plain_d20_f5() -> Plain:
    """Test 7's f_5 = exp(sum_j (-1)^{j+1} x_j^2) on the plain_d20_peak lattice size, as
    the exp of a signed quadratic (c = +1, -1, ..., w = 0); a from seed 7."""
    rng = np.random.default_rng(SEED_BASE + 7)
    n, d = 1048573, 20
    a = int(rng.integers(2, n))
    c = np.array([(-1.0) ** j for j in range(d)])
    return Plain("plain_d20_f5", d, n, a, EXP_QUADRATIC, np.concatenate([c, np.zeros(d)]))


def mdi_d100_gauss(nsets: int = 1) -> MdiSets:
    """Set 0 is the single seeded problem; set s does not depend on nsets."""
    rng = np.random.default_rng(SEED_BASE + 2)
    d, N = 100, 64
    r = rng.random((nsets, 2 * d))  # row s holds set s's draws: c then w
    c = 0.1 + 0.9 * r[:, :d]
    w = r[:, d:]
    return MdiSets("mdi_d100_gauss", d, np.full(d, N, dtype=np.int64), GAUSSIAN,
                   np.concatenate([c, w], axis=1))


def mdi_d100_gauss_plain_rule() -> Plain:
    """The plain rule beside the MDI-LR workload: set 0's Gaussian parameters on a
    Korobov lattice with n = 1048573 and a seeded a (its own stream of the same seed)."""
    w = mdi_d100_gauss(nsets=1)
    n = 1048573
    a = int(np.random.default_rng([SEED_BASE + 2, 1]).integers(2, n))
    return Plain("mdi_d100_gauss_plain_rule", w.d, n, a, GAUSSIAN, w.params[0].copy())


def batched_4096(count: int = 4096, d_range=(8, 200), n_range=(1 << 12, 1 << 22)) -> Batch:
    rng = np.random.default_rng(SEED_BASE + 3)
    primes = primes_between(*n_range)
    out = Batch("batched_4096")
    for b in range(count):
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        n = int(primes[rng.integers(0, primes.size)])
        a = int(rng.integers(2, n))
        fam = int(rng.integers(0, 3))  # exp-sum, product-peak, Gaussian
        out.problems.append(Plain(f"b{b}", d, n, a, fam, draw_params(rng, fam, d)))
    return out


def adjoint_d50_osc(nsets: int = 64) -> AdjointSets:
    rng = np.random.default_rng(SEED_BASE + 4)
    n, d = 16777213, 50
    a = int(rng.integers(2, n))
    r = rng.random((nsets, d + 1))  # row s holds set s's draws: c then u
    c = 2.0 * r[:, :d]
    u = r[:, d:]
    return AdjointSets("adjoint_d50_osc", d, n, a, OSCILLATORY, np.concatenate([u, c], axis=1))


def shifts_d20_peak(nshifts: int = 64) -> ShiftEnsemble:
    """Shift r does not depend on nshifts (row r of one draw)."""
    base = plain_d20_peak()
    rng = np.random.default_rng(SEED_BASE + 5)
    shifts = rng.random((nshifts, base.d))
    return ShiftEnsemble("shifts_d20_peak", base.d, base.n, base.a, base.family, base.params, shifts)


@dataclass
class MdiSum:
    name: str
    d: int
    N: int
    N_last: int
    gfamily: int
    params: np.ndarray  # [nsets, 3]


def mdi_sum_d100(nsets: int = 4096) -> MdiSum:
    """Set s does not depend on nsets (row s of one draw); row 0 is f_6."""
    d, N = 100, 64
    rng = np.random.default_rng(SEED_BASE + 6)
    r = rng.random((nsets, 3))
    params = np.stack([0.5 + 1.5 * r[:, 0], 0.5 + r[:, 1], 1.0 + d * r[:, 2]], axis=1)
    params[0] = (1.0, 1.0, d + 1.0)
    return MdiSum("mdi_sum_d100", d, N, N, 0, params)


@dataclass
class Search:
    name: str
    d: int
    n: int
    alpha: int
    a0: int
    count: int
    gamma: np.ndarray
    beta: float


@dataclass
class Cbc:
    name: str
    d: int
    n: int
    gamma: np.ndarray
    beta: float


def _inverse_square_weights(d: int) -> np.ndarray:
    return 1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2


def korobov_search_d20() -> Search:
    n, d = 65521, 20
    return Search("korobov_search_d20", d, n, 2, 1, (n - 1) // 2, _inverse_square_weights(d), 0.0)


def cbc_d20() -> Cbc:
    d = 20
    return Cbc("cbc_d20", d, 65521, _inverse_square_weights(d), 0.0)


@dataclass
class Implr:
    name: str
    d: int
    n: int
    a: int


def implr_d3() -> Implr:
    """Theorem 3.1's grid for the Korobov lattice with a = 1290, d = 3 and
    n = a^3 + 1 = 2146689001, the largest n = a^3 + 1 below 2^31 (the case
    n = 1 + a^d whose last direction has a + 1 nodes by eq. 3.5)."""
    a = 1290
    return Implr("implr_d3", 3, a ** 3 + 1, a)


def random_shifts(seed: int, nshifts: int, d: int) -> np.ndarray:
    """R uniform shifts in [0,1)^d for a small test case."""
    return np.random.default_rng(seed).random((nshifts, d))


def random_plain(seed: int, family: int, d: int, n: int, shift: bool = False) -> Plain:
    """A small seeded test problem (parity cases, edge cases)."""
    rng = np.random.default_rng(seed)
    a = draw_coprime(rng, n)
    p = draw_params(rng, family, d)
    s = rng.uniform(0.0, 1.0, d) if shift else None
    return Plain(f"rand{seed}", d, n, a, family, p, s)
