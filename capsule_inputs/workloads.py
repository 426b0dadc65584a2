"""Named synthetic workloads: the single-surface evaluations and request streams.

Every workload is formula-defined and seeded; nothing is read from disk.
delta = 2 h (the fixed global regularization delta = C' h_m with C' = 2,
Appendix "sensitivity to delta", last column), mu = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .forces import sh_force, uniform_force
from .surfaces import ELLIPSOID_SERVING, RBC, SPHERE, Shape, Surface, make_surface

SEED_C2 = 2_002
SEED_C3 = 3_003
SEED_C3_SUBSET = 3_303
SEED_C4 = 4_004
SEED_C5 = 5_005


@dataclass
class Problem:
    name: str
    surface: Surface
    f: np.ndarray          # (N, 3)
    delta: float
    mu: float = 1.0

    @property
    def N(self) -> int:
        return self.surface.N


def delta_2h(n: int) -> float:
    return 2.0 * math.pi / (n + 1)


def sphere_uniform(n: int = 18) -> Problem:
    """Unit sphere, uniform traction (0, 0, 1); exact surface velocity 2/3 e_z."""
    s = make_surface(SPHERE, n)
    return Problem(f"sphere_n{n}", s, uniform_force(s.N), delta_2h(n))


def rbc_sh(n: int, seed: int) -> Problem:
    s = make_surface(RBC, n)
    return Problem(f"rbc_n{n}", s, sh_force(s.x0, seed), delta_2h(n))


def shape_sh(shape: Shape, n: int, seed: int, name: str | None = None) -> Problem:
    s = make_surface(shape, n)
    return Problem(name or f"{shape.kind}_n{n}", s, sh_force(s.x0, seed), delta_2h(n))


def c1() -> Problem:
    return sphere_uniform(18)


def c2() -> Problem:
    return rbc_sh(64, SEED_C2)


def c3() -> Problem:
    return rbc_sh(256, SEED_C3)


def c3_subset(N: int = 6 * 256 * 256, k: int = 4096) -> np.ndarray:
    """4,096 target indices drawn without replacement for the large-N error check."""
    rng = np.random.default_rng(SEED_C3_SUBSET)
    return np.sort(rng.choice(N, size=k, replace=False))


# ----------------------------------------------------------------------------
# Request streams (serving).
# ----------------------------------------------------------------------------
SERVING_SHAPES = {"sphere": SPHERE, "ellipsoid": ELLIPSOID_SERVING, "rbc": RBC}


@dataclass
class Request:
    rid: int
    shape: str
    n: int
    seed: int
    arrival: float = 0.0     # seconds after stream start

    @property
    def N(self) -> int:
        return 6 * self.n * self.n

    def problem(self) -> Problem:
        return shape_sh(SERVING_SHAPES[self.shape], self.n, self.seed,
                        name=f"req{self.rid}_{self.shape}_n{self.n}")


@dataclass
class Stream:
    requests: list = field(default_factory=list)

    @property
    def pairs(self) -> int:
        return sum(r.N * r.N for r in self.requests)


def log_uniform_n(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def serving_stream(n_req: int = 256, n_lo: int = 16, n_hi: int = 192,
                   seed: int = SEED_C4, shapes=("sphere", "ellipsoid", "rbc")) -> Stream:
    """Requests with shape uniform over `shapes` and n log-uniform in [n_lo, n_hi].

    Arrival times are filled in by `poisson_arrivals` once the offered rate is known.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        shape = shapes[int(rng.integers(len(shapes)))]
        n = log_uniform_n(rng, n_lo, n_hi)
        reqs.append(Request(i, shape, n, seed * 1000 + i))
    return Stream(reqs)


def poisson_arrivals(stream: Stream, rate_hz: float, seed: int) -> Stream:
    """Assign Poisson arrival times (exponential gaps) at `rate_hz`; rate <= 0 means a burst at t=0."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in stream.requests:
        if rate_hz > 0:
            t += rng.exponential(1.0 / rate_hz)
        r.arrival = t
    return stream


def memory_admitted_stream(n_large: int = 64, n_small: int = 2000, n_large_side: int = 512,
                           seed: int = SEED_C5) -> Stream:
    """Large capsules (n = 512) interleaved with small ones (n log-uniform in [16, 64])."""
    rng = np.random.default_rng(seed)
    reqs = []
    every = max(1, n_small // max(1, n_large))
    rid = 0
    small_left, large_left = n_small, n_large
    while small_left or large_left:
        if large_left and (small_left == 0 or rid % (every + 1) == 0):
            shape = ("rbc", "ellipsoid")[int(rng.integers(2))]
            reqs.append(Request(rid, shape, n_large_side, seed * 10000 + rid))
            large_left -= 1
        else:
            shape = ("rbc", "ellipsoid")[int(rng.integers(2))]
            reqs.append(Request(rid, shape, log_uniform_n(rng, 16, 64), seed * 10000 + rid))
            small_left -= 1
        rid += 1
    return Stream(reqs)
