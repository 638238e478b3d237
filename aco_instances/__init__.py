"""Seeded synthetic Euclidean TSP instances.

Inputs only: this module holds none of the ACO arithmetic.  Both the GPU path
(its tests and benchmark) and the CPU oracle take their instances from here.

The paper measures on TSPLIB instances, which are not available here; seeded
synthetic cities of the same sizes stand in for them.  Two families:

* uniform   -- n cities i.i.d. uniform in the unit square;
* clustered -- K centres uniform in the unit square, each city picks a centre
               uniformly and adds isotropic Gaussian noise of std sigma
               (no clipping, so a few cities may fall outside the square).

Coordinates are FP32.  D_ij = fl32(sqrt(dx^2 + dy^2)) with dx, dy formed in
FP64 from the FP32 coordinates (exact), D_ii = 0.  Exact duplicate points are
re-drawn so that every off-diagonal distance is positive.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def _dedup(xy: np.ndarray, redraw) -> np.ndarray:
    for _ in range(100):
        _, first = np.unique(xy, axis=0, return_index=True)
        if first.shape[0] == xy.shape[0]:
            return xy
        dup = np.setdiff1d(np.arange(xy.shape[0]), first)
        xy[dup] = redraw(dup.shape[0])
    raise RuntimeError("could not draw distinct cities")


def uniform_cities(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2)).astype(np.float32)
    return _dedup(xy, lambda k: rng.random((k, 2)).astype(np.float32))


def clustered_cities(n: int, seed: int, clusters: int = 20, sigma: float = 0.02) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.random((clusters, 2))

    def draw(k):
        which = rng.integers(0, clusters, size=k)
        return (centres[which] + sigma * rng.standard_normal((k, 2))).astype(np.float32)

    return _dedup(draw(n), draw)


def circle_cities(n: int, radius: float = 0.5) -> np.ndarray:
    """n points evenly spaced on a circle (optimal tour: the polygon)."""
    ang = 2.0 * np.pi * np.arange(n) / n
    return np.stack([0.5 + radius * np.cos(ang), 0.5 + radius * np.sin(ang)], 1).astype(np.float32)


def distance_matrix(xy: np.ndarray) -> np.ndarray:
    xy = np.asarray(xy, dtype=np.float32).astype(np.float64)
    n = xy.shape[0]
    D = np.empty((n, n), np.float32)
    step = max(1, (1 << 22) // max(n, 1))
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        dx = xy[lo:hi, None, 0] - xy[None, :, 0]
        dy = xy[lo:hi, None, 1] - xy[None, :, 1]
        D[lo:hi] = np.sqrt(dx * dx + dy * dy).astype(np.float32)
    np.fill_diagonal(D, 0.0)
    return D


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named synthetic workload: instance recipe plus ACO parameters."""
    name: str
    n: int
    m: int
    alpha: float
    beta: float
    rho: float
    Q: float
    iters: int
    family: str = "uniform"
    clusters: int = 20
    sigma: float = 0.02
    tau0: float = 1.0
    gamma_max: float = 1.5
    gamma_min: float = 1.0
    elite_k: int = 0

    def cities(self, seed: int) -> np.ndarray:
        if self.family == "uniform":
            return uniform_cities(self.n, seed)
        return clustered_cities(self.n, seed, self.clusters, self.sigma)

    def dist(self, seed: int) -> np.ndarray:
        return distance_matrix(self.cities(seed))


WORKLOADS = {
    "uniform-n50-m50": Workload("uniform-n50-m50", 50, 50, 1.0, 2.0, 0.5, 1.0, 100),
    "uniform-n1000-m1000": Workload("uniform-n1000-m1000", 1000, 1000, 1.0, 2.0, 0.1, 1.0, 500),
    "clustered-n5000-m5000": Workload("clustered-n5000-m5000", 5000, 5000, 1.0, 3.0, 0.1, 1.0,
                                      200, family="clustered", clusters=20, sigma=0.02),
    "clustered-n2000-m2000": Workload("clustered-n2000-m2000", 2000, 2000, 1.0, 2.0, 0.1, 1.0,
                                      300, family="clustered", clusters=30, sigma=0.015),
}


def batch_sizes(count: int = 512, lo: int = 50, hi: int = 500, seed: int = 0) -> np.ndarray:
    """City counts of a batch of uneven instances, uniform on [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count).astype(np.int32)


@dataclasses.dataclass(frozen=True)
class BatchWorkload:
    """Many independent uniform instances of uneven size (seed of instance i = i)."""
    name: str
    count: int
    n_lo: int
    n_hi: int
    alpha: float
    beta: float
    rho: float
    Q: float
    iters: int
    size_seed: int = 0

    def sizes(self) -> np.ndarray:
        return batch_sizes(self.count, self.n_lo, self.n_hi, self.size_seed)

    def dists(self):
        return [distance_matrix(uniform_cities(int(n), i)) for i, n in enumerate(self.sizes())]


BATCH_WORKLOADS = {
    "batched-512-uniform-n50-500": BatchWorkload("batched-512-uniform-n50-500", 512, 50, 500,
                                                 1.0, 2.0, 0.2, 1.0, 300),
}
