"""Seeded synthetic inputs for the sparse-Cholesky path.

This module only draws numbers: point clouds, right-hand sides, Monte Carlo
index pairs and request traces.  It holds none of the method's arithmetic, so
both the product path and the CPU oracle can be fed from it without sharing
any computation.

Every generator uses ``numpy.random.Generator(PCG64(seed))``.  The recipes
follow the shapes of the paper's experiments (Section 4.4: points iid uniform
in the unit cube) and of the workloads the benchmark is quoted on.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points iid uniform in [0,1]^d, row-major (n, d) float64 (Section 4.4)."""
    return _rng(seed).random((n, d), dtype=np.float64)


def jittered_grid(m: int, seed: int, jitter: float = 0.4) -> np.ndarray:
    """m*m points on a jittered grid over [0,1]^2.

    Grid spacing h = 1/m, centres ((i+1/2)h, (j+1/2)h) with row-major index
    i*m + j; each coordinate is moved by an independent U(-jitter*h, jitter*h).
    """
    h = 1.0 / m
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    base = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h], axis=1)
    noise = _rng(seed).uniform(-jitter * h, jitter * h, size=base.shape)
    return np.ascontiguousarray(base + noise, dtype=np.float64)


def embedded_sincos(n: int, seed: int, n_freq: int = 10, scale: float = 3.0) -> np.ndarray:
    """Points of intrinsic dimension 2 embedded in R^(2*n_freq).

    (u, v) ~ U[0,1]^2 is mapped through n_freq seeded Gaussian frequencies
    w_m ~ N(0, scale^2 I_2) to (sin(w_m.u), cos(w_m.u))_m / sqrt(n_freq), so
    every point lies on the unit sphere of R^(2*n_freq).
    """
    g = _rng(seed)
    w = g.normal(0.0, scale, size=(n_freq, 2))
    u = g.random((n, 2))
    ph = u @ w.T
    x = np.empty((n, 2 * n_freq), dtype=np.float64)
    x[:, 0::2] = np.sin(ph)
    x[:, 1::2] = np.cos(ph)
    x /= np.sqrt(n_freq)
    return x


def gaussian_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """(n, nrhs) row-major N(0,1) right-hand sides."""
    return _rng(seed).standard_normal((n, nrhs))


def random_pairs(n: int, m: int, seed: int) -> np.ndarray:
    """(m, 2) int64 index pairs drawn iid uniform from {0..n-1}^2 (Section 4.4 error estimate)."""
    return _rng(seed).integers(0, n, size=(m, 2), dtype=np.int64)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    points: np.ndarray           # (n, d) float64, original order
    nu: float                    # Matern smoothness (1/2, 3/2 or 5/2)
    lengthscale: float
    rho: float
    nrhs: int
    rhs_seed: int
    description: str = ""

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])

    def rhs(self) -> np.ndarray:
        return gaussian_rhs(self.n, self.nrhs, self.rhs_seed)


def small_uniform_2d() -> Workload:
    """2,000 points iid uniform in [0,1]^2, Matern-3/2, l=0.2, rho=3, one RHS."""
    return Workload("uniform2d-n2000-matern32", uniform_points(2000, 2, 1001), 1.5, 0.2, 3.0, 1, 11001,
                    "N=2000 iid U[0,1]^2 (seed 1001), Matern nu=3/2 l=0.2, rho=3, 1 N(0,1) RHS")


def large_grid_2d(m: int = 1000) -> Workload:
    """m*m jittered grid (default 10^6 points), Matern-1/2, l=0.1, rho=4, 8 RHS."""
    return Workload(f"jittergrid2d-n{m*m}-matern12", jittered_grid(m, 1002), 0.5, 0.1, 4.0, 8, 11002,
                    f"N={m*m} jittered {m}x{m} grid over [0,1]^2 (+-0.4h, seed 1002), Matern nu=1/2 l=0.1, rho=4, 8 N(0,1) RHS")


def uniform_3d(n: int = 200_000) -> Workload:
    """n points iid uniform in [0,1]^3, Matern-5/2, l=0.2, rho=3."""
    return Workload(f"uniform3d-n{n}-matern52", uniform_points(n, 3, 1003), 2.5, 0.2, 3.0, 1, 11003,
                    f"N={n} iid U[0,1]^3 (seed 1003), Matern nu=5/2 l=0.2, rho=3")


def paper_uniform(n: int, d: int, seed: int = 7, rho: float = 3.0) -> Workload:
    """The paper's scaling workload: U[0,1]^d, Matern nu=1/2, l=0.2 (Section 4.4 tables)."""
    return Workload(f"paper-uniform{d}d-n{n}", uniform_points(n, d, seed), 0.5, 0.2, rho, 1, seed + 1,
                    f"N={n} iid U[0,1]^{d} (seed {seed}), Matern nu=1/2 l=0.2, rho={rho}")


@dataclass
class BatchInstance:
    points: np.ndarray
    lengthscale: float
    rhs_seed: int


def batched_instances(count: int = 512, n_lo: int = 500, n_hi: int = 50_000, seed: int = 4000) -> List[BatchInstance]:
    """Independent instances: N log-uniform in [n_lo, n_hi], U[0,1]^2 points,
    Matern-3/2 lengthscale U(0.05, 0.3), rho=3, one RHS each."""
    out = []
    for i in range(count):
        g = _rng(seed + i)
        n = int(np.floor(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        ell = float(g.uniform(0.05, 0.3))
        pts = g.random((n, 2))
        out.append(BatchInstance(pts, ell, seed + 100_000 + i))
    return out


@dataclass
class Request:
    arrival_s: float
    points: np.ndarray
    rhs_seed: int
    nrhs: int = 4


def serving_trace(count: int, rate_per_s: float, n_lo: int = 1000, n_hi: int = 200_000,
                  seed: int = 5000) -> List[Request]:
    """Poisson arrivals at a fixed rate; each request has N log-uniform in
    [n_lo, n_hi] with points of intrinsic dimension 2 embedded in R^20."""
    g = _rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += float(g.exponential(1.0 / rate_per_s))
        n = int(np.floor(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        reqs.append(Request(t, embedded_sincos(n, seed + 1 + i), seed + 50_000 + i))
    return reqs
