"""Seeded synthetic OT workloads (point clouds and marginals).

This module only draws inputs; it holds none of the solver's arithmetic and is
shared by the tests, the benchmark and the oracle-driven checks.  Generators use
NumPy's PCG64 with a fixed seed per workload so that every machine draws the
same FP32 points and FP64 marginals.

Marginals that come from Dirichlet draws get the full-support fix the paper
applies to its inputs (Appendix E): add 1e-6 to every entry, then renormalise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Workload:
    name: str
    x: np.ndarray          # n x d, float32, row-major
    y: np.ndarray          # m x d, float32, row-major
    r: np.ndarray          # n, float64, strictly positive, sums to 1
    c: np.ndarray          # m, float64, strictly positive, sums to 1
    eta: float
    tol: float             # stopping tolerance on ||row - r||_1 + ||col - c||_1 (0: fixed count)
    max_iter: int

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def m(self) -> int:
        return self.y.shape[0]

    @property
    def d(self) -> int:
        return self.x.shape[1]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def full_support(w: np.ndarray) -> np.ndarray:
    """Add 1e-6 to every entry and renormalise (Appendix E input preparation)."""
    w = np.asarray(w, dtype=np.float64) + 1e-6
    return w / w.sum()


def dirichlet_ones(rng: np.random.Generator, k: int) -> np.ndarray:
    """Dirichlet(1,...,1) draw as normalised Exp(1) variables, then the full-support fix."""
    e = rng.exponential(1.0, size=k)
    return full_support(e / e.sum())


def uniform_marginal(k: int) -> np.ndarray:
    return np.full(k, 1.0 / k)


def uniform_square(n: int = 256, m: int = 256, d: int = 2, seed: int = 1001) -> Workload:
    """256 x 256 points i.i.d. uniform on [0,1]^2, uniform marginals, eta = 1e-2,
    a fixed 500 iterations (the small parity workload)."""
    g = _rng(seed)
    x = g.random((n, d)).astype(np.float32)
    y = g.random((m, d)).astype(np.float32)
    return Workload(f"uniform{d}d_{n}x{m}", x, y, uniform_marginal(n), uniform_marginal(m),
                    eta=1e-2, tol=0.0, max_iter=500)


def gaussian_pair(n: int = 4096, m: int = 4096, seed: int = 1002) -> Workload:
    """Source ~ N(0, I_3), target ~ N(1.5 * 1, 0.5^2 I_3), Dirichlet(1) marginals,
    eta = 1e-3, run to residual <= 1e-4."""
    g = _rng(seed)
    x = g.standard_normal((n, 3)).astype(np.float32)
    y = (1.5 + 0.5 * g.standard_normal((m, 3))).astype(np.float32)
    r = dirichlet_ones(g, n)
    c = dirichlet_ones(g, m)
    return Workload(f"gauss3d_{n}x{m}", x, y, r, c, eta=1e-3, tol=1e-4, max_iter=100000)


def gmm64(n: int = 65536, m: int = 65536, d: int = 64, seed: int = 1003) -> Workload:
    """Both clouds from one 8-component Gaussian mixture in d = 64 (means ~ N(0, 4 I),
    unit-variance components, equal weights), independent draws, uniform marginals,
    eta = 1e-3, run to residual <= 1e-4."""
    g = _rng(seed)
    means = 2.0 * g.standard_normal((8, d))
    kx = g.integers(0, 8, size=n)
    ky = g.integers(0, 8, size=m)
    x = (means[kx] + g.standard_normal((n, d))).astype(np.float32)
    y = (means[ky] + g.standard_normal((m, d))).astype(np.float32)
    return Workload(f"gmm{d}d_{n}x{m}", x, y, uniform_marginal(n), uniform_marginal(m),
                    eta=1e-3, tol=1e-4, max_iter=100000)


def sphere_cube(n: int = 1 << 18, m: int = 1 << 18, seed: int = 1005) -> Workload:
    """Source uniform on the unit sphere in R^3 plus N(0, 0.01^2 I) noise, target uniform
    in the unit cube, uniform marginals, eta = 5e-3, run to residual <= 1e-4."""
    g = _rng(seed)
    v = g.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x = (v + 0.01 * g.standard_normal((n, 3))).astype(np.float32)
    y = g.random((m, 3)).astype(np.float32)
    return Workload(f"sphere_cube_{n}x{m}", x, y, uniform_marginal(n), uniform_marginal(m),
                    eta=5e-3, tol=1e-4, max_iter=100000)


def batch_problem(p: int) -> Workload:
    """Problem p of the 64-problem batch: n, m log-uniform in [512, 8192], d in {2, 3, 16},
    points uniform on [0,1]^d, Dirichlet(1) marginals, eta = 1e-3, residual <= 1e-4."""
    g = _rng(2000 + p)
    n = int(round(np.exp(g.uniform(np.log(512), np.log(8192)))))
    m = int(round(np.exp(g.uniform(np.log(512), np.log(8192)))))
    d = int(g.choice([2, 3, 16]))
    x = g.random((n, d)).astype(np.float32)
    y = g.random((m, d)).astype(np.float32)
    return Workload(f"batch{p}_{n}x{m}x{d}", x, y, dirichlet_ones(g, n), dirichlet_ones(g, m),
                    eta=1e-3, tol=1e-4, max_iter=100000)


def regular_polygon(n: int, seed: int = 0) -> Workload:
    """x_i = y_i = vertices of a regular n-gon on the unit circle, uniform marginals.
    The cost is circulant, so col(X^t) = c and theta = nu = 0 for every t."""
    ang = 2.0 * np.pi * np.arange(n) / n
    x = np.stack([np.cos(ang), np.sin(ang)], axis=1).astype(np.float32)
    return Workload(f"polygon_{n}", x, x.copy(), uniform_marginal(n), uniform_marginal(n),
                    eta=0.0, tol=0.0, max_iter=100)


def random_small(n: int, m: int, d: int, seed: int, uniform: bool = False,
                 eta: float = 0.0) -> Workload:
    """Small random problem for ragged-shape parity cases."""
    g = _rng(seed)
    x = g.random((n, d)).astype(np.float32)
    y = (0.3 + g.random((m, d))).astype(np.float32)
    r = uniform_marginal(n) if uniform else dirichlet_ones(g, n)
    c = uniform_marginal(m) if uniform else dirichlet_ones(g, m)
    return Workload(f"rand_{n}x{m}x{d}", x, y, r, c, eta=eta, tol=0.0, max_iter=100)


WORKLOADS = {
    "uniform2d_256": uniform_square,
    "gauss3d_4096": gaussian_pair,
    "gmm64d_65536": gmm64,
    "sphere_cube_262144": sphere_cube,
}


def synthetic_duals(m: int, seed: int, amp: float = 0.4):
    """A seeded dual state (nu, theta), each coordinate uniform in [-amp, amp]: a starting point
    for single-iteration parity checks at large sizes, where no reference trajectory exists."""
    g = _rng(seed)
    return g.uniform(-amp, amp, m), g.uniform(-amp, amp, m)
