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


@dataclass
class CostWorkload:
    """A problem given by its cost matrix (the explicit-cost input) instead of points."""
    name: str
    cost: np.ndarray       # n x m, float32, row-major, entries >= 0 (a device tensor for the large ones)
    r: np.ndarray
    c: np.ndarray
    eta: float


def image_marginal(k: int, g: np.random.Generator) -> np.ndarray:
    """A k x k 'image' as a marginal (row-major pixels): a few Gaussian blobs of random
    centre, width and weight on a faint background, with the full-support fix."""
    yy, xx = np.mgrid[0:k, 0:k].astype(np.float64)
    img = np.full((k, k), 0.02)
    for _ in range(int(g.integers(2, 6))):
        cy, cx = g.uniform(0, k - 1, 2)
        w = g.uniform(0.05, 0.3) * k
        img += g.uniform(0.2, 1.0) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * w * w))
    return full_support(img.ravel())


def grid_cost(k: int, kind: str = "sqeuclid") -> np.ndarray:
    """Ground cost between the pixels of two k x k grids (integer coordinates), the cost of
    image-pair transport benchmarks: sum_k |di|^2 ("sqeuclid"), sum_k |di| ("l1"),
    max_k |di| ("linf").  Integer entries, exact in FP32 for k <= 2^11."""
    yy, xx = np.divmod(np.arange(k * k), k)
    dy = np.abs(yy[:, None] - yy[None, :]).astype(np.float64)
    dx = np.abs(xx[:, None] - xx[None, :]).astype(np.float64)
    if kind == "sqeuclid":
        cmat = dy * dy + dx * dx
    elif kind == "l1":
        cmat = dy + dx
    else:
        cmat = np.maximum(dy, dx)
    return cmat.astype(np.float32)


def grid_cost_device(k: int, kind: str, device, rows_per_chunk: int = 4096):
    """grid_cost(k, kind) built on a torch device in row chunks (n = m = k^2 entries squared:
    16 GiB of FP32 at k = 256), for sizes whose matrix should not pass through host memory."""
    import torch
    n = k * k
    idx = torch.arange(n, device=device, dtype=torch.int64)
    yy, xx = idx // k, idx % k
    out = torch.empty(n, n, dtype=torch.float32, device=device)
    for i0 in range(0, n, rows_per_chunk):
        i1 = min(n, i0 + rows_per_chunk)
        dy = (yy[i0:i1, None] - yy[None, :]).abs()
        dx = (xx[i0:i1, None] - xx[None, :]).abs()
        if kind == "sqeuclid":
            blk = dy * dy + dx * dx
        elif kind == "l1":
            blk = dy + dx
        else:
            blk = torch.maximum(dy, dx)
        out[i0:i1] = blk.to(torch.float32)
    return out


def image_pair(k: int, kind: str = "sqeuclid", seed: int = 1101, eta: float = 0.0) -> CostWorkload:
    """Transport between two random k x k images (n = m = k^2) over the grid cost."""
    g = _rng(seed)
    return CostWorkload(f"images_{k}x{k}_{kind}", grid_cost(k, kind), image_marginal(k, g), image_marginal(k, g),
                        eta)


def image_pair_device(k: int = 256, kind: str = "sqeuclid", seed: int = 1201, device="cuda") -> CostWorkload:
    """image_pair at sizes whose matrix is built on the device (cost is a torch tensor there);
    k = 256 gives the n = m = 2^16 cost-matrix benchmark (16 GiB of FP32)."""
    g = _rng(seed)
    r, c = image_marginal(k, g), image_marginal(k, g)
    return CostWorkload(f"images_{k}x{k}_{kind}", grid_cost_device(k, kind, device), r, c, 0.0)


def random_cost(n: int, m: int, seed: int, eta: float = 1e-2) -> CostWorkload:
    """Non-metric cost: independent uniform [0, 1) entries, Dirichlet marginals."""
    g = _rng(seed)
    cost = g.random((n, m), dtype=np.float32)
    return CostWorkload(f"randcost_{n}x{m}", cost, dirichlet_ones(g, n), dirichlet_ones(g, m), eta)


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
