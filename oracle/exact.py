"""Ground-truth OT values for pinning the oracle (test infrastructure only).

These are textbook routines, independent of LAMP:

* brute force over permutations for n = m <= 8 with uniform marginals (by the
  Birkhoff-von Neumann theorem an optimal plan of the OT LP (problem primal_ot)
  is then a permutation matrix divided by n);
* scipy's assignment solver for the same uniform case at larger n;
* scipy's HiGHS linear-programming solver for general marginals;
* log-domain Sinkhorn iterations for the entropic problem (problem primal_eot).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment, linprog
from scipy.special import logsumexp


def brute_force_ot_uniform(C: np.ndarray) -> float:
    """min_sigma (1/n) sum_i C_{i sigma(i)} over all permutations (n <= 8)."""
    n, m = C.shape
    assert n == m and n <= 8
    best = np.inf
    for perm in itertools.permutations(range(n)):
        v = sum(C[i, perm[i]] for i in range(n))
        best = min(best, v)
    return float(best / n)


def assignment_ot_uniform(C: np.ndarray) -> float:
    """Uniform-marginal OT value via the Hungarian-type assignment solver."""
    n, m = C.shape
    assert n == m
    ri, ci = linear_sum_assignment(C)
    return float(C[ri, ci].sum() / n)


def lp_ot(C: np.ndarray, r: np.ndarray, c: np.ndarray):
    """min <C,X> s.t. X 1 = r, X^T 1 = c, X >= 0 (problem primal_ot) with HiGHS.
    Returns (value, plan)."""
    n, m = C.shape
    A_eq = np.zeros((n + m, n * m))
    for i in range(n):
        A_eq[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        A_eq[n + j, j::m] = 1.0
    b_eq = np.concatenate([r, c])
    res = linprog(C.ravel(), A_eq=A_eq, b_eq=b_eq, bounds=(0, None), method="highs",
                  options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    assert res.status == 0, res.message
    return float(res.fun), res.x.reshape(n, m)


def lp_ot_duals(C: np.ndarray, r: np.ndarray, c: np.ndarray):
    """Optimal LP duals (y_r, y_c) of the marginal constraints (HiGHS marginals):
    max <r, y_r> + <c, y_c> s.t. y_r,i + y_c,j <= C_ij."""
    n, m = C.shape
    A_eq = np.zeros((n + m, n * m))
    for i in range(n):
        A_eq[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        A_eq[n + j, j::m] = 1.0
    res = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([r, c]), bounds=(0, None),
                  method="highs")
    assert res.status == 0, res.message
    y = res.eqlin.marginals
    return float(res.fun), y[:n], y[n:]


def sinkhorn_eot(C: np.ndarray, r: np.ndarray, c: np.ndarray, eta: float, iters: int = 200000,
                 tol: float = 1e-14) -> np.ndarray:
    """Log-domain Sinkhorn for min <C,X> - eta H(X) over Pi(r, c) (problem primal_eot).
    Returns the plan X = exp((f_i + g_j - C_ij)/eta)."""
    f = np.zeros(C.shape[0])
    g = np.zeros(C.shape[1])
    lr, lc = np.log(r), np.log(c)
    for _ in range(iters):
        f = eta * (lr - logsumexp((g[None, :] - C) / eta, axis=1))
        g = eta * (lc - logsumexp((f[:, None] - C) / eta, axis=0))
        X = np.exp((f[:, None] + g[None, :] - C) / eta)
        if np.abs(X.sum(axis=1) - r).sum() < tol:
            break
    return np.exp((f[:, None] + g[None, :] - C) / eta)
