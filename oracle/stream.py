"""Row-block FP64 evaluation of one LAMP iteration without materialising C
(test infrastructure only; see oracle/__init__).

The arithmetic is that of ``oracle.lamp`` (Algorithm 2 with the log-domain
marginal of Section 4.1), evaluated for a block of rows at a time so that only
block x m numbers exist at once; the O(n + m) state is all that persists.  It
is used (a) to time the oracle on a bounded sample of a large workload, and
(b) to compute individual rows of a large problem for sampled parity checks.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp

from .lamp import Params, dual_mirror_map, sqeuclid_cost, tclip


def row_log_normalisers(x: np.ndarray, y: np.ndarray, s: float, cnorm: float,
                        theta: np.ndarray, lam: float, rows) -> np.ndarray:
    """log Z_i = LSE_j(-lam (C_ij + 2||C||_inf theta_j)) for the listed rows (Section 4.1)."""
    rows = np.asarray(rows)
    C = sqeuclid_cost(np.asarray(x, np.float64)[rows], y, s)
    return logsumexp(-lam * (C + 2.0 * cnorm * theta[None, :]), axis=1)


def marginal_pass(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, cnorm: float,
                  theta: np.ndarray, lam: float, rows=None, block: int = 64):
    """For the listed rows (default all): log Z_i of p^{1/lam}(theta) and the contribution
    of those rows to col_r(p^{1/lam}(theta)) (Section 4.1, both displays)."""
    n = x.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    K = 2.0 * cnorm
    logZ = np.empty(rows.shape[0])
    colp = np.zeros(y.shape[0])
    for b0 in range(0, rows.shape[0], block):
        idx = rows[b0:b0 + block]
        a = -lam * (sqeuclid_cost(np.asarray(x, np.float64)[idx], y, s) + K * theta[None, :])
        L = logsumexp(a, axis=1)
        logZ[b0:b0 + block] = L
        colp += np.sum(r[idx, None] * np.exp(a - L[:, None]), axis=0)
    return logZ, colp


def lamp_step_stream(x, y, r, c, s, cnorm, t, lam, nu, theta, prm: Params, block: int = 64):
    """One iteration of Algorithm 2 with both marginals from ``marginal_pass``.
    Returns (lam_next, nu_next, theta_next, dict of intermediates)."""
    prm = prm.resolved(cnorm)
    m = c.shape[0]
    calpha = c + prm.alpha / m
    lam_next = prm.tau1 + lam * (1.0 - prm.tau1 * prm.eta)
    w = prm.tau1 / lam_next
    nubar = nu + w * (theta - nu)
    LA, colA = marginal_pass(x, y, r, s, cnorm, nu, lam, block=block)
    theta_bar = dual_mirror_map(theta, colA, c, calpha, prm.tau2, cnorm)
    nu_next = nu + w * (theta_bar - nu)
    LB, colB = marginal_pass(x, y, r, s, cnorm, nubar, lam_next, block=block)
    theta_hat = dual_mirror_map(theta, colB, c, calpha, prm.tau2, cnorm)
    theta_next = tclip(theta_hat, prm.beta)
    info = dict(logZA=LA, logZB=LB, colA=colA, colB=colB, theta_bar=theta_bar,
                theta_hat=theta_hat, nubar=nubar, res=float(np.abs(colA - c).sum()))
    return lam_next, nu_next, theta_next, info
