"""Dense FP64 LAMP / PDMP oracle (test infrastructure only; see oracle/__init__).

Notation follows the paper: X is n x m, row(X) = X 1, col(X) = X^T 1,
||C||_inf = max_ij |C_ij|, p is row-stochastic and X = diag(r) p (Section 2).
K = 2 ||C||_inf is the factor in front of the dual in the saddle objective
(problem spp), lam_t = 1/eta_t is the inverse temperature with lam_0 = 0
(eta_0 = infinity, Algorithm 2).

Everything here but envelope_grad_y_columns (one column at a time) materialises the
n x m cost matrix, so it is meant for n*m up to a few million.  ``oracle.stream``
evaluates the same iteration in row blocks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import logsumexp

# --------------------------------------------------------------------------
# Problem data
# --------------------------------------------------------------------------


def sqeuclid_cost(x: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """C_ij = s * ||x_i - y_j||^2 in FP64 (the squared-Euclidean ground cost the
    paper generates on the fly from point clouds, Sections 1 and 4.1).

    Difference form, written out: no norm expansion, no reordering.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    diff = x[:, None, :] - y[None, :, :]
    return s * np.sum(diff * diff, axis=2)


def l1_cost(x: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """C_ij = s * sum_k |x_ik - y_jk| in FP64 (the l1 ground cost of the kernelized DOTmark
    experiments, Section 5 and Appendix E)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return s * np.sum(np.abs(x[:, None, :] - y[None, :, :]), axis=2)


def linf_cost(x: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """C_ij = s * max_k |x_ik - y_jk| in FP64 (the l_inf ground cost of the same experiments)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return s * np.max(np.abs(x[:, None, :] - y[None, :, :]), axis=2)


GROUND_COSTS = {"sqeuclid": sqeuclid_cost, "l1": l1_cost, "linf": linf_cost}


def ground_cost(x: np.ndarray, y: np.ndarray, s: float, kind: str = "sqeuclid") -> np.ndarray:
    return GROUND_COSTS[kind](x, y, s)


def max_cost(x: np.ndarray, y: np.ndarray, kind: str, block: int = 256) -> float:
    """max_ij of the unscaled ground cost (row blocks)."""
    best = 0.0
    for i0 in range(0, x.shape[0], block):
        best = max(best, float(np.max(ground_cost(x[i0:i0 + block], y, 1.0, kind))))
    return best


def max_sqdist(x: np.ndarray, y: np.ndarray, block: int = 256) -> float:
    """max_ij ||x_i - y_j||^2 in FP64 (difference form, row blocks)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    best = 0.0
    for i0 in range(0, x.shape[0], block):
        d = x[i0:i0 + block, None, :] - y[None, :, :]
        best = max(best, float(np.max(np.sum(d * d, axis=2))))
    return best


# --------------------------------------------------------------------------
# Primitives of Section 3.1
# --------------------------------------------------------------------------


def row(X: np.ndarray) -> np.ndarray:
    """row(X) = X 1 (Section 2)."""
    return X.sum(axis=1)


def col(X: np.ndarray) -> np.ndarray:
    """col(X) = X^T 1 (Section 2)."""
    return X.sum(axis=0)


def col_r(p: np.ndarray, r: np.ndarray) -> np.ndarray:
    """col_r(p) = col(diag(r) p) (problem l1_ot_primal)."""
    return col(r[:, None] * p)


def entropy(X: np.ndarray) -> float:
    """H(X) = -<X, log X> with 0 log 0 = 0 (Section 2)."""
    X = np.asarray(X, dtype=np.float64)
    nz = X > 0
    return float(-np.sum(X[nz] * np.log(X[nz])))


def kl(X: np.ndarray, Y: np.ndarray) -> float:
    """KL(X||Y) = Bregman divergence of -H, for X, Y in the simplex (Section 2)."""
    nz = X > 0
    return float(np.sum(X[nz] * (np.log(X[nz]) - np.log(Y[nz]))) - X.sum() + Y.sum())


def dual_to_primal(C: np.ndarray, theta: np.ndarray, lam: float, cnorm: float) -> np.ndarray:
    """p^eta(theta) = diag(Z)^-1 exp(-(C + 2||C||_inf 1 theta^T)/eta) with
    lam = 1/eta (equation def:dual_to_primal).  lam = 0 (eta = infinity) gives
    the uniform row-stochastic matrix (proof of Proposition equivalence).
    """
    a = -lam * (C + 2.0 * cnorm * theta[None, :])
    return np.exp(a - logsumexp(a, axis=1, keepdims=True))


def log_normaliser(C: np.ndarray, theta: np.ndarray, lam: float, cnorm: float) -> np.ndarray:
    """log Z_i for p^eta(theta): the row LogSumExp of -(C_i: + 2||C||_inf theta)/eta
    (Section 4.1, first display)."""
    return logsumexp(-lam * (C + 2.0 * cnorm * theta[None, :]), axis=1)


def primal_mirror_map(p0: np.ndarray, theta: np.ndarray, C: np.ndarray, tau: float,
                      eta: float, cnorm: float) -> np.ndarray:
    """M_tau^eta(p0; theta)_ij = p0_ij^(1 - tau eta) exp(-tau(C_ij + 2||C||_inf theta_j)) / Z_i
    (equation def:closed_form_opt, first line), evaluated in the log domain."""
    with np.errstate(divide="ignore"):
        a = (1.0 - tau * eta) * np.log(p0) - tau * (C + 2.0 * cnorm * theta[None, :])
    return np.exp(a - logsumexp(a, axis=1, keepdims=True))


def dual_mirror_arg(theta0: np.ndarray, colp: np.ndarray, c: np.ndarray, calpha: np.ndarray,
                    tau: float, cnorm: float) -> np.ndarray:
    """The argument of tanh in def:closed_form_opt (the step's natural parameter):
    2 tau ||C||_inf / c^alpha_j (col_r(p)_j - c_j) + (1/2) log((1 + theta0_j)/(1 - theta0_j))."""
    return (2.0 * tau * cnorm / calpha * (colp - c)
            + 0.5 * np.log((1.0 + theta0) / (1.0 - theta0)))


def dual_mirror_map(theta0: np.ndarray, colp: np.ndarray, c: np.ndarray, calpha: np.ndarray,
                    tau: float, cnorm: float) -> np.ndarray:
    """M_tau^eta(theta0; p)_j = tanh( 2 tau ||C||_inf / c^alpha_j (col_r(p)_j - c_j)
    + (1/2) log((1 + theta0_j)/(1 - theta0_j)) )  (equation def:closed_form_opt)."""
    return np.tanh(dual_mirror_arg(theta0, colp, c, calpha, tau, cnorm))


def tclip(theta: np.ndarray, beta: float) -> np.ndarray:
    """Coordinate-wise clip to [-tanh(beta/2), tanh(beta/2)] (Section 3.1)."""
    b = math.tanh(beta / 2.0)
    return np.clip(theta, -b, b)


def inv_eta_schedule(T: int, tau1: float, eta: float) -> np.ndarray:
    """lam_t = 1/eta_t for t = 0..T from eta_0 = infinity and the update
    (step:eta_update), in its inverse form eta_{t+1}^-1 = tau1 + eta_t^-1 (1 - tau1 eta)
    stated right after Algorithm 2."""
    lam = np.zeros(T + 1)
    for t in range(T):
        lam[t + 1] = tau1 + lam[t] * (1.0 - tau1 * eta)
    return lam


# --------------------------------------------------------------------------
# Parameters (Appendix E: "for all LAMP testing")
# --------------------------------------------------------------------------


@dataclass
class Params:
    eta: float = 0.0
    alpha: float = 0.01
    beta: float = 1.1
    tau1: float | None = None    # None -> 1 / (2 ||C||_inf)
    tau2: float | None = None    # None -> 1 / (2 ||C||_inf)

    def resolved(self, cnorm: float) -> "Params":
        t1 = self.tau1 if self.tau1 is not None else 1.0 / (2.0 * cnorm)
        t2 = self.tau2 if self.tau2 is not None else 1.0 / (2.0 * cnorm)
        return Params(self.eta, self.alpha, self.beta, t1, t2)


@dataclass
class LampState:
    """O(n + m) state of Algorithm 2 after t iterations."""
    t: int
    lam: float            # 1/eta_t
    nu: np.ndarray
    theta: np.ndarray


@dataclass
class LampTrace:
    """Per-iteration quantities of Algorithm 2, index t means iteration t -> t+1."""
    lam: list = field(default_factory=list)       # lam_t
    logZA: list = field(default_factory=list)     # log Z of p^{eta_t}(nu^t)
    logZB: list = field(default_factory=list)     # log Z of p^{eta_{t+1}}(nubar^{t+1})
    colA: list = field(default_factory=list)      # col_r(p^{eta_t}(nu^t)) = col(X^t)
    colB: list = field(default_factory=list)      # col_r(p^{eta_{t+1}}(nubar^{t+1}))
    theta_bar: list = field(default_factory=list)
    theta_hat: list = field(default_factory=list)
    theta_bar_arg: list = field(default_factory=list)   # thetabar = tanh(theta_bar_arg)
    theta_hat_arg: list = field(default_factory=list)   # thetahat = tanh(theta_hat_arg)
    nubar: list = field(default_factory=list)
    nu: list = field(default_factory=list)        # nu^{t+1}
    theta: list = field(default_factory=list)     # theta^{t+1}
    res: list = field(default_factory=list)       # ||col(X^t) - c||_1


def lamp_step(C: np.ndarray, r: np.ndarray, c: np.ndarray, state: LampState, prm: Params,
              cnorm: float, trace: LampTrace | None = None) -> LampState:
    """One iteration t -> t+1 of Algorithm 2 (LAMP), steps in the paper's order:
    eta_{t+1} (step:eta_update), nubar^{t+1} (step:lamp_mid_nu), thetabar^{t+1}
    (step:lamp_mid_theta), nu^{t+1} (step:lamp_main_nu), thetahat^{t+1}
    (step:lamp_main_theta), theta^{t+1} = tclip(thetahat^{t+1}, beta).

    The dual mirror maps use the closed form of def:closed_form_opt, which needs
    only the column marginal col_r(p^{eta}(.)) (remark after Proposition equivalence).
    """
    m = c.shape[0]
    calpha = c + prm.alpha / m
    lam_t = state.lam
    lam_next = prm.tau1 + lam_t * (1.0 - prm.tau1 * prm.eta)        # 1/eta_{t+1}
    w = prm.tau1 / lam_next                                          # tau1 * eta_{t+1}
    nu, theta = state.nu, state.theta

    nubar = nu + w * (theta - nu)
    pA = dual_to_primal(C, nu, lam_t, cnorm)
    colA = col_r(pA, r)
    a_bar = dual_mirror_arg(theta, colA, c, calpha, prm.tau2, cnorm)
    theta_bar = np.tanh(a_bar)
    nu_next = nu + w * (theta_bar - nu)
    pB = dual_to_primal(C, nubar, lam_next, cnorm)
    colB = col_r(pB, r)
    a_hat = dual_mirror_arg(theta, colB, c, calpha, prm.tau2, cnorm)
    theta_hat = np.tanh(a_hat)
    theta_next = tclip(theta_hat, prm.beta)

    if trace is not None:
        trace.lam.append(lam_t)
        trace.logZA.append(log_normaliser(C, nu, lam_t, cnorm))
        trace.logZB.append(log_normaliser(C, nubar, lam_next, cnorm))
        trace.colA.append(colA)
        trace.colB.append(colB)
        trace.theta_bar.append(theta_bar)
        trace.theta_hat.append(theta_hat)
        trace.theta_bar_arg.append(a_bar)
        trace.theta_hat_arg.append(a_hat)
        trace.nubar.append(nubar)
        trace.nu.append(nu_next)
        trace.theta.append(theta_next)
        trace.res.append(float(np.abs(colA - c).sum()))
    return LampState(state.t + 1, lam_next, nu_next, theta_next)


def lamp_init(m: int) -> LampState:
    """theta^0 = nu^0 = 0, eta_0 = infinity (Algorithm 2, REQUIRE line)."""
    return LampState(0, 0.0, np.zeros(m), np.zeros(m))


def lamp_dense(C: np.ndarray, r: np.ndarray, c: np.ndarray, prm: Params, T: int,
               cnorm: float | None = None, tol: float | None = None,
               state: LampState | None = None, trace: bool = True):
    """Run Algorithm 2 for at most T iterations.

    Stopping reading (the paper stops on ||col(X^t) - c||_1 + ||row(X^t) - r||_1,
    Appendix E): if ``tol`` is given, before iteration t >= 1 the residual of X^t is
    measured and, if it is <= tol, the run stops and returns the state holding
    nu^t, i.e. the iterate that met the tolerance.  The starting point t = 0 is not
    tested: with eta_0 = infinity it is the product coupling r (1/m)^T, which is
    feasible whenever c is uniform without being an iterate of the method.

    Returns (state, trace).  ``state.lam`` and ``state.nu`` define
    X^t = diag(r) p^{eta_t}(nu^t) (Proposition infeas_bound).
    """
    cnorm = float(np.max(np.abs(C))) if cnorm is None else cnorm
    prm = prm.resolved(cnorm)
    st = lamp_init(C.shape[1]) if state is None else state
    tr = LampTrace() if trace else None
    for _ in range(T):
        if tol is not None and st.t >= 1:
            X = plan(C, r, st, cnorm)
            if residuals(X, r, c)[2] <= tol:
                break
        st = lamp_step(C, r, c, st, prm, cnorm, tr)
    return st, tr


def plan(C: np.ndarray, r: np.ndarray, st: LampState, cnorm: float) -> np.ndarray:
    """X^t = diag(r) p^{eta_t}(nu^t) (Proposition infeas_bound / def primal_subs)."""
    return r[:, None] * dual_to_primal(C, st.nu, st.lam, cnorm)


def residuals(X: np.ndarray, r: np.ndarray, c: np.ndarray):
    """(||row(X) - r||_1, ||col(X) - c||_1, their sum) -- the stopping measure of Appendix E."""
    rr = float(np.abs(row(X) - r).sum())
    cc = float(np.abs(col(X) - c).sum())
    return rr, cc, rr + cc


# --------------------------------------------------------------------------
# Algorithm 1 (PDMP): explicit primal iterates, used to pin LAMP
# --------------------------------------------------------------------------


def pdmp_dense(C: np.ndarray, r: np.ndarray, c: np.ndarray, prm: Params, T: int,
               cnorm: float | None = None):
    """Algorithm 1 with p^0 = (1/m), theta^0 = 0.  Returns lists p[t], pbar[t+1]
    (index t+1 holds pbar^{t+1}), theta[t]."""
    cnorm = float(np.max(np.abs(C))) if cnorm is None else cnorm
    prm = prm.resolved(cnorm)
    n, m = C.shape
    calpha = c + prm.alpha / m
    p = np.full((n, m), 1.0 / m)
    theta = np.zeros(m)
    ps, pbars, thetas = [p], [None], [theta]
    for _ in range(T):
        pbar = primal_mirror_map(p, theta, C, prm.tau1, prm.eta, cnorm)
        theta_bar = dual_mirror_map(theta, col_r(p, r), c, calpha, prm.tau2, cnorm)
        p_next = primal_mirror_map(p, theta_bar, C, prm.tau1, prm.eta, cnorm)
        theta_hat = dual_mirror_map(theta, col_r(pbar, r), c, calpha, prm.tau2, cnorm)
        theta = tclip(theta_hat, prm.beta)
        p = p_next
        ps.append(p)
        pbars.append(pbar)
        thetas.append(theta)
    return ps, pbars, thetas


# --------------------------------------------------------------------------
# Algorithm 3 (Round)
# --------------------------------------------------------------------------


def round_plan(X: np.ndarray, r: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Round(X, r, c), Algorithm 3.  Reading: if ||delta_r||_1 = 0 the rank-one
    correction of Step 4 is skipped (then delta_c = 0 too)."""
    xr = np.minimum(r / row(X), 1.0)
    X1 = xr[:, None] * X
    yc = np.minimum(c / col(X1), 1.0)
    X2 = X1 * yc[None, :]
    dr = r - row(X2)
    dc = c - col(X2)
    nrm = np.abs(dr).sum()
    if nrm == 0.0:
        return X2
    return X2 + np.outer(dr, dc) / nrm


# --------------------------------------------------------------------------
# Dual functions (Appendix B) and certificates (Proposition infeas_bound)
# --------------------------------------------------------------------------


def dual_D(C: np.ndarray, r: np.ndarray, c: np.ndarray, theta: np.ndarray, cnorm: float) -> float:
    """D(theta) = sum_i r_i min_j {C_ij + 2||C||_inf theta_j} - 2||C||_inf <c, theta>
    (equation def:dual_spp, eta = 0)."""
    K = 2.0 * cnorm
    return float(r @ np.min(C + K * theta[None, :], axis=1) - K * (c @ theta))


def softmin(v: np.ndarray, eta: float, axis: int) -> np.ndarray:
    """softmin^eta(v) = -eta log sum exp(-v/eta) (Appendix B)."""
    return -eta * logsumexp(-v / eta, axis=axis)


def dual_D_eta(C: np.ndarray, r: np.ndarray, c: np.ndarray, theta: np.ndarray, cnorm: float,
               eta: float) -> float:
    """D^eta(theta) = sum_i r_i softmin^eta_j {C_ij + 2||C||_inf theta_j} - 2||C||_inf <c,theta>
    (equation def:dual_spp_e)."""
    K = 2.0 * cnorm
    return float(r @ softmin(C + K * theta[None, :], eta, axis=1) - K * (c @ theta))


def primal_penalised(C: np.ndarray, X: np.ndarray, r: np.ndarray, c: np.ndarray, cnorm: float,
                     eta: float = 0.0) -> float:
    """P^eta(X) = <C, X> + 2||C||_inf ||col(X) - c||_1 - eta H(X) (problem l1_ot_primal),
    with the row infeasibility added under the same factor (it is zero for X = diag(r)p)."""
    K = 2.0 * cnorm
    rr, cc, _ = residuals(X, r, c)
    return float(np.sum(C * X) + K * (rr + cc) - eta * entropy(X))


def saddle_K(C: np.ndarray, X: np.ndarray, theta: np.ndarray, c: np.ndarray, cnorm: float,
             eta: float = 0.0) -> float:
    """K^eta(X, theta) = <C,X> + 2||C||_inf <theta, col(X) - c> - eta H(X) (problem spp)."""
    return float(np.sum(C * X) + 2.0 * cnorm * theta @ (col(X) - c) - eta * entropy(X))


def prop_bound(colres: float, t: int, m: int, cnorm: float) -> float:
    """Right-hand side of (ineq:main_infeas_bounds): 4||C||_inf ||col(X^t)-c||_1 + 2||C||_inf log m / t."""
    return 4.0 * cnorm * colres + 2.0 * cnorm * math.log(m) / t


def intermediate_bound(colX: np.ndarray, c: np.ndarray, nu: np.ndarray, klstar: float, t: int,
                       cnorm: float) -> float:
    """2||C||_inf <-nu^t, col(X^t) - c> + 2||C||_inf KL(X*||X^0)/t, the first line of
    (ineq:ub_telescope_last_iter), scaled back by ||C||_inf (proof of Lemma last_iterate)."""
    return 2.0 * cnorm * float(-nu @ (colX - c)) + 2.0 * cnorm * klstar / t


def certificate(C: np.ndarray, r: np.ndarray, c: np.ndarray, st: LampState, prm: Params,
                cnorm: float) -> dict:
    """Computable certificate of X^t = diag(r) p^{eta_t}(nu^t): residuals, <C,X^t>,
    D(theta^t), D(nu^t), the penalised primal, their gap, <C, Round(X^t)> and the
    right-hand side of Proposition infeas_bound(a)."""
    X = plan(C, r, st, cnorm)
    rr, cc, _ = residuals(X, r, c)
    cost = float(np.sum(C * X))
    d_theta = dual_D(C, r, c, st.theta, cnorm)
    d_nu = dual_D(C, r, c, st.nu, cnorm)
    primal = cost + 2.0 * cnorm * (rr + cc)
    out = dict(t=st.t, row_res=rr, col_res=cc, cost=cost, dual_theta=d_theta, dual_nu=d_nu,
               primal_penalized=primal, gap=primal - max(d_theta, d_nu),
               rounded_cost=float(np.sum(C * round_plan(X, r, c))),
               prop_bound=prop_bound(cc, st.t, C.shape[1], cnorm) if st.t >= 1 else math.inf)
    if prm.eta > 0:
        out["dual_eta_theta"] = dual_D_eta(C, r, c, st.theta, cnorm, prm.eta)
    return out


def combined_gap(C: np.ndarray, X: np.ndarray, r: np.ndarray, c: np.ndarray, opt: float,
                 cnorm: float) -> float:
    """Equation (combined) as printed: <C, X - X*> + ||C||_inf(||col - c||_1 + ||row - r||_1)."""
    rr, cc, _ = residuals(X, r, c)
    return float(np.sum(C * X) - opt + cnorm * (rr + cc))


# --------------------------------------------------------------------------
# Envelope gradient (not in the paper: the derivative of the dual value at frozen duals)
# --------------------------------------------------------------------------


def envelope_value_rows(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, nu: np.ndarray,
                        lam: float, cnorm: float, kind: str = "sqeuclid") -> np.ndarray:
    """f_i(x_i) = r_i softmin^{1/lam}_j (C_ij + 2||C||_inf nu_j), C_ij = s dist(x_i, y_j), the
    i-th row term of D^eta(nu) (equation def:dual_spp_e) with eta = 1/lam and frozen s,
    ||C||_inf."""
    C = ground_cost(x, y, s, kind)
    return r * softmin(C + 2.0 * cnorm * nu[None, :], 1.0 / lam, axis=1)


def envelope_grad_x_metric(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, nu: np.ndarray,
                           lam: float, cnorm: float, kind: str) -> np.ndarray:
    """sum_j X_ij dC_ij/dx_i for the l1 and l_inf costs, X = diag(r) p^{1/lam}(nu):
    l1: dC_ij/dx_ik = s sign(x_ik - y_jk); l_inf: s sign(x_ik - y_jk) on the coordinate k of
    max_k |x_ik - y_jk| (the first one on ties), 0 elsewhere; sign(0) = 0.  Written with
    explicit loops over the pairs."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = ground_cost(x, y, s, kind)
    X = r[:, None] * dual_to_primal(C, nu, lam, cnorm)
    g = np.zeros_like(x)
    for i in range(x.shape[0]):
        for j in range(y.shape[0]):
            diff = x[i] - y[j]
            if kind == "l1":
                g[i] += X[i, j] * s * np.sign(diff)
            else:
                k = int(np.argmax(np.abs(diff)))
                g[i, k] += X[i, j] * s * np.sign(diff[k])
    return g


def envelope_grad_y(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, nu: np.ndarray,
                    lam: float, cnorm: float, kind: str = "sqeuclid") -> np.ndarray:
    """sum_i X_ij dC_ij/dy_j, X = diag(r) p^{1/lam}(nu): the derivative of
    D^eta(nu; x, y) = sum_i f_i(x_i) - 2||C||_inf <c, nu> with respect to y at frozen nu (Danskin).
    Squared Euclidean: dC_ij/dy_j = 2 s (y_j - x_i); l1: s sign(y_jk - x_ik); l_inf: the same on
    the coordinate of max_k |x_ik - y_jk| (first on ties); sign(0) = 0.  Explicit pair loops."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = ground_cost(x, y, s, kind)
    X = r[:, None] * dual_to_primal(C, nu, lam, cnorm)
    g = np.zeros_like(y)
    for j in range(y.shape[0]):
        for i in range(x.shape[0]):
            diff = y[j] - x[i]
            if kind == "sqeuclid":
                g[j] += X[i, j] * 2.0 * s * diff
            elif kind == "l1":
                g[j] += X[i, j] * s * np.sign(diff)
            else:
                k = int(np.argmax(np.abs(diff)))
                g[j, k] += X[i, j] * s * np.sign(diff[k])
    return g


def envelope_grad_y_columns(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, nu: np.ndarray,
                            lam: float, cnorm: float, cols, log_z: np.ndarray,
                            kind: str = "sqeuclid") -> np.ndarray:
    """The rows `cols` of envelope_grad_y, one column j at a time over every row i, given the row
    log-normalisers log Z_i = LSE_j(-lam (C_ij + 2||C||_inf nu_j)) of the same coupling (a full
    row pass supplies them at sizes where no n x m array fits; a column's gradient needs only
    its own column beside them): X_ij = r_i exp(-lam (C_ij + 2||C||_inf nu_j) - log Z_i)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    cols = np.asarray(cols, dtype=np.int64)
    g = np.zeros((cols.shape[0], y.shape[1]))
    for a, j in enumerate(cols):
        Cj = ground_cost(x, y[j:j + 1], s, kind)[:, 0]
        Xj = r * np.exp(-lam * (Cj + 2.0 * cnorm * nu[j]) - log_z)
        diff = y[j][None, :] - x
        if kind == "sqeuclid":
            g[a] = 2.0 * s * (Xj @ diff)
        elif kind == "l1":
            g[a] = s * (Xj @ np.sign(diff))
        else:
            k = np.argmax(np.abs(diff), axis=1)
            sg = np.sign(diff[np.arange(x.shape[0]), k])
            np.add.at(g[a], k, s * Xj * sg)
    return g


def envelope_grad_x(x: np.ndarray, y: np.ndarray, r: np.ndarray, s: float, nu: np.ndarray,
                    lam: float, cnorm: float) -> np.ndarray:
    """grad_{x_i} = sum_j X_ij dC_ij/dx_i = sum_j X_ij * 2 s (x_i - y_j), X = diag(r) p^{1/lam}(nu).
    This is the derivative of envelope_value_rows (Danskin); parity pinned by finite differences."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = sqeuclid_cost(x, y, s)
    X = r[:, None] * dual_to_primal(C, nu, lam, cnorm)
    g = np.zeros_like(x)
    for k in range(x.shape[1]):
        g[:, k] = np.sum(X * 2.0 * s * (x[:, k][:, None] - y[:, k][None, :]), axis=1)
    return g


# --------------------------------------------------------------------------
# The partial sums D_t of Proposition infeas_bound(b)
# --------------------------------------------------------------------------


def dual_entropy(nu: np.ndarray, calpha: np.ndarray) -> float:
    """H_c^alpha(nu) = sum_j c^alpha_j ((1+nu_j)/2 ln((1+nu_j)/2) + (1-nu_j)/2 ln((1-nu_j)/2)),
    the negative dual entropy of Section 3.1."""
    a = (1.0 + nu) / 2.0
    b = (1.0 - nu) / 2.0
    return float(calpha @ (a * np.log(a) + b * np.log(b)))


def dual_entropy_grad(nu: np.ndarray, calpha: np.ndarray) -> np.ndarray:
    """grad H_c^alpha(nu) = (1/2) c^alpha * ln((1+nu)/(1-nu))  (def:Ha_grad)."""
    return 0.5 * calpha * np.log((1.0 + nu) / (1.0 - nu))


def bregman_Ha(theta: np.ndarray, nu: np.ndarray, calpha: np.ndarray) -> float:
    """D_{H_c^alpha}(theta || nu) in the explicit form (def:DHa_explicit)."""
    a = (theta + 1.0) / 2.0 * np.log((theta + 1.0) / (nu + 1.0))
    b = (1.0 - theta) / 2.0 * np.log((1.0 - theta) / (1.0 - nu))
    return float(calpha @ (a + b))


def softplus(z: np.ndarray) -> np.ndarray:
    """ln(1 + e^z), evaluated without overflow."""
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def bregman_Ha_natural(a: np.ndarray, b: np.ndarray, calpha: np.ndarray) -> float:
    """D_{H_c^alpha}(tanh a || tanh b) from the natural parameters a, b (the tanh arguments of
    the mirror steps).  With theta = tanh a, (1 + theta)/2 = sigma(2a) and (1 - theta)/2 =
    sigma(-2a), so each coordinate of def:DHa_explicit is the Bernoulli KL
        sigma(2a) (2a - 2b) - softplus(2a) + softplus(2b),
    the same value in exact arithmetic, and finite where tanh a rounds to +-1 in floating point
    (a step with c^alpha_j ~ alpha/m and |col_j - c_j| >> c^alpha_j)."""
    sig = 0.5 * (1.0 + np.tanh(a))          # sigma(2a)
    return float(calpha @ (sig * (2.0 * a - 2.0 * b) - softplus(2.0 * a) + softplus(2.0 * b)))


def dt_sequence(C: np.ndarray, r: np.ndarray, c: np.ndarray, prm: Params, T: int,
                cnorm: float | None = None):
    """D_1, ..., D_T along Algorithm 2 from the start (def:sum_condition):

        D_t = sum_{s=0}^{t-1} D_H(thetabar^{s+1} || thetahat^{s+1}) - D_H(thetabar^{s+1} || theta^s)
                            + KL(Xbar^{s+1} || X^{s+1}) - KL(Xbar^{s+1} || X^s),

    with X^s = diag(r) p^{eta_s}(nu^s) and Xbar^{s+1} = diag(r) p^{eta_{s+1}}(nubar^{s+1})
    (Proposition infeas_bound), every KL taken on the dense matrices by its definition and the
    dual divergences from the steps' natural parameters (bregman_Ha_natural; theta^s is clipped
    to |theta| <= tanh(beta/2), so its parameter is atanh theta^s).
    Returns (array of D_t, final state, list of the iterates' traces)."""
    cnorm = float(np.max(np.abs(C))) if cnorm is None else cnorm
    prm = prm.resolved(cnorm)
    m = c.shape[0]
    calpha = c + prm.alpha / m
    st = lamp_init(m)
    X_s = plan(C, r, st, cnorm)
    D = 0.0
    out = []
    traces = []
    for _ in range(T):
        tr = LampTrace()
        nxt = lamp_step(C, r, c, st, prm, cnorm, tr)
        Xbar = r[:, None] * dual_to_primal(C, tr.nubar[0], nxt.lam, cnorm)
        X_next = plan(C, r, nxt, cnorm)
        a_bar, a_hat, b = tr.theta_bar_arg[0], tr.theta_hat_arg[0], np.arctanh(st.theta)
        D += (bregman_Ha_natural(a_bar, a_hat, calpha)
              - bregman_Ha_natural(a_bar, b, calpha)
              + kl(Xbar, X_next) - kl(Xbar, X_s))
        out.append(D)
        traces.append(tr)
        st, X_s = nxt, X_next
    return np.array(out), st, traces


def midpoint_bound(dt: float, t: int, m: int, alpha: float, cnorm: float) -> float:
    """Right-hand side of (ineq:spp_midpoint_conv): 2||C||_inf (log m + (1+alpha) log 2 + D_t) / t."""
    return 2.0 * cnorm * (math.log(m) + (1.0 + alpha) * math.log(2.0) + dt) / t
