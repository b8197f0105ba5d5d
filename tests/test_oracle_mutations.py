"""The oracle's pins are sensitive: each test plants one plausible mistake in an oracle
function (on the CPU, through monkeypatch) and checks that a pin in test_oracle_pins
fails.  Nothing here runs on a GPU."""
import math

import numpy as np
import pytest

from oracle import lamp as L
from tests import test_oracle_pins as pins


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_pin_tclip_radius():
    """beta = log 3 clips at exactly 1/2 (Algorithm 4)."""
    th = np.array([-0.9, -0.5, 0.2, 0.7])
    np.testing.assert_allclose(L.tclip(th, math.log(3.0)), [-0.5, -0.5, 0.2, 0.5], rtol=1e-15)


def test_mutation_dual_map_sign(monkeypatch):
    orig = L.dual_mirror_map
    monkeypatch.setattr(L, "dual_mirror_map",
                        lambda th0, colp, c, ca, tau, cn: orig(th0, 2 * c - colp, c, ca, tau, cn))
    _fails(pins.test_dual_mirror_map_is_the_argmax)


def test_mutation_dual_map_without_alpha(monkeypatch):
    orig = L.dual_mirror_map
    monkeypatch.setattr(L, "dual_mirror_map",
                        lambda th0, colp, c, ca, tau, cn: orig(th0, colp, c, c, tau, cn))
    _fails(pins.test_dual_mirror_map_is_the_argmax)


def test_mutation_tclip_radius(monkeypatch):
    monkeypatch.setattr(L, "tclip", lambda th, beta: np.clip(th, -math.tanh(beta), math.tanh(beta)))
    _fails(test_pin_tclip_radius)


def test_mutation_schedule_drops_decay(monkeypatch):
    def bad(T, tau1, eta):
        lam = np.zeros(T + 1)
        for t in range(T):
            lam[t + 1] = tau1 + lam[t]
        return lam
    monkeypatch.setattr(L, "inv_eta_schedule", bad)
    _fails(pins.test_inverse_temperature_closed_form, 1e-2)


def test_mutation_averaging_weight_uses_old_temperature(monkeypatch):
    orig_step = L.lamp_step

    def bad_step(C, r, c, state, prm, cnorm, trace=None):
        # w = tau1 / lam_t instead of tau1 / lam_{t+1}
        m = c.shape[0]
        calpha = c + prm.alpha / m
        lam_next = prm.tau1 + state.lam * (1.0 - prm.tau1 * prm.eta)
        w = prm.tau1 / max(state.lam, prm.tau1)
        nu, theta = state.nu, state.theta
        nubar = nu + w * (theta - nu)
        colA = L.col_r(L.dual_to_primal(C, nu, state.lam, cnorm), r)
        tb = L.dual_mirror_map(theta, colA, c, calpha, prm.tau2, cnorm)
        nu_next = nu + w * (tb - nu)
        colB = L.col_r(L.dual_to_primal(C, nubar, lam_next, cnorm), r)
        th = L.tclip(L.dual_mirror_map(theta, colB, c, calpha, prm.tau2, cnorm), prm.beta)
        if trace is not None:
            trace.nubar.append(nubar)
            trace.nu.append(nu_next)
            trace.theta.append(th)
        return L.LampState(state.t + 1, lam_next, nu_next, th)

    monkeypatch.setattr(L, "lamp_step", bad_step)
    assert orig_step is not bad_step
    _fails(pins.test_lamp_equals_pdmp, 1e-2)


def test_mutation_midpoint_uses_thetabar(monkeypatch):
    """nubar^{t+1} built from thetabar^{t+1} instead of theta^t."""
    def bad_step(C, r, c, state, prm, cnorm, trace=None):
        m = c.shape[0]
        calpha = c + prm.alpha / m
        lam_next = prm.tau1 + state.lam * (1.0 - prm.tau1 * prm.eta)
        w = prm.tau1 / lam_next
        nu, theta = state.nu, state.theta
        colA = L.col_r(L.dual_to_primal(C, nu, state.lam, cnorm), r)
        tb = L.dual_mirror_map(theta, colA, c, calpha, prm.tau2, cnorm)
        nubar = nu + w * (tb - nu)
        nu_next = nu + w * (tb - nu)
        colB = L.col_r(L.dual_to_primal(C, nubar, lam_next, cnorm), r)
        th = L.tclip(L.dual_mirror_map(theta, colB, c, calpha, prm.tau2, cnorm), prm.beta)
        if trace is not None:
            trace.nubar.append(nubar)
            trace.nu.append(nu_next)
            trace.theta.append(th)
        return L.LampState(state.t + 1, lam_next, nu_next, th)

    monkeypatch.setattr(L, "lamp_step", bad_step)
    _fails(pins.test_lamp_equals_pdmp, 0.0)


def test_mutation_column_normalised_map(monkeypatch):
    """Normalising p^eta(theta) over columns instead of rows (a transposed operand)."""
    from scipy.special import logsumexp

    def bad(C, theta, lam, cnorm):
        a = -lam * (C + 2.0 * cnorm * theta[None, :])
        return np.exp(a - logsumexp(a, axis=0, keepdims=True))
    monkeypatch.setattr(L, "dual_to_primal", bad)
    _fails(pins.test_row_feasibility)


def test_mutation_round_skips_column_scaling(monkeypatch):
    def bad(X, r, c):
        xr = np.minimum(r / L.row(X), 1.0)
        X2 = xr[:, None] * X
        dr = r - L.row(X2)
        dc = c - L.col(X2)
        return X2 + np.outer(dr, dc) / np.abs(dr).sum()
    monkeypatch.setattr(L, "round_plan", bad)
    _fails(pins.test_round_feasible_and_l1_bound)


def test_mutation_dual_drops_linear_term(monkeypatch):
    def bad(C, r, c, theta, cnorm):
        return float(r @ np.min(C + 2.0 * cnorm * theta[None, :], axis=1))
    monkeypatch.setattr(L, "dual_D", bad)
    _fails(pins.test_dual_function_attains_lp_optimum)


def test_mutation_gradient_factor(monkeypatch):
    orig = L.envelope_grad_x
    monkeypatch.setattr(L, "envelope_grad_x", lambda *a: 0.5 * orig(*a))
    _fails(pins.test_envelope_gradient_matches_finite_differences)


def test_mutation_column_gradient_without_normaliser(monkeypatch):
    """Forgetting the row log-normaliser in X_ij (the unnormalised coupling)."""
    orig = L.envelope_grad_y_columns
    monkeypatch.setattr(L, "envelope_grad_y_columns",
                        lambda x, y, r, s, nu, lam, cn, cols, lz, kind="sqeuclid":
                        orig(x, y, r, s, nu, lam, cn, cols, np.zeros_like(lz), kind))
    _fails(pins.test_envelope_gradient_columns_by_finite_differences, "sqeuclid")


def test_mutation_column_gradient_sign(monkeypatch):
    """x - y in place of y - x."""
    orig = L.envelope_grad_y_columns
    monkeypatch.setattr(L, "envelope_grad_y_columns", lambda *a, **k: -orig(*a, **k))
    _fails(pins.test_envelope_gradient_columns_by_finite_differences, "l1")


def test_mutation_dt_kl_arguments_swapped(monkeypatch):
    """KL(X^{s+1} || Xbar) in place of KL(Xbar || X^{s+1}) in the D_t summand."""
    orig = L.kl
    monkeypatch.setattr(L, "kl", lambda X, Y: orig(Y, X))
    _fails(pins.test_dt_summands_match_the_dual_and_primal_identities, 0.0)


def test_mutation_dt_dual_divergence_arguments_swapped(monkeypatch):
    """D_H(thetahat || thetabar) in place of D_H(thetabar || thetahat)."""
    orig = L.bregman_Ha_natural
    monkeypatch.setattr(L, "bregman_Ha_natural", lambda a, b, w: orig(b, a, w))
    _fails(pins.test_dt_summands_match_the_dual_and_primal_identities, 0.0)


def test_mutation_dt_dual_divergence_unweighted(monkeypatch):
    """The weights c^alpha dropped from the dual divergence."""
    orig = L.bregman_Ha_natural
    monkeypatch.setattr(L, "bregman_Ha_natural", lambda a, b, w: orig(a, b, np.ones_like(w)))
    _fails(pins.test_dt_summands_match_the_dual_and_primal_identities, 0.0)
    _fails(pins.test_dual_bregman_from_natural_parameters_high_precision)


def test_mutation_prop_bound_residual_coefficient(monkeypatch):
    """8 ||C||_inf in place of 4 ||C||_inf on the column residual."""
    monkeypatch.setattr(L, "prop_bound",
                        lambda cr, t, m, cn: 8.0 * cn * cr + 2.0 * cn * math.log(m) / t)
    _fails(pins.test_prop_bound_exact_value_on_one_step_example)


def test_mutation_prop_bound_log_nm(monkeypatch):
    """log(n m) in place of log m (n = m in the pin)."""
    monkeypatch.setattr(L, "prop_bound",
                        lambda cr, t, m, cn: 4.0 * cn * cr + 2.0 * cn * math.log(m * m) / t)
    _fails(pins.test_prop_bound_exact_value_on_one_step_example)


def test_mutation_midpoint_bound_drops_alpha(monkeypatch):
    """(1 + alpha) log 2 written as log 2."""
    monkeypatch.setattr(L, "midpoint_bound",
                        lambda dt, t, m, a, cn: 2.0 * cn * (math.log(m) + math.log(2.0) + dt) / t)
    _fails(pins.test_midpoint_bound_exact_value_on_one_step_example, 0.5)


def test_mutation_midpoint_bound_log_nm(monkeypatch):
    monkeypatch.setattr(L, "midpoint_bound", lambda dt, t, m, a, cn: 2.0 * cn * (
        math.log(m * m) + (1.0 + a) * math.log(2.0) + dt) / t)
    _fails(pins.test_midpoint_bound_exact_value_on_one_step_example, 0.01)


def test_mutation_dual_eta_sign_of_theta(monkeypatch):
    """C - 2||C||_inf theta inside the softmin."""
    def bad(C, r, c, theta, cnorm, eta):
        return float(r @ L.softmin(C - 2.0 * cnorm * theta[None, :], eta, axis=1)
                     - 2.0 * cnorm * (c @ theta))
    monkeypatch.setattr(L, "dual_D_eta", bad)
    _fails(pins.test_dual_eta_strong_duality_at_the_sinkhorn_plan)
    _fails(pins.test_dual_eta_is_the_minimum_over_row_stochastic_plans)


def test_mutation_dual_eta_temperature_inverted(monkeypatch):
    """softmin taken at 1/eta (the inverse temperature) in place of eta."""
    def bad(C, r, c, theta, cnorm, eta):
        return float(r @ L.softmin(C + 2.0 * cnorm * theta[None, :], 1.0 / eta, axis=1)
                     - 2.0 * cnorm * (c @ theta))
    monkeypatch.setattr(L, "dual_D_eta", bad)
    _fails(pins.test_dual_eta_sandwich_and_zero_temperature_limit, 1e-3)


def test_mutation_dual_eta_drops_linear_term(monkeypatch):
    def bad(C, r, c, theta, cnorm, eta):
        return float(r @ L.softmin(C + 2.0 * cnorm * theta[None, :], eta, axis=1))
    monkeypatch.setattr(L, "dual_D_eta", bad)
    _fails(pins.test_dual_eta_is_the_minimum_over_row_stochastic_plans)


def test_mutation_primal_penalty_factor(monkeypatch):
    """||C||_inf in place of 2 ||C||_inf on the infeasibility."""
    def bad(C, X, r, c, cnorm, eta=0.0):
        rr, cc, _ = L.residuals(X, r, c)
        return float(np.sum(C * X) + cnorm * (rr + cc) - eta * L.entropy(X))
    monkeypatch.setattr(L, "primal_penalised", bad)
    _fails(pins.test_primal_penalised_values_and_weak_duality)


def test_mutation_primal_entropy_sign(monkeypatch):
    def bad(C, X, r, c, cnorm, eta=0.0):
        rr, cc, _ = L.residuals(X, r, c)
        return float(np.sum(C * X) + 2.0 * cnorm * (rr + cc) + eta * L.entropy(X))
    monkeypatch.setattr(L, "primal_penalised", bad)
    _fails(pins.test_primal_penalised_values_and_weak_duality)


def test_mutation_combined_gap_factor(monkeypatch):
    """The rounding lemma's 2 ||C||_inf in place of the printed ||C||_inf."""
    def bad(C, X, r, c, opt, cnorm):
        rr, cc, _ = L.residuals(X, r, c)
        return float(np.sum(C * X) - opt + 2.0 * cnorm * (rr + cc))
    monkeypatch.setattr(L, "combined_gap", bad)
    _fails(pins.test_combined_gap_values)
