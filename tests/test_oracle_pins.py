"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form,
a worked example, a textbook/library routine (brute force, assignment, LP,
Sinkhorn), an identity or an error bound stated in the paper, or finite
differences.  CPU only.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.special import logsumexp

from oracle import exact
from oracle import lamp as L
from oracle import stream
from paper_2511_11359_amd import workloads as W


def _problem(n, m, d, seed, uniform=False):
    wl = W.random_small(n, m, d, seed, uniform=uniform)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_sqdist(x, y)
    C = L.sqeuclid_cost(x, y, s)
    return C, wl.r, wl.c, x, y, s


# ---------------------------------------------------------------- schedule


@pytest.mark.parametrize("eta", [0.0, 1e-3, 1e-2, 0.3])
def test_inverse_temperature_closed_form(eta):
    """eta_t^-1 = (1 - (1 - tau1 eta)^t)/eta, -> tau1 t as eta -> 0 (remark after Alg. 2)."""
    tau1 = 0.5
    lam = L.inv_eta_schedule(400, tau1, eta)
    t = np.arange(401)
    ref = tau1 * t if eta == 0 else (1.0 - (1.0 - tau1 * eta) ** t) / eta
    assert lam[1] == pytest.approx(tau1, rel=1e-15)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=0)


# ---------------------------------------------------------------- mirror maps


def test_dual_mirror_map_is_the_argmax():
    """The closed form (def:closed_form_opt) maximises tau<grad G, theta> - D_{H_c^alpha}(theta||theta0)
    coordinate by coordinate (def:mirror_maps); solved here by a bounded 1-D search."""
    g = np.random.default_rng(0)
    m, cnorm, tau = 7, 1.7, 0.3
    c = g.dirichlet(np.ones(m))
    calpha = c + 0.01 / m
    theta0 = g.uniform(-0.8, 0.8, m)
    colp = g.dirichlet(np.ones(m))
    closed = L.dual_mirror_map(theta0, colp, c, calpha, tau, cnorm)
    grad = 2.0 * cnorm * (colp - c)      # gradient of K(X, .) in theta (problem spp)
    for j in range(m):
        def neg(th):
            a = (th + 1) / 2 * math.log((th + 1) / (theta0[j] + 1))
            b = (1 - th) / 2 * math.log((1 - th) / (1 - theta0[j]))
            return -(tau * grad[j] * th - calpha[j] * (a + b))
        res = minimize_scalar(neg, bounds=(-1 + 1e-12, 1 - 1e-12), method="bounded",
                              options=dict(xatol=1e-13))
        assert res.x == pytest.approx(closed[j], abs=1e-7)


def test_primal_mirror_map_optimality_conditions():
    """M_tau^eta(p0; theta) (def:closed_form_opt) satisfies the optimality conditions of its
    definition (def:mirror_maps): within each row, tau r_i (C + eta(log p0 + 1) + K theta)_ij
    + r_i log(p_ij / p0_ij) is constant in j, and p is row-stochastic."""
    g = np.random.default_rng(1)
    n, m, tau, eta, cnorm = 4, 6, 0.4, 0.05, 2.0
    C = g.random((n, m)) * cnorm
    r = g.dirichlet(np.ones(n))
    p0 = g.dirichlet(np.ones(m), size=n)
    theta = g.uniform(-1, 1, m)
    p = L.primal_mirror_map(p0, theta, C, tau, eta, cnorm)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, atol=1e-14)
    grad = r[:, None] * (C + eta * (np.log(p0) + 1.0) + 2.0 * cnorm * theta[None, :])
    stat = tau * grad + r[:, None] * np.log(p / p0)
    np.testing.assert_allclose(stat - stat[:, :1], 0.0, atol=1e-12)


def test_lemma_primal_md_eq_dual_avg():
    """p^{eta'}(theta') = M_tau^eta(p^gamma(theta_a); theta_b) with eta' = gamma/(1 + tau(gamma - eta)),
    theta' = theta_a + tau eta' (theta_b - theta_a)  (Lemma primal_md_eq_dual_avg)."""
    g = np.random.default_rng(2)
    n, m, cnorm = 5, 8, 1.3
    C = g.random((n, m)) * cnorm
    for eta, gamma, tau in [(0.0, 0.7, 0.4), (0.05, 0.2, 0.5), (0.5, 3.0, 1.9)]:
        assert tau * eta <= 1
        ta, tb = g.uniform(-1, 1, m), g.uniform(-1, 1, m)
        eta_p = gamma / (1.0 + tau * (gamma - eta))
        theta_p = ta + tau * eta_p * (tb - ta)
        lhs = L.dual_to_primal(C, theta_p, 1.0 / eta_p, cnorm)
        rhs = L.primal_mirror_map(L.dual_to_primal(C, ta, 1.0 / gamma, cnorm), tb, C, tau, eta, cnorm)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- LAMP == PDMP


@pytest.mark.parametrize("eta", [0.0, 1e-3, 1e-2, 0.2])
def test_lamp_equals_pdmp(eta):
    """p^t = p^{eta_t}(nu^t) and pbar^{t+1} = p^{eta_{t+1}}(nubar^{t+1}) (Proposition equivalence):
    Algorithm 2 (dual-only) against Algorithm 1 (explicit primal iterates), n != m."""
    C, r, c, *_ = _problem(9, 6, 2, seed=3)
    cnorm = float(C.max())
    prm = L.Params(eta=eta)
    T = 60
    ps, pbars, thetas = L.pdmp_dense(C, r, c, prm, T, cnorm)
    st, tr = L.lamp_dense(C, r, c, prm, T, cnorm)
    lam = L.inv_eta_schedule(T, prm.resolved(cnorm).tau1, eta)
    nu = np.zeros(6)
    for t in range(T):
        np.testing.assert_allclose(L.dual_to_primal(C, nu, lam[t], cnorm), ps[t], rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(L.dual_to_primal(C, tr.nubar[t], lam[t + 1], cnorm), pbars[t + 1],
                                   rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(tr.theta[t], thetas[t + 1], atol=1e-12)
        nu = tr.nu[t]


def test_first_iterate_closed_form():
    """eta_0 = inf: p^{eta_0}(0) = 1/m, so col(X^0) = 1/m, thetabar^1 = tanh(kappa (1/m - c)/c^alpha),
    w_1 = 1 so nu^1 = thetabar^1 and nubar^1 = theta^0 = 0 (Alg. 2, proof of Prop. equivalence)."""
    C, r, c, *_ = _problem(7, 5, 3, seed=4)
    cnorm = float(C.max())
    prm = L.Params(eta=1e-3)
    st, tr = L.lamp_dense(C, r, c, prm, 1, cnorm)
    m = 5
    calpha = c + 0.01 / m
    kappa = 2 * (1 / (2 * cnorm)) * cnorm
    np.testing.assert_allclose(tr.colA[0], np.full(m, 1.0 / m), rtol=1e-14)
    np.testing.assert_allclose(tr.theta_bar[0], np.tanh(kappa * (1 / m - c) / calpha), rtol=1e-13)
    np.testing.assert_allclose(st.nu, tr.theta_bar[0], rtol=1e-13)
    np.testing.assert_array_equal(tr.nubar[0], np.zeros(m))
    np.testing.assert_allclose(tr.logZA[0], np.full(7, math.log(m)), rtol=1e-14)


def test_symmetric_two_by_two_worked_example():
    """C = [[0,1],[1,0]], r = c = (1/2, 1/2), eta = 0: by symmetry col(X^t) = c, so theta = nu = 0
    for all t, lam_t = t/2 and <C, X^t> = e^{-t/2}/(1 + e^{-t/2}); the bound of Proposition
    infeas_bound(a) is 2 log 2 / t."""
    C = np.array([[0.0, 1.0], [1.0, 0.0]])
    r = c = np.array([0.5, 0.5])
    prm = L.Params(eta=0.0)
    st = L.lamp_init(2)
    for t in range(1, 40):
        st = L.lamp_step(C, r, c, st, prm.resolved(1.0), 1.0)
        assert st.t == t and st.lam == pytest.approx(t / 2, rel=1e-15)
        np.testing.assert_allclose(st.theta, 0.0, atol=1e-14)
        np.testing.assert_allclose(st.nu, 0.0, atol=1e-14)
        X = L.plan(C, r, st, 1.0)
        e = math.exp(-t / 2)
        assert float(np.sum(C * X)) == pytest.approx(e / (1 + e), rel=1e-13)
        assert float(np.sum(C * L.round_plan(X, r, c))) <= L.prop_bound(0.0, t, 2, 1.0)


def test_circulant_polygon_closed_form():
    """Regular n-gon, x = y, uniform marginals: the cost is circulant, so every column of X^t sums
    to 1/n, theta = nu = 0 and log Z_i = LSE_j(-lam_t C_0j) for every i."""
    n = 12
    ang = 2 * np.pi * np.arange(n) / n
    x = np.stack([np.cos(ang), np.sin(ang)], 1)
    C = L.sqeuclid_cost(x, x, 0.25)              # ||C||_inf = 1
    r = c = np.full(n, 1.0 / n)
    st, tr = L.lamp_dense(C, r, c, L.Params(eta=1e-2), 50, 1.0)
    for t in range(50):
        np.testing.assert_allclose(tr.colA[t], 1.0 / n, rtol=1e-12)
        np.testing.assert_allclose(tr.theta[t], 0.0, atol=1e-12)
        np.testing.assert_allclose(tr.logZA[t], logsumexp(-tr.lam[t] * C[0]), rtol=1e-13)


def test_row_feasibility():
    """row(X^t) = r for every t (eq:row_feasible)."""
    C, r, c, *_ = _problem(10, 7, 2, seed=5)
    cnorm = float(C.max())
    st = L.lamp_init(7)
    prm = L.Params(eta=0.0).resolved(cnorm)
    for _ in range(30):
        st = L.lamp_step(C, r, c, st, prm, cnorm)
        X = L.plan(C, r, st, cnorm)
        np.testing.assert_allclose(L.row(X), r, rtol=1e-13)


# ---------------------------------------------------------------- Round


def test_round_feasible_and_l1_bound():
    """Round(X, r, c) is in Pi(r, c) and ||X - Round X||_1 <= 2(||row - r||_1 + ||col - c||_1)
    (Algorithm 3, Lemma jason_rounding)."""
    g = np.random.default_rng(6)
    for _ in range(20):
        n, m = g.integers(2, 9, 2)
        X = g.random((n, m)) ** 3
        X /= X.sum() * g.uniform(0.7, 1.3)
        r, c = g.dirichlet(np.ones(n)), g.dirichlet(np.ones(m))
        Xt = L.round_plan(X, r, c)
        assert Xt.min() >= -1e-15
        np.testing.assert_allclose(Xt.sum(1), r, atol=1e-14)
        np.testing.assert_allclose(Xt.sum(0), c, atol=1e-14)
        rr, cc, _ = L.residuals(X, r, c)
        assert np.abs(X - Xt).sum() <= 2 * (rr + cc) + 1e-13


# ---------------------------------------------------------------- ground truth


def test_exact_solvers_agree():
    """Brute force over permutations, the assignment solver and the HiGHS LP agree (Birkhoff)."""
    g = np.random.default_rng(7)
    for n in [2, 3, 5, 7]:
        C = g.random((n, n))
        u = np.full(n, 1.0 / n)
        bf = exact.brute_force_ot_uniform(C)
        assert exact.assignment_ot_uniform(C) == pytest.approx(bf, rel=1e-12)
        assert exact.lp_ot(C, u, u)[0] == pytest.approx(bf, rel=1e-8)


@pytest.mark.parametrize("eta,beta", [(0.0, 1.1), (0.0, math.log(3)), (1e-2, 1.1)])
def test_certificate_ordering_and_last_iterate_bound(eta, beta):
    """For every t >= 1: D(theta^t) <= OPT <= <C, Round X^t> <= P(X^t) (Appendix B duality,
    Lemma jason_rounding), and for eta = 0 the last-iterate bounds of Proposition infeas_bound(a):
    <C, Round X^t> - OPT <= 4||C||_inf ||col(X^t) - c||_1 + 2||C||_inf log m / t, and the
    intermediate bound <C, X^t - X*> <= 2||C||_inf <-nu^t, col - c> + 2||C||_inf KL(X*||X^0)/t."""
    n = m = 6
    C, r, c, *_ = _problem(n, m, 2, seed=8)
    cnorm = float(C.max())
    opt, Xstar = exact.lp_ot(C, r, c)
    prm = L.Params(eta=eta, beta=beta).resolved(cnorm)
    X0 = r[:, None] * np.full((n, m), 1.0 / m)
    klstar = L.kl(np.maximum(Xstar, 0), X0)
    st = L.lamp_init(m)
    for t in range(1, 400):
        st = L.lamp_step(C, r, c, st, prm, cnorm)
        cert = L.certificate(C, r, c, st, prm, cnorm)
        assert cert["dual_theta"] <= opt + 1e-12
        assert cert["dual_nu"] <= opt + 1e-12
        assert opt <= cert["rounded_cost"] + 1e-12
        assert cert["rounded_cost"] <= cert["primal_penalized"] + 1e-12
        if eta == 0.0:
            assert cert["rounded_cost"] - opt <= cert["prop_bound"] + 1e-12
            X = L.plan(C, r, st, cnorm)
            ib = L.intermediate_bound(L.col(X), c, st.nu, klstar, t, cnorm)
            assert cert["cost"] - opt <= ib + 1e-12


def test_dual_function_attains_lp_optimum():
    """Strong duality for the saddle dual (def:dual_spp): with the LP's optimal column dual y_c,
    D(theta) at K theta = -y_c equals OPT (proof of Lemma b_choice), and D is invariant to
    adding a constant to theta (r and c both sum to 1)."""
    C, r, c, *_ = _problem(6, 5, 2, seed=17)
    cnorm = float(C.max())
    opt, yr, yc = exact.lp_ot_duals(C, r, c)
    theta = -yc / (2.0 * cnorm)
    assert L.dual_D(C, r, c, theta, cnorm) == pytest.approx(opt, rel=1e-9, abs=1e-12)
    assert L.dual_D(C, r, c, theta + 0.1, cnorm) == pytest.approx(opt, rel=1e-9, abs=1e-12)


def test_lamp_converges_to_assignment_optimum():
    """eta = 0 on uniform n = m = 5 (brute-force OPT): the certificate gap closes."""
    g = np.random.default_rng(9)
    x, y = g.random((5, 2)), g.random((5, 2))
    C = L.sqeuclid_cost(x, y, 1.0 / L.max_sqdist(x, y))
    u = np.full(5, 0.2)
    opt = exact.brute_force_ot_uniform(C)
    st, _ = L.lamp_dense(C, u, u, L.Params(eta=0.0), 20000, 1.0, trace=False)
    cert = L.certificate(C, u, u, st, L.Params(eta=0.0).resolved(1.0), 1.0)
    assert cert["rounded_cost"] - opt <= cert["prop_bound"]
    assert cert["rounded_cost"] == pytest.approx(opt, abs=5e-4)
    assert max(cert["dual_theta"], cert["dual_nu"]) == pytest.approx(opt, abs=5e-4)


def test_eot_fixed_point_is_the_sinkhorn_plan():
    """For 0 < eta <= ||C||_inf / log(max_j 1/c_j) the penalised problem and EOT share their unique
    minimiser (Lemma l1_prob_equiv(b)); LAMP's plan converges to the Sinkhorn EOT plan."""
    C, r, c, *_ = _problem(5, 4, 2, seed=10)
    cnorm = float(C.max())
    eta = 0.05
    assert eta <= cnorm / math.log(1 / c.min())
    Xs = exact.sinkhorn_eot(C, r, c, eta)
    st, _ = L.lamp_dense(C, r, c, L.Params(eta=eta), 20000, cnorm, trace=False)
    X = L.plan(C, r, st, cnorm)
    np.testing.assert_allclose(X, Xs, atol=1e-7)


def test_pd_obj_relation_identity():
    """-<r, log Z^t(theta)> - t<col(X~), theta> = (t/2)<C, X~> - H(X~) + H(r) with ||C||_inf = 1,
    X~ = diag(r) p^{eta_t}(theta), eta_t = 2/t (Lemma pd_obj_relation)."""
    C, r, c, *_ = _problem(6, 9, 2, seed=11)
    g = np.random.default_rng(12)
    for t in [1, 3, 17]:
        theta = g.uniform(-1, 1, 9)
        Xt = r[:, None] * L.dual_to_primal(C, theta, t / 2.0, 1.0)
        logZ = logsumexp(-t * (C / 2.0 + theta[None, :]), axis=1)
        lhs = -(r @ logZ) - t * (L.col(Xt) @ theta)
        rhs = t / 2.0 * np.sum(C * Xt) - L.entropy(Xt) + L.entropy(r[:, None])
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------- gradient


def test_envelope_gradient_matches_finite_differences():
    """grad_{x_i} sum_j X_ij C_ij at frozen (nu, lam, s) equals the derivative of
    r_i softmin_j(C_ij + K nu_j) (Danskin); central differences in FP64."""
    g = np.random.default_rng(13)
    x, y = g.random((6, 3)), g.random((8, 3))
    r = g.dirichlet(np.ones(6))
    nu = g.uniform(-0.5, 0.5, 8)
    s, lam, cnorm = 0.7, 40.0, 1.0
    G = L.envelope_grad_x(x, y, r, s, nu, lam, cnorm)
    h = 1e-6
    for i in range(6):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (L.envelope_value_rows(xp, y, r, s, nu, lam, cnorm)[i]
                  - L.envelope_value_rows(xm, y, r, s, nu, lam, cnorm)[i]) / (2 * h)
            assert G[i, k] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_envelope_gradient_of_the_eot_value():
    """At LAMP's EOT fixed point the envelope gradient equals d/dx of the re-solved EOT value
    V(x) = min_{X in Pi(r,c)} <C(x), X> - eta H(X) (Sinkhorn re-solve per perturbation)."""
    g = np.random.default_rng(14)
    x, y = g.random((4, 2)), g.random((4, 2))
    r, c = np.full(4, 0.25), np.full(4, 0.25)
    s = 1.0 / L.max_sqdist(x, y)
    eta = 0.05
    C = L.sqeuclid_cost(x, y, s)
    st, _ = L.lamp_dense(C, r, c, L.Params(eta=eta), 20000, 1.0, trace=False)
    G = L.envelope_grad_x(x, y, r, s, st.nu, st.lam, 1.0)

    def V(xx):
        Cx = L.sqeuclid_cost(xx, y, s)
        X = exact.sinkhorn_eot(Cx, r, c, eta)
        return float(np.sum(Cx * X) - eta * L.entropy(X))

    h = 1e-5
    for i, k in itertools.product(range(4), range(2)):
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        assert G[i, k] == pytest.approx((V(xp) - V(xm)) / (2 * h), rel=1e-4, abs=1e-7)


# ---------------------------------------------------------------- streaming form


def test_stream_step_matches_dense_step():
    """The row-block evaluation gives the same iteration as the dense one (n != m, several blocks
    with a ragged tail)."""
    wl = W.random_small(150, 70, 3, seed=15)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_sqdist(x, y)
    C = L.sqeuclid_cost(x, y, s)
    prm = L.Params(eta=1e-3)
    st, tr = L.lamp_dense(C, wl.r, wl.c, prm, 25, 1.0)
    lam = st.lam
    lam2, nu2, th2, info = stream.lamp_step_stream(x, y, wl.r, wl.c, s, 1.0, st.t, lam, st.nu,
                                                   st.theta, prm, block=64)
    st2, tr2 = L.lamp_dense(C, wl.r, wl.c, prm, 1, 1.0, state=st)
    np.testing.assert_allclose(nu2, st2.nu, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(th2, st2.theta, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(info["logZA"], tr2.logZA[0], rtol=1e-13)
    np.testing.assert_allclose(info["colB"], tr2.colB[0], rtol=1e-11)
    rows = [0, 63, 64, 149]
    np.testing.assert_allclose(stream.row_log_normalisers(x, y, s, 1.0, st.nu, lam, rows),
                               tr2.logZA[0][rows], rtol=1e-13)


@pytest.mark.parametrize("eta", [0.0, 1e-2])
def test_rowpass_c_step_matches_dense_step(eta):
    """The C full-size pass (every row's log-normaliser, listed columns' marginals and dual
    steps) gives the dense iteration, for the difference-form cost of FP32 points and for a cost
    given by separate norms and FP64 inner products (here built from the same points, so both
    define the same C up to rounding)."""
    from oracle import rowpass
    wl = W.random_small(150, 97, 4, seed=18)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_sqdist(x, y)
    C = L.sqeuclid_cost(x, y, s)
    prm = L.Params(eta=eta)
    st, _ = L.lamp_dense(C, wl.r, wl.c, prm, 30, 1.0, trace=False)
    st2, tr = L.lamp_dense(C, wl.r, wl.c, prm, 1, 1.0, state=st)
    cols = np.array([0, 1, 31, 32, 63, 64, 95, 96])
    gram = (x, y, np.sum(x * x, axis=1), np.sum(y * y, axis=1))
    for cost, rtol in [(rowpass.Cost(s, 1.0, x=wl.x, y=wl.y), 1e-12), (rowpass.Cost(s, 1.0, gram=gram), 1e-9)]:
        out = rowpass.step_sampled(cost, wl.r, wl.c, st.lam, st.nu, st.theta, prm, 1.0, cols)
        np.testing.assert_allclose(out["logZA"], tr.logZA[0], rtol=rtol, atol=1e-13)
        np.testing.assert_allclose(out["logZB"], tr.logZB[0], rtol=rtol, atol=1e-13)
        for key, ref in [("colA", tr.colA[0]), ("colB", tr.colB[0]), ("theta_bar", tr.theta_bar[0]),
                         ("theta_hat", tr.theta_hat[0]), ("nu", st2.nu), ("theta", st2.theta)]:
            np.testing.assert_allclose(out[key], ref[cols], rtol=rtol, atol=1e-14, err_msg=key)
        assert out["lam_next"] == st2.lam
    # whole runs to a tolerance: the same stopping iterate as the dense run
    st_d, _ = L.lamp_dense(C, wl.r, wl.c, prm, 3000, 1.0, tol=1e-4, trace=False)
    run = rowpass.solve(rowpass.Cost(s, 1.0, x=wl.x, y=wl.y), wl.r, wl.c, prm, 1.0, 3000, tol=1e-4, keep=(7,))
    assert run["t"] == st_d.t and run["res"] <= 1e-4
    np.testing.assert_allclose(run["nu"], st_d.nu, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(run["theta"], st_d.theta, rtol=1e-10, atol=1e-13)
    assert run["lam"] == pytest.approx(st_d.lam, rel=1e-15)
    st7, _ = L.lamp_dense(C, wl.r, wl.c, prm, 7, 1.0, trace=False)
    np.testing.assert_allclose(run["saved"][7][1], st7.nu, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("eta", [0.0, 1e-2])
def test_rowpass_c_row_costs_give_the_plan_cost(eta):
    """The C pass's per-row expected costs E_i = sum_j p_ij C_ij (given its row log-normalisers):
    r . E equals <C, X^t> of the dense certificate, and E_i equals the row's share, for both
    cost forms, at the state after 30 iterations (n != m)."""
    from oracle import rowpass
    wl = W.random_small(150, 97, 4, seed=19)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_sqdist(x, y)
    C = L.sqeuclid_cost(x, y, s)
    prm = L.Params(eta=eta)
    st, _ = L.lamp_dense(C, wl.r, wl.c, prm, 30, 1.0, trace=False)
    ref = L.certificate(C, wl.r, wl.c, st, prm, 1.0)["cost"]
    rows_ref = np.sum(L.plan(C, wl.r, st, 1.0) * C, axis=1) / wl.r
    gram = (x, y, np.sum(x * x, axis=1), np.sum(y * y, axis=1))
    for cost, rtol in [(rowpass.Cost(s, 1.0, x=wl.x, y=wl.y), 1e-12), (rowpass.Cost(s, 1.0, gram=gram), 1e-9)]:
        lz = cost.log_normalisers([st.nu], [st.lam])
        E = cost.row_costs([st.nu], [st.lam], lz)[0]
        np.testing.assert_allclose(E, rows_ref, rtol=rtol, atol=1e-15)
        assert float(wl.r @ E) == pytest.approx(ref, rel=rtol)


def test_cmax_c_routine_matches_numpy():
    from oracle import cmax
    wl = W.random_small(300, 211, 5, seed=16)
    assert cmax.max_sqdist(wl.x, wl.y) == L.max_sqdist(wl.x.astype(np.float64), wl.y.astype(np.float64))


def test_tolerance_is_tested_from_the_first_iterate():
    """Appendix E stopping rule, reading for t = 0: with uniform c the product coupling X^0 is
    exactly feasible, so a test at t = 0 would end every such run before it starts; the run
    instead stops at the first t >= 1 whose residual meets the tolerance."""
    wl = W.random_small(40, 32, 2, seed=3, uniform=True, eta=1e-2)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    C = L.sqeuclid_cost(x, y, 1.0 / L.max_sqdist(x, y))
    st0 = L.lamp_init(wl.m)
    assert L.residuals(L.plan(C, wl.r, st0, 1.0), wl.r, wl.c)[2] <= 1e-15
    st, _ = L.lamp_dense(C, wl.r, wl.c, L.Params(eta=wl.eta), 400, 1.0, tol=1e-3, trace=False)
    assert st.t >= 1
    assert L.residuals(L.plan(C, wl.r, st, 1.0), wl.r, wl.c)[2] <= 1e-3
    prev = L.lamp_dense(C, wl.r, wl.c, L.Params(eta=wl.eta), st.t - 1, 1.0, trace=False)[0]
    assert st.t == 1 or L.residuals(L.plan(C, wl.r, prev, 1.0), wl.r, wl.c)[2] > 1e-3


def test_l1_and_linf_costs_by_definition_and_1d_wasserstein():
    """The l1 / l_inf ground costs: written-out definitions on a tiny case, their relation on
    the line (both equal |x - y| in d = 1), and the LP optimum with the l1 cost in d = 1 with
    uniform marginals against the sorted-matching closed form (1/n) sum |x_(i) - y_(i)|."""
    rng = np.random.default_rng(13)
    x = rng.random((4, 3))
    y = rng.random((5, 3))
    C1 = L.l1_cost(x, y, 2.0)
    Ci = L.linf_cost(x, y, 2.0)
    for i in range(4):
        for j in range(5):
            diffs = [abs(x[i, k] - y[j, k]) for k in range(3)]
            assert C1[i, j] == pytest.approx(2.0 * sum(diffs), rel=1e-15)
            assert Ci[i, j] == pytest.approx(2.0 * max(diffs), rel=1e-15)
    assert L.max_cost(x, y, "l1") == pytest.approx(float(np.max(C1)) / 2.0)
    x1 = rng.random((7, 1))
    y1 = rng.random((7, 1))
    assert np.allclose(L.l1_cost(x1, y1, 1.0), L.linf_cost(x1, y1, 1.0))
    u = np.full(7, 1.0 / 7)
    opt, _ = exact.lp_ot(L.l1_cost(x1, y1, 1.0), u, u)
    assert opt == pytest.approx(np.mean(np.abs(np.sort(x1[:, 0]) - np.sort(y1[:, 0]))), abs=1e-12)


@pytest.mark.parametrize("kind", ["l1", "linf"])
def test_metric_envelope_gradient_by_finite_differences(kind):
    """The l1 / l_inf envelope gradient against central differences of the row term at
    generic points (no kinks within h)."""
    wl = W.random_small(6, 9, 3, seed=17, eta=1e-1)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_cost(x, y, kind)
    rng = np.random.default_rng(2)
    nu = 0.3 * rng.standard_normal(wl.m)
    lam = 7.0
    g = L.envelope_grad_x_metric(x, y, wl.r, s, nu, lam, 1.0, kind)
    h = 1e-6
    for i in range(wl.n):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (L.envelope_value_rows(xp, y, wl.r, s, nu, lam, 1.0, kind)[i]
                  - L.envelope_value_rows(xm, y, wl.r, s, nu, lam, 1.0, kind)[i]) / (2 * h)
            assert g[i, k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1", "linf"])
def test_envelope_gradient_wrt_targets_by_finite_differences(kind):
    """The gradient with respect to the target points against central differences of the
    whole dual value sum_i f_i (every row term depends on each y_j)."""
    wl = W.random_small(5, 6, 2, seed=23, eta=1e-1)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_cost(x, y, kind)
    rng = np.random.default_rng(4)
    nu = 0.3 * rng.standard_normal(wl.m)
    lam = 5.0
    g = L.envelope_grad_y(x, y, wl.r, s, nu, lam, 1.0, kind)
    h = 1e-6
    for j in range(wl.m):
        for k in range(2):
            yp, ym = y.copy(), y.copy()
            yp[j, k] += h
            ym[j, k] -= h
            fd = (np.sum(L.envelope_value_rows(x, yp, wl.r, s, nu, lam, 1.0, kind))
                  - np.sum(L.envelope_value_rows(x, ym, wl.r, s, nu, lam, 1.0, kind))) / (2 * h)
            assert g[j, k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1", "linf"])
def test_envelope_gradient_columns_by_finite_differences(kind):
    """The column-at-a-time y-gradient (given the row log-normalisers) against central differences
    of the whole dual value, on listed columns, for each ground cost."""
    wl = W.random_small(7, 9, 3, seed=29, eta=1e-1)
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / L.max_cost(x, y, kind)
    rng = np.random.default_rng(6)
    nu = 0.3 * rng.standard_normal(wl.m)
    lam = 4.0
    C = L.ground_cost(x, y, s, kind)
    cols = [0, 4, 8]
    g = L.envelope_grad_y_columns(x, y, wl.r, s, nu, lam, 1.0, cols, L.log_normaliser(C, nu, lam, 1.0), kind)
    h = 1e-6
    for a, j in enumerate(cols):
        for k in range(3):
            yp, ym = y.copy(), y.copy()
            yp[j, k] += h
            ym[j, k] -= h
            fd = (np.sum(L.envelope_value_rows(x, yp, wl.r, s, nu, lam, 1.0, kind))
                  - np.sum(L.envelope_value_rows(x, ym, wl.r, s, nu, lam, 1.0, kind))) / (2 * h)
            assert g[a, k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


# ---------------------------------------------------------------- D_t (Proposition infeas_bound(b))


def test_dt_symmetric_two_by_two_closed_form():
    """C = [[0,1],[1,0]], r = c = (1/2, 1/2), eta = 0: theta = nu = nubar = 0 for all t, so
    thetabar = thetahat = theta = 0 (no dual terms), Xbar^{s+1} = X^{s+1}, and each summand of
    D_t is -KL(X^{s+1} || X^s).  Both rows of X^t are (a_t, 1 - a_t)/2 with
    a_t = 1/(1 + e^{-t/2}), so D_t = -sum_{s<t} [a_{s+1} ln(a_{s+1}/a_s)
    + (1 - a_{s+1}) ln((1 - a_{s+1})/(1 - a_s))]."""
    C = np.array([[0.0, 1.0], [1.0, 0.0]])
    r = c = np.array([0.5, 0.5])
    T = 40
    D, _, _ = L.dt_sequence(C, r, c, L.Params(eta=0.0), T)
    a = [1.0 / (1.0 + math.exp(-t / 2.0)) for t in range(T + 1)]
    ref, acc = [], 0.0
    for s in range(T):
        p, q = a[s + 1], a[s]
        acc -= p * math.log(p / q) + (1.0 - p) * math.log((1.0 - p) / (1.0 - q))
        ref.append(acc)
    np.testing.assert_allclose(D, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("eta", [0.0, 1e-2])
def test_dt_kl_difference_matches_lemma_kl_diff(eta):
    """Lemma kl_diff: with row(Xbar) = r the KL difference of each summand has the closed form
        KL(Xbar^{s+1}||X^{s+1}) - KL(Xbar^{s+1}||X^s) = (lam_{s+1} - lam_s) <C, Xbar^{s+1}>
            + K <col(Xbar^{s+1}), lam_{s+1} nu^{s+1} - lam_s nu^s> + <r, log Z^{s+1} - log Z^s>
    (any eta; K = 2||C||_inf).  For eta = 0 and ||C||_inf = 1 (lam_t = t/2) it is the negative of
    the printed identity  -<col(Xbar), thetabar^{s+1}> - <C, Xbar>/2 - <r, log Z^{s+1}> + <r, log Z^s>.
    Both are checked against the dense KL of the oracle."""
    C, r, c, *_ = _problem(7, 5, 2, seed=23)
    C = C / C.max()
    prm = L.Params(eta=eta).resolved(1.0)
    st = L.lamp_init(5)
    for s in range(25):
        tr = L.LampTrace()
        nxt = L.lamp_step(C, r, c, st, prm, 1.0, tr)
        Xbar = r[:, None] * L.dual_to_primal(C, tr.nubar[0], nxt.lam, 1.0)
        X_s, X_n = L.plan(C, r, st, 1.0), L.plan(C, r, nxt, 1.0)
        dense = L.kl(Xbar, X_n) - L.kl(Xbar, X_s)
        lz_s = L.log_normaliser(C, st.nu, st.lam, 1.0)
        lz_n = L.log_normaliser(C, nxt.nu, nxt.lam, 1.0)
        general = ((nxt.lam - st.lam) * float(np.sum(C * Xbar))
                   + 2.0 * float(L.col(Xbar) @ (nxt.lam * nxt.nu - st.lam * st.nu))
                   + float(r @ (lz_n - lz_s)))
        assert dense == pytest.approx(general, rel=1e-10, abs=1e-13)
        if eta == 0.0:
            printed = (-float(L.col(Xbar) @ tr.theta_bar[0]) - 0.5 * float(np.sum(C * Xbar))
                       - float(r @ lz_n) + float(r @ lz_s))
            assert dense == pytest.approx(-printed, rel=1e-10, abs=1e-13)
        st = nxt


def test_dual_bregman_divergence_by_definition():
    """D_H(theta||nu) = H(theta) - H(nu) - <grad H(nu), theta - nu> for the negative dual entropy
    H_c^alpha of Section 3.1 equals both explicit forms (def:DHa_explicit, def:DHa); the gradient
    (def:Ha_grad) matches central differences of H."""
    rng = np.random.default_rng(5)
    m = 9
    calpha = rng.dirichlet(np.ones(m)) + 0.01 / m
    for _ in range(5):
        th = rng.uniform(-0.95, 0.95, m)
        nu = rng.uniform(-0.95, 0.95, m)
        g = L.dual_entropy_grad(nu, calpha)
        by_def = L.dual_entropy(th, calpha) - L.dual_entropy(nu, calpha) - float(g @ (th - nu))
        second = float(calpha / 2.0 @ np.log((1.0 - th ** 2) / (1.0 - nu ** 2))
                       + th @ (L.dual_entropy_grad(th, calpha) - g))
        assert L.bregman_Ha(th, nu, calpha) == pytest.approx(by_def, rel=1e-11, abs=1e-14)
        assert second == pytest.approx(by_def, rel=1e-11, abs=1e-14)
        h = 1e-6
        fd = np.array([(L.dual_entropy(nu + h * e, calpha) - L.dual_entropy(nu - h * e, calpha)) / (2 * h)
                       for e in np.eye(m)])
        np.testing.assert_allclose(fd, g, rtol=1e-7, atol=1e-9)


def test_dt_midpoint_bound_holds_at_the_lp_saddle_point():
    """Proposition infeas_bound(b) with the exact saddle point of problem spp (eta = 0): X* from
    the LP and theta* = (k - y_c)/(2||C||_inf) from its column duals, centred into [-1/2, 1/2]
    (then D(theta*) = OPT, the dual function of def:dual_spp).  For every t:
        min_{1<=s<=t} K(Xbar^s, theta*) - K(X*, thetabar^s) <= 2||C||_inf (log m + (1+a) log 2 + D_t)/t."""
    for seed, (n, m) in [(31, (6, 5)), (32, (5, 7))]:
        C, r, c, *_ = _problem(n, m, 2, seed=seed)
        cnorm = float(C.max())
        opt, X_star = exact.lp_ot(C, r, c)
        _, _, yc = exact.lp_ot_duals(C, r, c)
        k = 0.5 * (yc.max() + yc.min())
        theta_star = (k - yc) / (2.0 * cnorm)
        assert np.all(np.abs(theta_star) <= 0.5 + 1e-12)
        assert L.dual_D(C, r, c, theta_star, cnorm) == pytest.approx(opt, rel=1e-8, abs=1e-12)
        prm = L.Params(eta=0.0)
        T = 60
        D, _, traces = L.dt_sequence(C, r, c, prm, T, cnorm)
        best = math.inf
        lam = L.inv_eta_schedule(T, 1.0 / (2.0 * cnorm), 0.0)
        for s in range(1, T + 1):
            tr = traces[s - 1]   # the step s-1 -> s produced nubar^s and thetabar^s
            Xbar = r[:, None] * L.dual_to_primal(C, tr.nubar[0], lam[s], cnorm)
            gap = (L.saddle_K(C, Xbar, theta_star, c, cnorm)
                   - L.saddle_K(C, X_star, tr.theta_bar[0], c, cnorm))
            best = min(best, gap)
            assert best <= L.midpoint_bound(D[s - 1], s, m, prm.alpha, cnorm) + 1e-12


@pytest.mark.parametrize("eta", [0.0, 1e-2])
def test_dt_summands_match_the_dual_and_primal_identities(eta):
    """Every increment D_{s+1} - D_s of the oracle's D_t equals a closed form built from other
    quantities: Lemma Dha_diff at theta* = thetahat^{s+1} gives the dual part,
        D_H(thetabar||thetahat) - D_H(thetabar||theta^s) = -D_H(thetahat||theta^s)
                                                           - <thetabar - thetahat, col(Xbar) - c>,
    and the general-eta form of Lemma kl_diff the primal part (see the test above)."""
    C, r, c, *_ = _problem(6, 7, 2, seed=41)
    cnorm = float(C.max())
    prm = L.Params(eta=eta)
    T = 30
    D, _, traces = L.dt_sequence(C, r, c, prm, T, cnorm)
    res = prm.resolved(cnorm)
    calpha = c + res.alpha / 7
    st = L.lamp_init(7)
    prev = 0.0
    for s in range(T):
        tr = traces[s]
        nxt = L.lamp_step(C, r, c, st, res, cnorm)
        tbar, that, colB = tr.theta_bar[0], tr.theta_hat[0], tr.colB[0]
        dual = -L.bregman_Ha(that, st.theta, calpha) - float((tbar - that) @ (colB - c))
        Xbar = r[:, None] * L.dual_to_primal(C, tr.nubar[0], nxt.lam, cnorm)
        primal = ((nxt.lam - st.lam) * float(np.sum(C * Xbar))
                  + 2.0 * cnorm * float(colB @ (nxt.lam * nxt.nu - st.lam * st.nu))
                  + float(r @ (L.log_normaliser(C, nxt.nu, nxt.lam, cnorm)
                               - L.log_normaliser(C, st.nu, st.lam, cnorm))))
        assert D[s] - prev == pytest.approx(dual + primal, rel=1e-9, abs=1e-12)
        prev = D[s]
        st = nxt


def test_dual_bregman_from_natural_parameters_high_precision():
    """bregman_Ha_natural(a, b) = D_H(tanh a || tanh b): against def:DHa_explicit evaluated with
    60-digit decimal arithmetic (exact tanh, no rounding of 1 - theta), for moderate and for
    saturated arguments (|a| up to 60, where tanh a is +-1 in FP64), and against the FP64
    explicit form where that one is accurate."""
    import decimal
    ctx = decimal.Context(prec=60)
    Dm = decimal.Decimal

    def dha_exact(a, b, w):
        tot = Dm(0)
        for ai, bi, wi in zip(a, b, w):
            ea, eb = ctx.exp(Dm(2 * ai)), ctx.exp(Dm(2 * bi))
            pa, qa = ea / (ea + 1), 1 / (ea + 1)          # (1 + tanh a)/2, (1 - tanh a)/2
            pb, qb = eb / (eb + 1), 1 / (eb + 1)
            tot += Dm(wi) * (pa * ctx.ln(pa / pb) + qa * ctx.ln(qa / qb))
        return float(tot)

    rng = np.random.default_rng(9)
    m = 7
    w = rng.dirichlet(np.ones(m)) + 0.01 / m
    for scale in [0.5, 3.0, 60.0]:
        a = rng.uniform(-scale, scale, m)
        b = rng.uniform(-0.55, 0.55, m)          # a clipped theta^s: |tanh b| <= 0.5
        got = L.bregman_Ha_natural(a, b, w)
        assert got == pytest.approx(dha_exact(a, b, w), rel=1e-12, abs=1e-14)
        if scale <= 3.0:
            assert got == pytest.approx(L.bregman_Ha(np.tanh(a), np.tanh(b), w), rel=1e-10, abs=1e-13)


# ---------------------------------------------------------------- value functions and bounds


def _row_identical_example(alpha=0.01):
    """Two identical rows, C = [[0, 2], [0, 2]] (||C||_inf = 2), r = c = (1/2, 1/2), eta = 0.
    Worked by hand: col(X^0) = c, so thetabar^1 = nu^1 = nubar^1 = 0 and lam_1 = tau1 = 1/4;
    every row of X^1 (and of Xbar^1) is p/2 with p = softmax(-(0, 2)/4) = ((1 + t)/2, (1 - t)/2),
    t = tanh(1/4), so ||col(X^1) - c||_1 = tanh(1/4), OPT = 1 (half the mass must pay 2),
    and the step's natural parameter is thetahat^1 = tanh(a), a = +-(p_1 - 1/2)/c^alpha_j =
    +-tanh(1/4)/(1 + alpha)."""
    C = np.array([[0.0, 2.0], [0.0, 2.0]])
    r = c = np.array([0.5, 0.5])
    return C, r, c, L.Params(eta=0.0, alpha=alpha)


def test_prop_bound_exact_value_on_one_step_example():
    """Proposition infeas_bound(a) at t = 1 of the two-identical-rows example:
    4 ||C||_inf tanh(1/4) + 2 ||C||_inf log 2 = 8 tanh(1/4) + 4 log 2 (m = 2; n m = 4 would give
    4 log 4), and it bounds the rounded cost's error; on the symmetric 2 x 2 example
    (col(X^t) = c) the certificate's bound is exactly 2 log 2 / t."""
    C, r, c, prm = _row_identical_example()
    st = L.lamp_step(C, r, c, L.lamp_init(2), prm.resolved(2.0), 2.0)
    cert = L.certificate(C, r, c, st, prm.resolved(2.0), 2.0)
    t1 = math.tanh(0.25)
    assert cert["col_res"] == pytest.approx(t1, rel=1e-14)
    assert cert["prop_bound"] == pytest.approx(8.0 * t1 + 4.0 * math.log(2.0), rel=1e-14)
    assert cert["rounded_cost"] - 1.0 <= cert["prop_bound"]

    C2 = np.array([[0.0, 1.0], [1.0, 0.0]])
    st = L.lamp_init(2)
    p2 = L.Params(eta=0.0).resolved(1.0)
    for t in range(1, 30):
        st = L.lamp_step(C2, r, c, st, p2, 1.0)
        cert = L.certificate(C2, r, c, st, p2, 1.0)
        assert cert["prop_bound"] == pytest.approx(2.0 * math.log(2.0) / t, rel=1e-14)


@pytest.mark.parametrize("alpha", [0.01, 0.5])
def test_midpoint_bound_exact_value_on_one_step_example(alpha):
    """Proposition infeas_bound(b) at t = 1 of the two-identical-rows example.  thetabar^1 = theta^0
    = 0 and Xbar^1 = X^1, so D_1 = D_H(0 || thetahat^1) - KL(X^1 || X^0) with
    D_H(0 || tanh a) = sum_j c^alpha_j ln cosh a_j (def:DHa_explicit) = (1 + alpha) ln cosh(a) and
    KL(X^1 || X^0) = ln 2 - h(p_1) (h the binary entropy in nats); the bound is
    2 ||C||_inf (ln 2 + (1 + alpha) ln 2 + D_1) = 4 (ln 2 + (1 + alpha) ln 2 + D_1)."""
    C, r, c, prm = _row_identical_example(alpha)
    D, _, _ = L.dt_sequence(C, r, c, prm, 1, 2.0)
    t1 = math.tanh(0.25)
    a = t1 / (1.0 + alpha)
    p1 = 0.5 * (1.0 + t1)
    h = -p1 * math.log(p1) - (1.0 - p1) * math.log(1.0 - p1)
    d1 = (1.0 + alpha) * math.log(math.cosh(a)) - (math.log(2.0) - h)
    assert D[0] == pytest.approx(d1, rel=1e-12, abs=1e-15)
    ref = 4.0 * (math.log(2.0) + (1.0 + alpha) * math.log(2.0) + d1)
    assert L.midpoint_bound(D[0], 1, 2, alpha, 2.0) == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("eta", [1e-3, 3e-2, 0.3])
def test_dual_eta_sandwich_and_zero_temperature_limit(eta):
    """softmin^eta lies in [min - eta log m, min] for every row (Appendix B), and r sums to one,
    so D(theta) - eta log m <= D^eta(theta) <= D(theta) (def:dual_spp_e against def:dual_spp);
    with a unique minimiser in every row D^eta -> D faster than eta log m."""
    C, r, c, *_ = _problem(7, 9, 2, seed=41)
    cnorm = float(C.max())
    g = np.random.default_rng(42)
    for _ in range(5):
        th = g.uniform(-1.0, 1.0, 9)
        d0 = L.dual_D(C, r, c, th, cnorm)
        de = L.dual_D_eta(C, r, c, th, cnorm, eta)
        assert d0 - eta * math.log(9) - 1e-13 <= de <= d0 + 1e-13
    th = g.uniform(-1.0, 1.0, 9)
    assert abs(L.dual_D_eta(C, r, c, th, cnorm, 1e-5) - L.dual_D(C, r, c, th, cnorm)) < 1e-6


def test_dual_eta_is_the_minimum_over_row_stochastic_plans():
    """D^eta(theta) is K^eta minimised over row-stochastic p (problem spp, def:dual_spp_e), up to
    the constant eta H(r) that H(diag(r) p) carries.  With m = 2 each row of p is (q, 1 - q) and
    K^eta separates over rows, so the minimum is found here by a 1-D search per row over the
    logit of q, not from the LogSumExp formula."""
    C, r, c, *_ = _problem(3, 2, 2, seed=43)
    cnorm = float(C.max())
    K = 2.0 * cnorm
    for eta, th in [(0.1, np.array([0.3, -0.6])), (0.02, np.array([-0.2, 0.45]))]:
        total = -K * float(c @ th)
        for i in range(3):
            def row_obj(u, i=i):      # u = log(q / (1 - q))
                lq, l1q = -np.logaddexp(0.0, -u), -np.logaddexp(0.0, u)
                x = r[i] * np.exp([lq, l1q])
                return float(x @ (C[i] + K * th) + eta * (x @ (np.log(r[i]) + np.array([lq, l1q]))))
            total += minimize_scalar(row_obj, bracket=(-5.0, 5.0), method="brent",
                                     options=dict(xtol=1e-14)).fun
        hr = L.entropy(r[:, None])
        assert L.dual_D_eta(C, r, c, th, cnorm, eta) == pytest.approx(total + eta * hr, abs=1e-12)


def test_dual_eta_strong_duality_at_the_sinkhorn_plan():
    """At the EOT solution X_eta = exp((f_i + g_j - C_ij)/eta) (Sinkhorn, problem primal_eot) the
    column potential gives theta* = -g/(2||C||_inf) with D^eta(theta*) = <C, X_eta> - eta H(X_eta)
    + eta H(r), and theta* maximises D^eta (it is concave): random perturbations only lower it."""
    C, r, c, *_ = _problem(5, 4, 2, seed=45)
    cnorm = float(C.max())
    eta = 0.05
    Xs = exact.sinkhorn_eot(C, r, c, eta)
    g = eta * np.log(Xs[0] / Xs[0, 0]) + C[0] - C[0, 0]      # g_j - g_0 from row 0
    th = -g / (2.0 * cnorm)
    th -= 0.5 * (th.max() + th.min())
    val = float(np.sum(C * Xs)) - eta * L.entropy(Xs) + eta * L.entropy(r[:, None])
    top = L.dual_D_eta(C, r, c, th, cnorm, eta)
    assert top == pytest.approx(val, rel=1e-10, abs=1e-12)
    rng = np.random.default_rng(46)
    for _ in range(20):
        assert L.dual_D_eta(C, r, c, th + rng.normal(scale=0.05, size=4), cnorm, eta) < top


def test_primal_penalised_values_and_weak_duality():
    """P^eta of problem l1_ot_primal: on the LP plan X* it is OPT (HiGHS); moving eps of mass onto
    one entry adds eps C_ij and eps to each of the row and column residuals, each priced at
    2||C||_inf; on the product plan r c^T (feasible) it is <C, r c^T> - eta (H(r) + H(c)); and
    D^eta(theta) <= P^eta(diag(r) p) + eta H(r) for every theta in [-1, 1]^m and row-stochastic p."""
    C, r, c, *_ = _problem(5, 6, 2, seed=47)
    cnorm = float(C.max())
    opt, Xstar = exact.lp_ot(C, r, c)
    Xstar = np.maximum(Xstar, 0.0)
    assert L.primal_penalised(C, Xstar, r, c, cnorm) == pytest.approx(opt, abs=1e-9)
    eps = 1e-3
    Xp = Xstar.copy()
    Xp[2, 4] += eps
    assert L.primal_penalised(C, Xp, r, c, cnorm) == pytest.approx(
        opt + eps * C[2, 4] + 4.0 * cnorm * eps, abs=1e-9)
    eta = 0.07
    prod = np.outer(r, c)
    hr, hc = L.entropy(r[:, None]), L.entropy(c[:, None])
    assert L.primal_penalised(C, prod, r, c, cnorm, eta) == pytest.approx(
        float(r @ C @ c) - eta * (hr + hc), rel=1e-13)
    g = np.random.default_rng(48)
    for _ in range(20):
        th = g.uniform(-1.0, 1.0, 6)
        X = r[:, None] * g.dirichlet(np.ones(6), size=5)
        for e in (0.0, eta):
            de = L.dual_D(C, r, c, th, cnorm) if e == 0.0 else L.dual_D_eta(C, r, c, th, cnorm, e)
            assert de <= L.primal_penalised(C, X, r, c, cnorm, e) + e * hr + 1e-12


def test_combined_gap_values():
    """Equation (combined) as printed (coefficient ||C||_inf): zero on the LP plan, and eps C_ij +
    ||C||_inf (eps + eps) after eps of mass is added to one entry."""
    C, r, c, *_ = _problem(5, 6, 2, seed=49)
    cnorm = float(C.max())
    opt, Xstar = exact.lp_ot(C, r, c)
    Xstar = np.maximum(Xstar, 0.0)
    assert L.combined_gap(C, Xstar, r, c, opt, cnorm) == pytest.approx(0.0, abs=1e-9)
    eps = 2e-3
    Xp = Xstar.copy()
    Xp[1, 3] += eps
    assert L.combined_gap(C, Xp, r, c, opt, cnorm) == pytest.approx(
        eps * C[1, 3] + 2.0 * cnorm * eps, abs=1e-9)
