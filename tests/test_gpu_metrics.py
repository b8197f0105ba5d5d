"""GPU parity of the l1 and l_inf ground costs (the kernelized experiments of Section 5)
against the FP64 oracle, through the C ABI: first iterations, the certificate with
<C, Round(X)>, the cost normalisation, the envelope gradient, and the argument checks of the
forms that need the squared Euclidean cost.  Tolerances as for the squared Euclidean cost."""
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import fp32_trajectory_allowance, rel_dual, rel_inf, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

DUAL_TOL = 1e-6
COL_TOL = 1e-6
LOGZ_ATOL = 2e-6
COST_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(n, m, d, kind, seed, eta=1e-2):
    wl = W.random_small(n, m, d, seed=seed, eta=eta)
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    s = 1.0 / OL.max_cost(x, y, kind)
    C = OL.ground_cost(x, y, s, kind)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0, metric=kind)
    return wl, x, y, s, C, prob


SHAPES = [(200, 150, 2, "l1"), (130, 171, 3, "linf"), (97, 80, 5, "l1"), (64, 50, 1, "linf"),
          (120, 90, 4, "linf"), (33, 40, 7, "linf")]


@pytest.mark.parametrize("shape", SHAPES)
def test_metric_first_steps_match_oracle(shape):
    """Iterations 0..4 from the fresh state: marginals, log-normalisers, duals."""
    n, m, d, kind = shape
    wl, x, y, s, C, prob = _problem(n, m, d, kind, seed=400 + d)
    _say("case", kind, wl.name)
    _, tr_or = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=wl.eta), 5, 1.0)
    params = P.make_params(eta=wl.eta)
    st = P.State.fresh(m)
    for k in range(5):
        res, tr = P.step(prob, params, st, trace=True)
        assert res == pytest.approx(tr_or.res[k], rel=1e-6, abs=COL_TOL)
        assert rel_l1(to_np(tr["col_a"]), tr_or.colA[k]) <= COL_TOL
        assert rel_l1(to_np(tr["col_b"]), tr_or.colB[k]) <= COL_TOL
        assert np.max(np.abs(to_np(tr["log_za"]) - tr_or.logZA[k])) <= LOGZ_ATOL
        assert np.max(np.abs(to_np(tr["log_zb"]) - tr_or.logZB[k])) <= LOGZ_ATOL
        assert rel_dual(to_np(st.nu), tr_or.nu[k]) <= DUAL_TOL
        assert rel_dual(to_np(st.theta), tr_or.theta[k]) <= DUAL_TOL


def rel_l1(a, ref):
    return np.abs(np.asarray(a) - ref).sum() / np.abs(ref).sum()


@pytest.mark.parametrize("kind", ["l1", "linf"])
def test_metric_cost_scale(kind):
    """s = 1 / max_ij dist(x_i, y_j) on the device against the oracle's maximum."""
    wl, x, y, s, C, prob = _problem(300, 211, 3, kind, seed=31)
    gpu = P.Problem(wl.x, wl.y, wl.r, wl.c, metric=kind)
    s_gpu, dmax = P.cost_scale(gpu)
    assert s_gpu == pytest.approx(s, rel=1e-14)


@pytest.mark.parametrize("kind", ["l1", "linf"])
def test_metric_trajectory_certificate_and_round(kind):
    """60 iterations with the graph loop, then the certificate: duals, <C, X>, D(theta), D(nu)
    and <C, Round(X)> against the oracle's dense evaluation."""
    wl, x, y, s, C, prob = _problem(180, 150, 3, kind, seed=37)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, 60, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=60, check_every=20)
    st, _, status = P.solve(prob, params)
    assert status == 0 and st.t == 60
    cert = P.certificate(prob, params, st)
    _say(kind, {k: (cert[k], cert_or[k]) for k in ["cost", "rounded_cost", "dual_theta", "col_res"]})
    # 60 iterations accumulate FP32-level marginal errors in the duals (tests/gpu_util.py)
    traj = max(DUAL_TOL, 2.0 * fp32_trajectory_allowance(C, wl.r, wl.c, prm, 60))
    _say("trajectory allowance", traj)
    assert rel_dual(to_np(st.nu), st_or.nu) <= traj
    assert rel_dual(to_np(st.theta), st_or.theta) <= traj
    assert abs(cert["cost"] - cert_or["cost"]) <= COST_TOL * abs(cert_or["cost"])
    assert abs(cert["col_res"] - cert_or["col_res"]) <= COL_TOL
    assert abs(cert["rounded_cost"] - cert_or["rounded_cost"]) <= 2e-5
    for key in ["dual_theta", "dual_nu"]:   # D is 2K-Lipschitz in the duals (K = 2)
        assert abs(cert[key] - cert_or[key]) <= 2 * 2.0 * traj * 0.5, key
    assert max(cert["dual_theta"], cert["dual_nu"]) <= cert["rounded_cost"] + 1e-12
    assert cert["rounded_cost"] <= cert["primal_penalized"] + 1e-12


@pytest.mark.parametrize("kind,d", [("l1", 2), ("linf", 3), ("l1", 6)])
def test_metric_backward_matches_oracle_gradient(kind, d):
    """Envelope (sub)gradient with respect to x at the state after 40 iterations."""
    wl, x, y, s, C, prob = _problem(90, 70, d, kind, seed=41 + d)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=40)
    st, _, _ = P.solve(prob, params)
    g = to_np(P.backward(prob, params, st, grad_out=1.0))
    g_or = OL.envelope_grad_x_metric(x, y, wl.r, s, to_np(st.nu), st.inv_eta, 1.0, kind)
    err = rel_inf(g, g_or)
    _say(kind, d, "gradient rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("kind", ["l1", "linf"])
def test_metric_rejected_by_inner_product_forms(kind):
    """The matrix-core forms and the batching form evaluate inner products: a problem with
    another ground cost is rejected with LAMP_EINVAL, nothing runs."""
    wl, x, y, s, C, prob = _problem(40, 30, 2, kind, seed=5)
    with pytest.raises(P.LampError) as ei:
        P.step(prob, P.make_params(eta=wl.eta, precision="bf16_mfma"), P.State.fresh(30))
    assert "squared Euclidean" in str(ei.value)
    with pytest.raises(P.LampError):
        P.solve_batched([prob], P.make_params(eta=wl.eta, max_iter=3))


@pytest.mark.parametrize("kind,d", [("sqeuclid", 3), ("sqeuclid", 20), ("l1", 2), ("linf", 3), ("l1", 6)])
def test_backward_y_matches_oracle_gradient(kind, d):
    """Envelope gradient with respect to the target points at the state after 40 iterations."""
    wl, x, y, s, C, prob = _problem(80, 95, d, kind, seed=61 + d)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=40)
    st, _, _ = P.solve(prob, params)
    g = to_np(P.backward_y(prob, params, st, grad_out=1.0))
    g_or = OL.envelope_grad_y(x, y, wl.r, s, to_np(st.nu), st.inv_eta, 1.0, kind)
    err = rel_inf(g, g_or)
    _say(kind, d, "y-gradient rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("kind,d,n,m", [("sqeuclid", 3, 3000, 2200), ("l1", 2, 1800, 2600)])
def test_backward_y_across_splits(kind, d, n, m):
    """The y-adjoint where both of its passes run many splits with ragged last splits (the row
    sums over 18-24 column splits, the column pass over row splits), against the oracle's
    gradient at the state after 40 iterations."""
    wl, x, y, s, C, prob = _problem(n, m, d, kind, seed=91 + d)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=40)
    st, _, _ = P.solve(prob, params)
    g = to_np(P.backward_y(prob, params, st, grad_out=1.0))
    g_or = OL.envelope_grad_y(x, y, wl.r, s, to_np(st.nu), st.inv_eta, 1.0, kind)
    err = rel_inf(g, g_or)
    _say(kind, d, n, m, "y-gradient rel err", err)
    assert err <= 1e-5


def test_autograd_gradients_wrt_both_clouds():
    """LampOT returns the x and y envelope gradients through the two adjoint entry points."""
    wl, x, y, s, C, prob = _problem(70, 60, 2, "sqeuclid", seed=71)
    xt = torch.tensor(wl.x, device="cuda", requires_grad=True)
    yt = torch.tensor(wl.y, device="cuda", requires_grad=True)
    cost = P.LampOT.apply(xt, yt, wl.r, wl.c, 1e-2, 0.0, 50, s)
    cost.backward()
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=1e-2), 50, 1.0, trace=False)
    gx = OL.envelope_grad_x(x, y, wl.r, s, st_or.nu, st_or.lam, 1.0)
    gy = OL.envelope_grad_y(x, y, wl.r, s, st_or.nu, st_or.lam, 1.0)
    assert rel_inf(to_np(xt.grad), gx) <= 1e-4
    assert rel_inf(to_np(yt.grad), gy) <= 1e-4
