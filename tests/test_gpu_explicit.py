"""GPU parity of the explicit-cost input (lamp_problem.cost with LAMP_EXPLICIT: the caller's
n x m FP32 matrix instead of point clouds) against the FP64 oracle run on the same matrix,
through the C ABI.  Inputs: non-metric uniform costs with Dirichlet marginals and image-pair
grid costs (the non-kernelized image-transport problems of Section 5 and Appendix E, drawn
synthetically).  The oracle functions take C itself, so the same oracle code checks both
input forms.  Tolerances as for the point-cloud costs (the sweeps evaluate the same FP64
arguments, FP32 exponentials and sums)."""
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import fp32_trajectory_allowance, rel_dual, rel_l1, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

DUAL_TOL = 1e-6
COL_TOL = 1e-6
LOGZ_ATOL = 2e-6
COST_TOL = 1e-5
DT_STEP_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(wl, given_scale=False):
    """Oracle matrix C = s cost (FP64 of the FP32 entries, s = 1 / max) and the GPU problem;
    the library computes s itself unless given_scale."""
    cost64 = wl.cost.astype(np.float64)
    s = 1.0 / float(np.max(cost64))
    C = s * cost64
    kw = dict(cost_scale=s, cost_norm=1.0) if given_scale else {}
    return C, P.Problem.from_cost(wl.cost, wl.r, wl.c, **kw)


CASES = [lambda: W.random_cost(200, 150, seed=501),
         lambda: W.random_cost(1, 9, seed=502),
         lambda: W.random_cost(33, 700, seed=503),
         lambda: W.random_cost(517, 1029, seed=504),
         lambda: W.image_pair(6, "sqeuclid", seed=505, eta=1e-2),
         lambda: W.image_pair(5, "l1", seed=506, eta=0.0),
         lambda: W.image_pair(7, "linf", seed=507, eta=1e-3),
         lambda: W.random_cost(13, 1, seed=508),
         lambda: W.random_cost(1, 1, seed=511)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_explicit_first_steps_match_oracle(case):
    """Iterations 0..4 from the fresh state: residual, both column marginals, log-normalisers,
    duals.  Shapes span several row-sweep blocks and column splits with ragged tails, a single
    row, a single column, a 1 x 1 problem, and the three grid costs."""
    wl = CASES[case]()
    C, prob = _problem(wl)
    _say("case", wl.name, "eta", wl.eta)
    _, tr_or = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=wl.eta), 5, 1.0)
    params = P.make_params(eta=wl.eta)
    st = P.State.fresh(prob.m)
    for k in range(5):
        res, tr = P.step(prob, params, st, trace=True)
        assert res == pytest.approx(tr_or.res[k], rel=1e-6, abs=COL_TOL)
        assert rel_l1(to_np(tr["col_a"]), tr_or.colA[k]) <= COL_TOL
        assert rel_l1(to_np(tr["col_b"]), tr_or.colB[k]) <= COL_TOL
        assert np.max(np.abs(to_np(tr["log_za"]) - tr_or.logZA[k])) <= LOGZ_ATOL
        assert np.max(np.abs(to_np(tr["log_zb"]) - tr_or.logZB[k])) <= LOGZ_ATOL
        assert rel_dual(to_np(st.nu), tr_or.nu[k]) <= DUAL_TOL
        assert rel_dual(to_np(st.theta), tr_or.theta[k]) <= DUAL_TOL


def test_explicit_cost_scale():
    """s = 1 / max_ij cost_ij on the device, exact (a maximum of FP32 values)."""
    wl = W.random_cost(300, 211, seed=31)
    s_gpu, cmax = P.cost_scale(P.Problem.from_cost(wl.cost, wl.r, wl.c))
    assert cmax == float(np.max(wl.cost.astype(np.float64)))
    assert s_gpu == 1.0 / cmax


@pytest.mark.parametrize("make", [lambda: W.random_cost(180, 150, seed=37),
                                  lambda: W.image_pair(8, "sqeuclid", seed=38, eta=1e-2)])
def test_explicit_trajectory_certificate_round_and_dt(make):
    """60 tracked iterations with the graph loop, then the certificate: duals, <C, X>,
    <C, Round(X)>, D(theta), D(nu) and D_T against the oracle's dense evaluation."""
    wl = make()
    C, prob = _problem(wl, given_scale=True)
    T = 60
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, T, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    D, _, _ = OL.dt_sequence(C, wl.r, wl.c, prm, T, 1.0)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=T, check_every=20, track_dt=True)
    st, _, status = P.solve(prob, params)
    assert status == 0 and st.t == T
    cert = P.certificate(prob, params, st)
    _say(wl.name, {k: (cert[k], cert_or[k]) for k in ["cost", "rounded_cost", "dual_theta", "col_res"]},
         "D_T", cert["dt"], D[-1])
    traj = max(DUAL_TOL, 2.0 * fp32_trajectory_allowance(C, wl.r, wl.c, prm, T))
    assert rel_dual(to_np(st.nu), st_or.nu) <= traj
    assert rel_dual(to_np(st.theta), st_or.theta) <= traj
    assert abs(cert["cost"] - cert_or["cost"]) <= COST_TOL * abs(cert_or["cost"])
    assert abs(cert["col_res"] - cert_or["col_res"]) <= COL_TOL
    assert abs(cert["rounded_cost"] - cert_or["rounded_cost"]) <= 2e-5
    for key in ["dual_theta", "dual_nu"]:   # D is 2K-Lipschitz in the duals (K = 2)
        assert abs(cert[key] - cert_or[key]) <= 2 * 2.0 * traj * 0.5, key
    assert abs(cert["dt"] - D[-1]) <= T * (DT_STEP_TOL + 5e-7)
    assert max(cert["dual_theta"], cert["dual_nu"]) <= cert["rounded_cost"] + 1e-12


def test_explicit_matrix_of_a_point_cloud_and_the_point_form():
    """The squared Euclidean cost matrix of a point-cloud problem, rounded to FP32 and given
    explicitly, against the oracle on that rounded matrix; the point form of the same problem
    against the oracle on the unrounded cost; 30 iterations each."""
    wl = W.random_small(150, 120, 3, seed=77, eta=1e-2)
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    s = 1.0 / OL.max_sqdist(x, y)
    cost32 = OL.sqeuclid_cost(x, y, 1.0).astype(np.float32)
    prm = OL.Params(eta=wl.eta)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=30, check_every=10)
    runs = [(s * cost32.astype(np.float64), P.Problem.from_cost(cost32, wl.r, wl.c, cost_scale=s, cost_norm=1.0)),
            (OL.sqeuclid_cost(x, y, s), P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0))]
    for C, prob in runs:
        st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, 30, 1.0, trace=False)
        st, _, _ = P.solve(prob, params)
        traj = max(DUAL_TOL, 2.0 * fp32_trajectory_allowance(C, wl.r, wl.c, prm, 30))
        _say(prob.metric, rel_dual(to_np(st.nu), st_or.nu), traj)
        assert rel_dual(to_np(st.nu), st_or.nu) <= traj
        assert rel_dual(to_np(st.theta), st_or.theta) <= traj


def test_explicit_one_step_at_several_splits():
    """One step from a seeded dual state at n = 4096, m = 3000: six column splits of the row
    sweep (the last ragged) and 64 row splits of the column sweep; every column marginal and
    dual against the oracle."""
    wl = W.random_cost(4096, 3000, seed=509, eta=1e-3)
    C, prob = _problem(wl, given_scale=True)
    nu, th = W.synthetic_duals(3000, seed=510, amp=0.3)
    lam = 50.0
    prm = OL.Params(eta=wl.eta)
    state = OL.LampState(nu=nu.copy(), theta=th.copy(), t=7, lam=lam)
    st_or, tr_or = OL.lamp_dense(C, wl.r, wl.c, prm, 1, 1.0, state=state)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), 7, lam, 0.0)
    res, tr = P.step(prob, P.make_params(eta=wl.eta), st, trace=True)
    assert res == pytest.approx(tr_or.res[0], rel=1e-6, abs=COL_TOL)
    assert rel_l1(to_np(tr["col_a"]), tr_or.colA[0]) <= COL_TOL
    assert rel_l1(to_np(tr["col_b"]), tr_or.colB[0]) <= COL_TOL
    assert np.max(np.abs(to_np(tr["log_zb"]) - tr_or.logZB[0])) <= LOGZ_ATOL
    assert rel_dual(to_np(st.nu), st_or.nu) <= DUAL_TOL
    assert rel_dual(to_np(st.theta), st_or.theta) <= DUAL_TOL


def test_explicit_rejected_forms():
    """Matrix-core forms (inner products of points), the point adjoints and the batching form
    reject a cost-matrix problem with LAMP_EINVAL."""
    wl = W.random_cost(40, 30, seed=5)
    prob = P.Problem.from_cost(wl.cost, wl.r, wl.c)
    with pytest.raises(P.LampError):
        P.step(prob, P.make_params(eta=wl.eta, precision="bf16_mfma"), P.State.fresh(30))
    st, _, _ = P.solve(prob, P.make_params(eta=wl.eta, max_iter=3))
    for fn in (P.backward, P.backward_y):
        with pytest.raises(P.LampError) as ei:
            fn(prob, P.make_params(eta=wl.eta), st)
        assert "point clouds" in str(ei.value)
    with pytest.raises(P.LampError):
        P.solve_batched([prob], P.make_params(eta=wl.eta, max_iter=3))


def test_explicit_zero_cost_is_rejected():
    """A cost matrix with no positive entry has no normalisation s = 1 / max cost: the library
    computes the maximum and reports LAMP_EDOMAIN; nothing iterates."""
    wl = W.random_cost(20, 30, seed=12)
    prob = P.Problem.from_cost(np.zeros((20, 30), dtype=np.float32), wl.r, wl.c)
    with pytest.raises(P.LampError) as ei:
        P.solve(prob, P.make_params(eta=wl.eta, max_iter=3))
    assert ei.value.status == -2 and "zero" in str(ei.value)


def _rounded(wl, dtype):
    """The matrix stored in `dtype` and its exact FP64 values (what the library widens to)."""
    t = torch.tensor(wl.cost).to(getattr(torch, dtype))
    return t, t.double().numpy()


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
@pytest.mark.parametrize("case", [3, 4])
def test_explicit_half_storage_first_steps(dtype, case):
    """2-byte cost storage (lamp_problem.cost_type): each entry is widened exactly, so the oracle
    runs on the FP64 values of the rounded matrix with the tolerances of the FP32 storage;
    several splits with ragged tails (517 x 1029) and an image-pair grid cost."""
    wl = CASES[case]()
    t, cost64 = _rounded(wl, dtype)
    C = cost64 / float(np.max(cost64))
    prob = P.Problem.from_cost(t, wl.r, wl.c)
    assert prob.cost.dtype == getattr(torch, dtype)
    _say("case", wl.name, dtype)
    _, tr_or = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=wl.eta), 5, 1.0)
    params = P.make_params(eta=wl.eta)
    st = P.State.fresh(prob.m)
    for k in range(5):
        res, tr = P.step(prob, params, st, trace=True)
        assert res == pytest.approx(tr_or.res[k], rel=1e-6, abs=COL_TOL)
        assert rel_l1(to_np(tr["col_a"]), tr_or.colA[k]) <= COL_TOL
        assert rel_l1(to_np(tr["col_b"]), tr_or.colB[k]) <= COL_TOL
        assert np.max(np.abs(to_np(tr["log_zb"]) - tr_or.logZB[k])) <= LOGZ_ATOL
        assert rel_dual(to_np(st.nu), tr_or.nu[k]) <= DUAL_TOL
        assert rel_dual(to_np(st.theta), tr_or.theta[k]) <= DUAL_TOL


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_explicit_half_storage_trajectory_and_certificate(dtype):
    """60 tracked iterations and the certificate (cost, Round, dual values, D_T) over a 2-byte
    matrix against the oracle on its exact values."""
    wl = W.random_cost(180, 150, seed=37)
    t, cost64 = _rounded(wl, dtype)
    s = 1.0 / float(np.max(cost64))
    C = s * cost64
    prob = P.Problem.from_cost(t, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    T = 60
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, T, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    D, _, _ = OL.dt_sequence(C, wl.r, wl.c, prm, T, 1.0)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=T, check_every=20, track_dt=True)
    st, _, status = P.solve(prob, params)
    assert status == 0 and st.t == T
    cert = P.certificate(prob, params, st)
    traj = max(DUAL_TOL, 2.0 * fp32_trajectory_allowance(C, wl.r, wl.c, prm, T))
    _say(dtype, rel_dual(to_np(st.nu), st_or.nu), traj, cert["cost"], cert_or["cost"])
    assert rel_dual(to_np(st.nu), st_or.nu) <= traj
    assert rel_dual(to_np(st.theta), st_or.theta) <= traj
    assert abs(cert["cost"] - cert_or["cost"]) <= COST_TOL * abs(cert_or["cost"])
    assert abs(cert["rounded_cost"] - cert_or["rounded_cost"]) <= 2e-5
    assert abs(cert["dt"] - D[-1]) <= T * (DT_STEP_TOL + 5e-7)


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_explicit_runs_are_bitwise_identical(dtype):
    """Partials are merged in a fixed order: two solves of the same explicit problem give
    identical duals and certificates, bit for bit."""
    wl = W.random_cost(300, 260, seed=77)
    t = torch.tensor(wl.cost).to(getattr(torch, dtype))
    prob = P.Problem.from_cost(t, wl.r, wl.c)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=50, check_every=16)
    a, _, _ = P.solve(prob, params)
    b, _, _ = P.solve(prob, params)
    assert torch.equal(a.nu, b.nu) and torch.equal(a.theta, b.theta)
    ca, cb = P.certificate(prob, params, a), P.certificate(prob, params, b)
    assert all(ca[k] == cb[k] for k in ("cost", "rounded_cost", "dual_theta", "dual_nu", "col_res"))
