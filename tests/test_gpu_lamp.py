"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (derived in DESIGN.md, "Tolerances"): duals theta, nu, thetabar,
thetahat within 1e-6 norm-wise relative; column marginals within 1e-6 relative
in l1; row log-normalisers within 2e-6 absolute; transport cost within 1e-5
relative.
"""
import math
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from oracle import stream as OS
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import (U32, fp32_trajectory_allowance, gpu_problem, mfma_term_bound, oracle_problem,
                            split_fp16, split_fp16_scale,
                            rel_dual, rel_inf, rel_l1, round_to_type, to_np)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

DUAL_TOL = 1e-6          # relative to max(||ref||_inf, clip radius): see tests/gpu_util.py
COL_TOL = 1e-6
LOGZ_ATOL = 2e-6
COST_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare_step(tr_gpu, tr_or, k, st_gpu, st_or, tag):
    errs = dict(
        logZA=np.max(np.abs(to_np(tr_gpu["log_za"]) - tr_or.logZA[k])),
        logZB=np.max(np.abs(to_np(tr_gpu["log_zb"]) - tr_or.logZB[k])),
        colA=rel_l1(to_np(tr_gpu["col_a"]), tr_or.colA[k]),
        colB=rel_l1(to_np(tr_gpu["col_b"]), tr_or.colB[k]),
        theta_bar=rel_dual(to_np(tr_gpu["theta_bar"]), tr_or.theta_bar[k]),
        theta_hat=rel_dual(to_np(tr_gpu["theta_hat"]), tr_or.theta_hat[k]),
        nu=rel_dual(to_np(st_gpu.nu), st_or.nu),
        theta=rel_dual(to_np(st_gpu.theta), st_or.theta),
    )
    plain = dict(nu=rel_inf(to_np(st_gpu.nu), st_or.nu), theta=rel_inf(to_np(st_gpu.theta), st_or.theta))
    _say(tag, {k2: f"{v:.2e}" for k2, v in errs.items()},
         "plain relative (no floor):", {k2: f"{v:.2e}" for k2, v in plain.items()})
    assert errs["logZA"] <= LOGZ_ATOL and errs["logZB"] <= LOGZ_ATOL, errs
    assert errs["colA"] <= COL_TOL and errs["colB"] <= COL_TOL, errs
    for key in ["theta_bar", "theta_hat", "nu", "theta"]:
        assert errs[key] <= DUAL_TOL, (key, errs)


def _gpu_state(nu, theta, t, lam):
    dev = "cuda"
    return P.State(torch.tensor(nu, dtype=torch.float64, device=dev),
                   torch.tensor(theta, dtype=torch.float64, device=dev), t, lam)


@pytest.mark.parametrize("shape", [(256, 256, 2), (300, 173, 3), (97, 1031, 1), (517, 64, 5),
                                   (130, 260, 16), (70, 90, 20),
                                   (1, 1, 1), (1, 7, 2), (9, 1, 3), (33, 47, 128),
                                   (700, 1037, 24), (9000, 1300, 64), (9000, 700, 100)])
def test_first_steps_match_oracle(shape):
    """Iterations 0..4 from the fresh state, several tiles and ragged tails, each dimension path,
    the degenerate single-row / single-column problems and the largest supported d.  The last
    three run the FP64 matrix-core sweeps (operand widths 32, 64, 128) with n and m off the
    16-point tiles; at n = 9000 the split ranges hold two or three tiles, so that the paired
    iterations, the masked last iterations of a range and both LDS buffers all run."""
    n, m, d = shape
    wl = W.random_small(n, m, d, seed=100 + d, eta=1e-2)
    _say("case", wl.name)
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=wl.eta)
    st_or, tr_or = OL.lamp_dense(C, wl.r, wl.c, prm, 5, 1.0)
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=wl.eta)
    st = P.State.fresh(m)
    ost = OL.lamp_init(m)
    for k in range(5):
        res, tr = P.step(prob, params, st, trace=True)
        ost = OL.LampState(k + 1, 0.0, tr_or.nu[k], tr_or.theta[k])
        assert st.t == k + 1
        # res is an l1 distance of unit-mass vectors: FP32 column error 1e-6 of the mass
        assert res == pytest.approx(tr_or.res[k], rel=1e-6, abs=COL_TOL)
        _compare_step(tr, tr_or, k, st, ost, f"{wl.name} t={k}")


@pytest.mark.parametrize("t", [10, 100, 499])
def test_step_from_oracle_state(t):
    """256 x 256 uniform square, eta = 1e-2: one GPU step from the oracle's FP64 state at t."""
    wl = W.uniform_square()
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, t, 1.0, trace=False)
    st_next, tr_or = OL.lamp_dense(C, wl.r, wl.c, prm, 1, 1.0, state=st_or)
    prob = gpu_problem(wl, s)
    st = _gpu_state(st_or.nu, st_or.theta, st_or.t, st_or.lam)
    res, tr = P.step(prob, P.make_params(eta=wl.eta), st, trace=True)
    assert st.inv_eta == st_next.lam
    _compare_step(tr, tr_or, 0, st, st_next, f"uniform t={t}")


def test_trajectory_500_and_certificate():
    """The small parity workload: 500 iterations with the graph-captured loop, then the
    certificate.  Duals within 1e-6, cost within 1e-5 of the oracle."""
    wl = W.uniform_square()
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, 500, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=500, check_every=50)
    st, rep, status = P.solve(prob, params)
    assert status == 0 and st.t == 500 and rep["iters"] == 500
    e_nu = rel_dual(to_np(st.nu), st_or.nu)
    e_th = rel_dual(to_np(st.theta), st_or.theta)
    cert = P.certificate(prob, params, st)
    e_cost = abs(cert["cost"] - cert_or["cost"]) / abs(cert_or["cost"])
    _say("trajectory 500", f"nu {e_nu:.2e} theta {e_th:.2e} cost {e_cost:.2e}",
         f"plain relative (no floor): nu {rel_inf(to_np(st.nu), st_or.nu):.2e} "
         f"theta {rel_inf(to_np(st.theta), st_or.theta):.2e}",
         "col_res", cert["col_res"], cert_or["col_res"], "row_res", cert["row_res"])
    assert e_nu <= DUAL_TOL and e_th <= DUAL_TOL
    assert e_cost <= COST_TOL
    # col_res = ||col - c||_1 is a difference of unit-mass vectors: compared on that scale
    assert abs(cert["col_res"] - cert_or["col_res"]) <= 1e-6
    assert cert["row_res"] <= 1e-6
    # D is 2K-Lipschitz in the sup norm of its argument (each row minimum moves by at most
    # K ||d theta||_inf, the linear term by K ||c||_1 ||d theta||_inf): with duals equal to
    # 1e-6 x 0.5 the dual values agree to 2 K 5e-7 = 2e-6; P and the bound inherit the cost
    # and column-residual tolerances
    K = 2.0
    for key in ["dual_theta", "dual_nu"]:
        assert abs(cert[key] - cert_or[key]) <= 2 * K * DUAL_TOL * 0.5, key
    assert abs(cert["primal_penalized"] - cert_or["primal_penalized"]) <= (
        COST_TOL * abs(cert_or["cost"]) + K * 1e-6 + K * 1e-6)
    assert abs(cert["prop_bound"] - cert_or["prop_bound"]) <= 4 * 1e-6 + 1e-12
    assert cert["dual_theta"] <= cert["primal_penalized"]


def test_solve_stops_at_tolerance_and_resume():
    """Solve to a tolerance: the returned iterate meets it; resuming from a checkpoint reproduces
    the uninterrupted run; two runs are bitwise identical."""
    wl = W.random_small(400, 350, 3, seed=7, eta=1e-3)
    x, y, s, C = oracle_problem(wl)
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=wl.eta, tol=5e-3, max_iter=20000, check_every=32)
    st, rep, status = P.solve(prob, params)
    _say("solve", rep)
    assert status == 0 and rep["converged"] == 1
    # the oracle run to the same tolerance stops at the same iterate
    st_or, tr_or = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=wl.eta), 20000, 1.0, tol=5e-3)
    _say("oracle stops at", st_or.t, "gpu at", st.t)
    assert st.t == st_or.t
    assert rep["final_res"] <= 5e-3
    X = OL.plan(C, wl.r, st_or, 1.0)
    assert rep["final_res"] == pytest.approx(OL.residuals(X, wl.r, wl.c)[1], rel=1e-5)
    # st.t iterations accumulate FP32-level marginal errors in the duals: compare against
    # the oracle's own spread under half-ulp perturbations of its marginals (twice that)
    traj = max(DUAL_TOL, 2.0 * fp32_trajectory_allowance(C, wl.r, wl.c, OL.Params(eta=wl.eta), st_or.t))
    _say("trajectory allowance", traj)
    assert rel_dual(to_np(st.nu), st_or.nu) <= traj
    assert rel_dual(to_np(st.theta), st_or.theta) <= traj
    st2, rep2, _ = P.solve(prob, params)
    assert st2.t == st.t and torch.equal(st2.nu, st.nu) and torch.equal(st2.theta, st.theta)
    # checkpoint / resume: 60 + 60 iterations against 120
    p60 = P.make_params(eta=wl.eta, max_iter=60, check_every=16)
    a, _, _ = P.solve(prob, p60)
    a, _, _ = P.solve(prob, p60, a)
    b, _, _ = P.solve(prob, P.make_params(eta=wl.eta, max_iter=120, check_every=16))
    assert a.t == b.t == 120 and a.inv_eta == b.inv_eta
    # a resumed call starts from exact row offsets instead of the carried ones, which changes
    # the FP32 rounding of the exponent arguments: equal to the parity tolerance
    assert rel_dual(to_np(a.nu), to_np(b.nu)) <= DUAL_TOL
    assert rel_dual(to_np(a.theta), to_np(b.theta)) <= DUAL_TOL


@pytest.mark.parametrize("t", [3, 40])
def test_certificate_round_matches_oracle(t):
    """<C, Round(X^t)> (Algorithm 3 applied on the device without forming X) against the
    oracle's dense Round, on non-uniform marginals early in the run (large residuals, so
    every step of Round acts); and the ordering D <= <C, Round X> <= P(X)."""
    wl = W.random_small(300, 211, 3, seed=21, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, t, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=t)
    st, _, _ = P.solve(prob, params)
    cert = P.certificate(prob, params, st)
    _say("round", t, cert["rounded_cost"], cert_or["rounded_cost"], "cost", cert["cost"], "col_res",
         cert["col_res"])
    # a Lipschitz function of the plan (||C||_inf = 1): the plans agree to ~1e-6 in l1
    assert abs(cert["rounded_cost"] - cert_or["rounded_cost"]) <= 2e-5
    assert max(cert["dual_theta"], cert["dual_nu"]) <= cert["rounded_cost"] + 1e-12
    assert cert["rounded_cost"] <= cert["primal_penalized"] + 1e-12


def test_uniform_marginals_stop_after_first_iterate():
    """With uniform c the starting coupling is feasible; the tolerance is tested from t = 1 on,
    so the run stops where the oracle's does, after at least one iteration."""
    wl = W.random_small(300, 256, 2, seed=11, uniform=True, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    st, rep, status = P.solve(gpu_problem(wl, s), P.make_params(eta=wl.eta, tol=1e-3, max_iter=5000))
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=wl.eta), 5000, 1.0, tol=1e-3, trace=False)
    _say("uniform marginals: gpu stops at", st.t, "oracle at", st_or.t)
    assert status == 0 and st.t == st_or.t >= 1


def test_cost_scale_matches_oracle():
    for (n, m, d) in [(256, 256, 2), (1000, 777, 3), (123, 456, 16), (50, 60, 20)]:
        wl = W.random_small(n, m, d, seed=n)
        s, md = P.cost_scale(P.Problem(wl.x, wl.y, wl.r, wl.c))
        ref = OL.max_sqdist(wl.x.astype(np.float64), wl.y.astype(np.float64))
        assert md == pytest.approx(ref, rel=1e-13)


def test_backward_matches_oracle_gradient():
    """Envelope gradient at the GPU-independent oracle state (t = 60) against the oracle's."""
    wl = W.random_small(200, 150, 3, seed=11, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, 60, 1.0, trace=False)
    g_or = OL.envelope_grad_x(x, y, wl.r, s, st_or.nu, st_or.lam, 1.0)
    prob = gpu_problem(wl, s)
    st = _gpu_state(st_or.nu, st_or.theta, st_or.t, st_or.lam)
    g = to_np(P.backward(prob, P.make_params(eta=wl.eta), st, grad_out=1.0))
    err = rel_inf(g, g_or)
    _say("grad err", err)
    assert err <= 1e-5


def test_status_codes():
    wl = W.random_small(20, 30, 2, seed=3)
    bad_r = wl.r.copy()
    bad_r[0] = -bad_r[0]
    with pytest.raises(P.LampError) as e:
        P.step(P.Problem(wl.x, wl.y, bad_r, wl.c), P.make_params(), P.State.fresh(30))
    assert e.value.status == -2
    with pytest.raises(P.LampError) as e:
        P.step(P.Problem(wl.x, wl.y, wl.r * 1.01, wl.c), P.make_params(), P.State.fresh(30))
    assert e.value.status == -2 and "sums to" in str(e.value)
    bad_c = wl.c.copy()
    bad_c[7] = np.nan
    bad_c[19] = 0.0
    with pytest.raises(P.LampError) as e:   # the first entry that is not a positive finite mass
        P.step(P.Problem(wl.x, wl.y, wl.r, bad_c), P.make_params(), P.State.fresh(30))
    assert e.value.status == -2 and "c[7]" in str(e.value)
    with pytest.raises(P.LampError) as e:
        P.step(P.Problem(wl.x, wl.y, wl.r, wl.c), P.make_params(eta=5.0), P.State.fresh(30))
    assert e.value.status == -1
    # coincident clouds: every distance is zero, no normalisation s = 1 / max exists
    with pytest.raises(P.LampError) as e:
        P.step(P.Problem(np.zeros((20, 2), np.float32), np.zeros((30, 2), np.float32), wl.r, wl.c),
               P.make_params(), P.State.fresh(30))
    assert e.value.status == -2
    st = P.State.fresh(30)
    st.theta[3] = 1.0   # atanh(1) = inf
    st.t, st.inv_eta = 5, 2.5
    with pytest.raises(P.LampError) as e:
        P.step(P.Problem(wl.x, wl.y, wl.r, wl.c), P.make_params(), st)
    assert e.value.status == -5


def test_circulant_polygon_large():
    """Regular 16384-gon, x = y, uniform marginals, eta = 0: col(X^t) = c, theta = nu = 0 up to
    the FP32 rounding of the vertex coordinates, log Z_i the same for every row."""
    n = 16384
    wl = W.regular_polygon(n)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=0.25, cost_norm=1.0)
    params = P.make_params(eta=0.0, max_iter=40)
    st, rep, status = P.solve(prob, params)
    assert status == 0 and st.t == 40
    th = to_np(st.theta)
    assert np.max(np.abs(th)) <= 1e-4
    res, tr = P.step(prob, params, st, trace=True)
    lz = to_np(tr["log_za"])
    ref = OS.row_log_normalisers(wl.x.astype(np.float64), wl.y.astype(np.float64), 0.25, 1.0,
                                 np.zeros(n), 40 * 0.5, [0])[0]
    _say("polygon", np.max(np.abs(th)), lz.min(), lz.max(), ref, res)
    assert np.max(np.abs(lz - ref)) <= 1e-3
    assert res <= 1e-4


# ---------------------------------------------------------------- matrix-core forms

def _rounded_cost(wl, s, dtype, parts=False):
    """The cost the matrix-core forms evaluate: points centred on mu = (x_0 + y_0)/2 in FP64,
    rounded to the operand type, dot products exact, norms from the unrounded centred points.
    With `parts`, also (xr, yr, nx, ny)."""
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    # the library rounds each FP64 centred coordinate once, to nearest even, to the operand type
    name = str(dtype).replace("torch.", "")
    xr = round_to_type(xc, name)
    yr = round_to_type(yc, name)
    nx = np.sum(xc * xc, axis=1)
    ny = np.sum(yc * yc, axis=1)
    C = s * (nx[:, None] + ny[None, :] - 2.0 * xr @ yr.T)
    return (C, (xr, yr, nx, ny)) if parts else C


def _split_cost(wl, s):
    """The cost the split FP16 form evaluates: centred points times the range scale, split as
    hi + lo in FP16, the dot product x_hi.y_hi + x_hi.y_lo + x_lo.y_hi divided by the scale
    squared, norms from the unrounded centred points.  Also (effective x, effective y, nx, ny)."""
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    sc = split_fp16_scale(xc, yc)
    xh, xl = split_fp16(xc, sc)
    yh, yl = split_fp16(yc, sc)
    dot = (xh @ yh.T + xh @ yl.T + xl @ yh.T) / (sc * sc)
    nx = np.sum(xc * xc, axis=1)
    ny = np.sum(yc * yc, axis=1)
    C = s * (nx[:, None] + ny[None, :] - 2.0 * dot)
    return C, ((xh + xl) / sc, (yh + yl) / sc, nx, ny)


MFMA_KSTEP = {"fp32_mfma": 2, "bf16_mfma": 16, "fp16_mfma": 16, "fp16x3_mfma": 16}


def _mfma_tolerances(form, parts, s, lam, duals, n, m, d):
    """(log-normaliser, column) tolerances of a matrix-core step: the per-term bound of
    tests.gpu_util.mfma_term_bound plus FP32 partial sums of at most a whole column (row) range."""
    xr, yr, nx, ny = parts
    kp = 16 if d <= 16 else (64 if d <= 64 else 128)
    if form == "fp32_mfma" and d <= 4:
        kp = 4
    if form == "fp16x3_mfma":   # three parts of d entries per point
        kp = next(k for k in (16, 64, 128, 192) if 3 * d <= k)
    term = mfma_term_bound(xr, yr, ny, s, lam, duals, kp, MFMA_KSTEP[form])
    logz = term + (m / 32 + 6) * U32
    return logz, logz + term + (n / 32 + 6) * U32


MFMA_FORMS = [("fp32_mfma", torch.float32), ("bf16_mfma", torch.bfloat16),
              ("fp16_mfma", torch.float16)]


@pytest.mark.parametrize("form,dtype", MFMA_FORMS)
@pytest.mark.parametrize("shape", [(256, 256, 2), (300, 173, 3), (160, 200, 64), (97, 130, 16),
                                   (3, 5, 1), (40, 33, 128)])
def test_mfma_step_matches_oracle_on_rounded_cost(form, dtype, shape):
    """One step of each matrix-core form from an oracle state (t = 20, eta = 1e-2) against the
    oracle run on the cost those forms evaluate (operands rounded to the operand type).  The
    remaining differences are FP32 accumulation and exponent assembly: tolerance 1e-4."""
    _mfma_step_check(form, dtype, shape)


@pytest.mark.parametrize("shape", [(256, 256, 2), (300, 173, 3), (160, 200, 64), (97, 130, 16), (3, 5, 1),
                                   (200, 150, 40), (5, 4, 21)])
def test_split_fp16_step_matches_oracle_on_its_cost(shape):
    """One step of the split FP16 form (x.y as x_hi.y_hi + x_hi.y_lo + x_lo.y_hi from FP16
    parts of the range-scaled centred points) against the oracle run on the cost that form
    evaluates, with the same derived tolerances as the other matrix-core forms (its
    contraction runs over 3 d entries: 16, 64, 128 or 192)."""
    _mfma_step_check("fp16x3_mfma", None, shape)


def test_split_fp16_cost_is_close_to_exact():
    """The split form's cost against the exact one.  hi + lo carries each scaled coordinate to
    2^-23 relative and the dropped x_lo.y_lo is 2^-22 of a product, so 2 s x.y moves by at most
    6 x 2^-22 s sum_k |x_k y_k| <= 1.5e-6 s diam^2 (centred points lie within one diameter of the
    origin), under 2^-19 max C; measured about 5e-8 (FP16 points: 1e-4); and d = 65 is
    rejected."""
    wl = W.random_small(300, 280, 64, seed=77, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    Cs, _ = _split_cost(wl, s)
    Ch, _ = _rounded_cost(wl, s, torch.float16, parts=True)
    e_split, e_half = np.max(np.abs(Cs - C)), np.max(np.abs(Ch - C))
    _say(f"max |C~ - C|: split {e_split:.3e}, FP16 points {e_half:.3e}")
    assert e_split <= 2.0 ** -19 * np.max(C)
    bad = W.random_small(10, 10, 65, seed=1)
    with pytest.raises(P.LampError):
        P.step(P.Problem(bad.x, bad.y, bad.r, bad.c), P.make_params(eta=1e-2, precision="fp16x3_mfma"),
               P.State.fresh(10))


@pytest.mark.parametrize("form,dtype", [("bf16_mfma", torch.bfloat16), ("fp32_mfma", torch.float32)])
def test_mfma_step_with_large_tau1(form, dtype):
    """The one-chain column sweep (d = 64, 128) either scales each column's sum by 2^CA_j once
    (|CA_j| <= 2 LOG2E K tau1 <= 64) or adds CA_j to every exponent: tau1 = 11 (bound 63.5)
    runs the first at offsets up to the limit, tau1 = 12 (bound 69.2) the second.  At t = 1
    lam_{t+1} is about 2.3 times that of the t = 20, tau1 = 1/2 cases; the FP32
    exponent-assembly error grows with lam (c = 2 s lam LOG2E), and the derived bound with it,
    but the column tolerance stays at 2e-5."""
    for tau1 in (11.0, 12.0):
        _mfma_step_check(form, dtype, (160, 200, 64), tau1=tau1, eta=1e-3, t=1)
        _mfma_step_check(form, dtype, (40, 33, 128), tau1=tau1, eta=1e-3, t=1)


def _mfma_step_check(form, dtype, shape, tau1=None, eta=1e-2, t=20):
    n, m, d = shape
    wl = W.random_small(n, m, d, seed=300 + d, eta=eta)
    _say("case", form, wl.name, "tau1", tau1)
    x, y, s, C = oracle_problem(wl)
    Cr, parts = _split_cost(wl, s) if form == "fp16x3_mfma" else _rounded_cost(wl, s, dtype, parts=True)
    prm = OL.Params(eta=wl.eta, tau1=tau1)
    st_or, _ = OL.lamp_dense(Cr, wl.r, wl.c, prm, t, 1.0, trace=False)
    st_next, tr_or = OL.lamp_dense(Cr, wl.r, wl.c, prm, 1, 1.0, state=st_or)
    prob = gpu_problem(wl, s)
    st = _gpu_state(st_or.nu, st_or.theta, st_or.t, st_or.lam)
    res, tr = P.step(prob, P.make_params(eta=wl.eta, precision=form, tau1=tau1 or 0.0), st, trace=True)
    # FP32 exponent assembly: each term carries a relative error ~ ln2 (ulp(g)/2 +
    # c ulp(h + x.y)/2) <~ 1e-5 here; a column's error then moves its dual by
    # kappa |d col_j| / c^alpha_j, which is large only for columns of tiny mass.
    ca, cb = to_np(tr["col_a"]), to_np(tr["col_b"])
    ecol = max(np.max(np.abs(ca / tr_or.colA[0] - 1)), np.max(np.abs(cb / tr_or.colB[0] - 1)))
    calpha = wl.c + 0.01 / m
    allow = 1e-6 + 2.0 * 2e-5 * np.maximum(tr_or.colA[0], tr_or.colB[0]) / calpha
    dual_err = {k: np.max(np.abs(a - b) / allow) for k, (a, b) in dict(
        theta_bar=(to_np(tr["theta_bar"]), tr_or.theta_bar[0]),
        theta_hat=(to_np(tr["theta_hat"]), tr_or.theta_hat[0]),
        theta=(to_np(st.theta), st_next.theta)).items()}
    elz = max(np.max(np.abs(to_np(tr["log_za"]) - tr_or.logZA[0])),
              np.max(np.abs(to_np(tr["log_zb"]) - tr_or.logZB[0])))
    lam_next = OL.inv_eta_schedule(t + 1, prm.resolved(1.0).tau1, wl.eta)[-1]
    ltol, ctol = _mfma_tolerances(form, parts, s, lam_next, [st_or.nu, st_or.theta], n, m, d)
    _say(form, wl.name, f"max row log-normaliser err {elz:.2e} (derived bound {ltol:.2e})")
    _say(form, wl.name, f"max column rel err {ecol:.2e} (derived bound {ctol:.2e})",
         {k: f"{v:.2f}" for k, v in dual_err.items()})
    assert elz <= ltol
    assert ecol <= min(2e-5, ctol)
    for k, v in dual_err.items():
        assert v <= 1.0, (k, dual_err)
    assert rel_dual(to_np(st.nu), st_next.nu) <= 1e-4


@pytest.mark.parametrize("form", ["fp32_mfma", "bf16_mfma"])
def test_mfma_solve_runs_graph(form):
    """The graph-captured loop with a matrix-core form: 200 iterations, residual decreasing."""
    wl = W.random_small(700, 650, 3, seed=21, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    prob = gpu_problem(wl, s)
    st, rep, status = P.solve(prob, P.make_params(eta=wl.eta, max_iter=200, precision=form,
                                                  check_every=25))
    _say(form, rep)
    assert status == 0 and st.t == 200
    assert rep["final_res"] < 0.05


# ---------------------------------------------------------------- batching form

def test_batched_solve_matches_single_solves():
    """Problems of uneven n, m, d solved in one batched launch per phase reproduce the
    single-problem solves: same stopping iteration, duals equal to the parity tolerance."""
    probs_w = [W.random_small(n, m, d, seed=40 + k, eta=1e-2)
               for k, (n, m, d) in enumerate([(300, 200, 2), (128, 450, 3), (257, 257, 16),
                                              (90, 77, 5), (600, 311, 3)])]
    probs = []
    for wl in probs_w:
        s, _ = P.cost_scale(P.Problem(wl.x, wl.y, wl.r, wl.c))
        probs.append(P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0))
    params = P.make_params(eta=1e-2, tol=2e-3, max_iter=3000, check_every=16)
    states, reps, status = P.solve_batched(probs, params)
    _say("batched", [(r["iters"], r["converged"], f"{r['final_res']:.2e}") for r in reps])
    assert status == 0
    for prob, st, rep, wl in zip(probs, states, reps, probs_w):
        single, srep, _ = P.solve(prob, params)
        assert rep["converged"] == 1 and st.t == single.t, (rep, srep)
        # lam_t of each returned state follows from its own t (the same host recursion)
        assert st.inv_eta == single.inv_eta
        assert rel_dual(to_np(st.nu), to_np(single.nu)) <= DUAL_TOL
        assert rel_dual(to_np(st.theta), to_np(single.theta)) <= DUAL_TOL
    # against the oracle for the smallest problem
    wl = probs_w[3]
    x, y, s, C = oracle_problem(wl)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=1e-2), 3000, 1.0, tol=2e-3, trace=False)
    assert states[3].t == st_or.t
    assert rel_dual(to_np(states[3].nu), st_or.nu) <= DUAL_TOL


def test_autograd_function_gradient():
    """LampOT: the transport cost of the solved iterate as a function of x; backward gives the
    envelope gradient, which matches the oracle's at the oracle's own iterate (same iteration
    count, so the same state up to the parity tolerance)."""
    wl = W.random_small(120, 90, 3, seed=51, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    xt = torch.tensor(wl.x, device="cuda", requires_grad=True)
    cost = P.LampOT.apply(xt, torch.tensor(wl.y, device="cuda"), wl.r, wl.c, 1e-2, 0.0, 80, s)
    cost.backward()
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=1e-2), 80, 1.0, trace=False)
    g_or = OL.envelope_grad_x(x, y, wl.r, s, st_or.nu, st_or.lam, 1.0)
    cost_or = float(np.sum(C * OL.plan(C, wl.r, st_or, 1.0)))
    assert float(cost.detach()) == pytest.approx(cost_or, rel=1e-5)
    assert rel_inf(to_np(xt.grad), g_or) <= 1e-4


def test_schedule_epoch_rollover_single_and_batched():
    """More than one 4096-entry schedule table: 4200 iterations at eta = 0, where lam_t = t / 2
    still grows by tau1 = 1/2 per iteration, so a schedule entry read at the wrong index moves every
    exponent by at least C_ij / 2.  One call of 4200 iterations uploads a new table at t = 4096 and
    continues lam_t from the epoch base (step:eta_update); t and lam_t (the same FP64 recursion)
    equal the oracle's exactly.  The duals equal those of the same run made of two calls, 4000
    then 200 iterations (the second call starts a fresh table: no rollover inside either call), up
    to the FP32 differences of the offsets a call starts from (measured below 1e-6 of the clip
    radius); the bound 1e-5 sits three orders of magnitude below what a wrong entry does.  Against
    the oracle the duals are printed.  The batched solve (two problems) rolls over too."""
    T, T1 = 4200, 4000
    ROLL_TOL = 1e-5
    wls = [W.random_small(64, 64, 2, seed=81), W.random_small(80, 70, 3, seed=82)]
    lam_ref = OL.inv_eta_schedule(T, 0.5, 0.0)[-1]
    probs, chunked = [], []
    for wl in wls:
        x, y, s, C = oracle_problem(wl)
        st_or, _ = OL.lamp_dense(C, wl.r, wl.c, OL.Params(eta=0.0), T, 1.0, trace=False)
        probs.append(gpu_problem(wl, s))
        st, rep, status = P.solve(probs[-1], P.make_params(eta=0.0, max_iter=T, check_every=100))
        st2, _, _ = P.solve(probs[-1], P.make_params(eta=0.0, max_iter=T1, check_every=100))
        st2, _, _ = P.solve(probs[-1], P.make_params(eta=0.0, max_iter=T - T1, check_every=100), st2)
        chunked.append(st2)
        e_nu, e_th = rel_dual(to_np(st.nu), to_np(st2.nu)), rel_dual(to_np(st.theta), to_np(st2.theta))
        _say(wl.name, f"t {st.t} lam {st.inv_eta!r} (oracle {st_or.lam!r}); against the two-call run: nu "
                      f"{e_nu:.2e} theta {e_th:.2e}; against the oracle: nu {rel_dual(to_np(st.nu), st_or.nu):.2e} "
                      f"theta {rel_dual(to_np(st.theta), st_or.theta):.2e}")
        assert status == 0 and st.t == T == st_or.t == st2.t
        assert st.inv_eta == st_or.lam == lam_ref == st2.inv_eta == T / 2
        assert e_nu <= ROLL_TOL and e_th <= ROLL_TOL
    states, reps, status = P.solve_batched(probs, P.make_params(eta=0.0, max_iter=T, check_every=100))
    assert status == 0
    for st, st2 in zip(states, chunked):
        assert st.t == T and st.inv_eta == lam_ref
        assert rel_dual(to_np(st.nu), to_np(st2.nu)) <= ROLL_TOL
        assert rel_dual(to_np(st.theta), to_np(st2.theta)) <= ROLL_TOL


def test_row_fallback_path_at_large_tau1():
    """tau1 = 100 at eta = 0 (lam grows by 100 per iteration): between two iterations the
    exponents of a row move by up to tau1 (max_j C_ij - min_j C_ij) plus 3 tau1 K / 2 nats through
    the duals, beyond what the previous iteration's offsets keep inside [2^-60, 2^60], so rows
    take the exact FP64 recomputation of row_finish, and the A coupling's row factor reaches
    hundreds of binary orders (it lives in the exponent, not in an FP32 weight).  A 30-iteration
    solve completes and counts the recomputed rows (row_fallbacks > 0); each step from an oracle
    state matches the oracle.  (Along the whole run the iteration is chaotic at this step size:
    the oracle itself, with its column marginals perturbed by 2^-24 relative, ends O(1) away, so
    trajectories are not compared.)"""
    wl = W.random_small(64, 80, 2, seed=71)
    x, y, s, C = oracle_problem(wl)
    prm = OL.Params(eta=0.0, tau1=100.0)
    T = 30
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=0.0, tau1=100.0, max_iter=T, check_every=5)
    st, rep, status = P.solve(prob, params)
    _say("tau1 = 100", rep)
    assert status == 0 and st.t == T
    assert rep["row_fallbacks"] > 0
    for k in (1, 2, 5, 17):
        st_k, _ = OL.lamp_dense(C, wl.r, wl.c, prm, k, 1.0, trace=False)
        st_n, tr_n = OL.lamp_dense(C, wl.r, wl.c, prm, 1, 1.0, state=st_k)
        g = _gpu_state(st_k.nu, st_k.theta, st_k.t, st_k.lam)
        res, tr = P.step(prob, params, g, trace=True)
        _compare_step(tr, tr_n, 0, g, st_n, f"tau1 = 100, step from t = {k}")


@pytest.mark.parametrize("kind,eta", [("sqeuclid", 1e-2), ("sqeuclid", 0.05), ("l1", 0.02)])
def test_certificate_entropic_dual_values(kind, eta):
    """D^eta(theta^t) and D^eta(nu^t) (def:dual_spp_e) from the certificate against the oracle's
    dual_D_eta evaluated at the GPU's own state (so only the D^eta evaluation is compared): each row's
    softmin is mu_i - eta ln S_i with the minimum mu_i exact in FP64 and S_i a sum of FP32
    exponentials (each <= 1, one of them 1), whose relative error is a few 2^-24: a row moves by
    eta x 3 x 2^-24, the weighted sum by as much; allowed eta 1e-6.  At eta = 0 both are NaN."""
    wl = W.random_small(120, 90, 2, seed=91, eta=eta)
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    s = 1.0 / OL.max_cost(x, y, kind)
    C = OL.ground_cost(x, y, s, kind)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0, metric=kind)
    params = P.make_params(eta=eta, max_iter=60, check_every=20)
    st, rep, status = P.solve(prob, params)
    assert status == 0 and st.t == 60
    cert = P.certificate(prob, params, st)
    th, nu = to_np(st.theta), to_np(st.nu)
    ref_t = OL.dual_D_eta(C, wl.r, wl.c, th, 1.0, eta)
    ref_n = OL.dual_D_eta(C, wl.r, wl.c, nu, 1.0, eta)
    _say(kind, eta, f"D^eta(theta) gpu {cert['dual_eta_theta']:.12e} oracle {ref_t:.12e}; "
                    f"D^eta(nu) gpu {cert['dual_eta_nu']:.12e} oracle {ref_n:.12e}")
    assert abs(cert["dual_eta_theta"] - ref_t) <= eta * 1e-6
    assert abs(cert["dual_eta_nu"] - ref_n) <= eta * 1e-6
    # def:dual_spp_e against def:dual_spp: D - eta log m <= D^eta <= D
    assert cert["dual_theta"] - eta * math.log(90) - 1e-12 <= cert["dual_eta_theta"] <= cert["dual_theta"] + 1e-12
    plain = P.certificate(prob, P.make_params(eta=0.0), st)
    assert math.isnan(plain["dual_eta_theta"]) and math.isnan(plain["dual_eta_nu"])


@pytest.mark.parametrize("d", [20, 32, 64])
def test_certificate_fields_at_wide_dimensions(d):
    """Every certificate field against the oracle's certificate of the GPU's own state (so only
    the certificate's evaluation is compared) at d = 32 and 64, the dimensions with compiled
    certificate passes beyond the sweeps' own, and d = 20 (run-time form).  Bounds: the minima
    of D(theta), D(nu) are FP64 (1e-12); <C, X^t> and the row sums carry FP32 exponentials of
    FP64 arguments, 22 x 2^-24 relative at most per row (derived in test_gpu_cost.py), so
    2e-6; the column residual comes from the FP32 column sweep (its 1e-6 l1 tolerance);
    <C, Round X> as in test_certificate_round_matches_oracle; D^eta as in
    test_certificate_entropic_dual_values."""
    wl = W.random_small(230, 170, d, seed=700 + d, eta=1e-2)
    x, y, s, C = oracle_problem(wl)
    prob = gpu_problem(wl, s)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=30)
    st, _, _ = P.solve(prob, params)
    cert = P.certificate(prob, params, st)
    ost = OL.LampState(st.t, st.inv_eta, to_np(st.nu), to_np(st.theta))
    ref = OL.certificate(C, wl.r, wl.c, ost, OL.Params(eta=wl.eta).resolved(1.0), 1.0)
    _say(f"d = {d}: cost {cert['cost']:.12e} / {ref['cost']:.12e}, row_res {cert['row_res']:.3e} / "
         f"{ref['row_res']:.3e}, col_res {cert['col_res']:.6e} / {ref['col_res']:.6e}, round "
         f"{cert['rounded_cost']:.9e} / {ref['rounded_cost']:.9e}")
    assert abs(cert["cost"] - ref["cost"]) <= 2e-6 * ref["cost"]
    assert abs(cert["row_res"] - ref["row_res"]) <= 2e-6
    assert abs(cert["col_res"] - ref["col_res"]) <= 2e-6
    for key in ("dual_theta", "dual_nu"):
        assert abs(cert[key] - ref[key]) <= 1e-12, key
    assert abs(cert["rounded_cost"] - ref["rounded_cost"]) <= 2e-5
    assert abs(cert["dual_eta_theta"] - ref["dual_eta_theta"]) <= wl.eta * 1e-6
