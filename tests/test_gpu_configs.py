"""GPU parity on the two workloads that stand beside the headline one: the 4096 x 4096
Gaussian pair (d = 3, Dirichlet marginals, eta = 1e-3, run to ||col(X^t) - c||_1 <= 1e-4) and
the 64-problem batch (n, m log-uniform in [512, 8192], d in {2, 3, 16}, eta = 1e-3), against the
oracle's full-size C pass (oracle/rowpass.c, FP64): every row's log-normalisers and every
column's marginals and dual steps.  Tolerances as in test_gpu_fullsize (FP32 form)."""
import json
import os
import sys
import time

import numpy as np
import pytest

from oracle import cmax
from oracle import lamp as OL
from oracle import rowpass as RP
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import rel_dual, rel_inf, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cost_scales.json")))
LOGZ_ATOL = 2e-6
COL_RTOL = 4e-6          # per column: normaliser error + FP32 exponential of an FP64 argument + sums
COL_FLOOR = 1e-30        # a column whose every term is below FP32's normal range sums to ~0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _step_parity(tag, prob, wl, t, lam, nu, th, cost):
    """One GPU step from (t, lam, nu, theta) against the oracle's full step: every row, every
    column.  The dual bounds follow from the column tolerance (def:closed_form_opt)."""
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam)
    res, tr = P.step(prob, P.make_params(eta=wl.eta), st, trace=True)
    torch.cuda.synchronize()
    m = wl.m
    ref = RP.step_sampled(cost, wl.r, wl.c, lam, nu, th, OL.Params(eta=wl.eta), 1.0, np.arange(m))
    ea = np.max(np.abs(to_np(tr["log_za"]) - ref["logZA"]))
    eb = np.max(np.abs(to_np(tr["log_zb"]) - ref["logZB"]))
    ca, cb = to_np(tr["col_a"]), to_np(tr["col_b"])
    fl = COL_FLOOR / COL_RTOL
    rca = np.max(np.abs(ca - ref["colA"]) / np.maximum(ref["colA"], fl))
    rcb = np.max(np.abs(cb - ref["colB"]) / np.maximum(ref["colB"], fl))
    calpha = wl.c + 0.01 / m
    lim_bar = 1e-14 + (COL_RTOL * ref["colA"] + COL_FLOOR) / calpha
    lim_hat = 1e-14 + (COL_RTOL * ref["colB"] + COL_FLOOR) / calpha
    d_bar = np.abs(to_np(tr["theta_bar"]) - ref["theta_bar"])
    d_hat = np.abs(to_np(tr["theta_hat"]) - ref["theta_hat"])
    d_nu = np.abs(to_np(st.nu) - ref["nu"])
    d_th = np.abs(to_np(st.theta) - ref["theta"])
    w = 0.5 / ref["lam_next"]
    _say(tag, f"t {t}: logZ {max(ea, eb):.2e}, col rel {max(rca, rcb):.2e}, duals plain rel "
              f"nu {rel_inf(to_np(st.nu), ref['nu']):.2e} theta {rel_inf(to_np(st.theta), ref['theta']):.2e}, "
              f"floored nu {rel_dual(to_np(st.nu), ref['nu']):.2e} theta {rel_dual(to_np(st.theta), ref['theta']):.2e}")
    assert ea <= LOGZ_ATOL and eb <= LOGZ_ATOL
    assert rca <= COL_RTOL and rcb <= COL_RTOL
    assert np.all(d_bar <= lim_bar) and np.all(d_hat <= lim_hat)
    assert np.all(d_nu <= 1e-14 + w * lim_bar) and np.all(d_th <= lim_hat)
    assert st.t == t + 1 and st.inv_eta == ref["lam_next"]
    assert res == pytest.approx(float(np.abs(ref["colA"] - wl.c).sum()), rel=1e-5, abs=1e-9)


def test_gauss3d_4096_steps_and_stop_iteration():
    """The 4096 x 4096 Gaussian workload: the oracle runs Algorithm 2 from the start to the
    tolerance (full steps); one GPU step from its state at t = 1, 10, 100 and 400 matches it on
    every row and column; the GPU solve from the start stops at the same iteration, and its duals
    there agree with the oracle's to what 400+ FP32 iterations allow (printed beside)."""
    key = "gauss3d_4096"
    wl = W.gaussian_pair()
    s = GOLD[key]["cost_scale"]
    cost = RP.Cost(s, 1.0, x=wl.x, y=wl.y)
    t0 = time.time()
    keep = (1, 10, 100, 400)
    run = RP.solve(cost, wl.r, wl.c, OL.Params(eta=wl.eta), 1.0, 5000, tol=wl.tol, keep=keep)
    _say(f"oracle: stops at t = {run['t']} (residual {run['res']:.6e}), {time.time() - t0:.1f} s")
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    for t in keep:
        if t in run["saved"]:
            lam, nu, th = run["saved"][t]
            _step_parity(key, prob, wl, t, lam, nu, th, cost)
    st, rep, status = P.solve(prob, P.make_params(eta=wl.eta, tol=wl.tol, max_iter=5000))
    _say("gpu solve", rep, f"nu plain rel {rel_inf(to_np(st.nu), run['nu']):.2e}, "
                           f"theta plain rel {rel_inf(to_np(st.theta), run['theta']):.2e}")
    assert status == 0 and rep["converged"] == 1
    assert st.t == run["t"]
    assert st.inv_eta == pytest.approx(run["lam"], rel=1e-14)
    assert rep["final_res"] <= wl.tol


def _batch(count):
    wls = [W.batch_problem(p) for p in range(count)]
    scales = [1.0 / cmax.max_sqdist(w.x, w.y) for w in wls]
    probs = [P.Problem(w.x, w.y, w.r, w.c, cost_scale=s, cost_norm=1.0) for w, s in zip(wls, scales)]
    return wls, scales, probs


def test_batch64_one_step_every_problem():
    """The 64-problem batch: one batched iteration at t = 50 from seeded synthetic states (one
    launch per phase for the whole batch), every problem's updated duals against the oracle's
    full step on every column."""
    wls, scales, probs = _batch(64)
    t = 50
    lam = OL.inv_eta_schedule(t + 1, 0.5, 1e-3)
    starts = [W.synthetic_duals(w.m, 600 + p) for p, w in enumerate(wls)]
    states = [P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam[t])
              for nu, th in starts]
    states, reps, status = P.solve_batched(probs, P.make_params(eta=1e-3, max_iter=1, check_every=1), states)
    assert status == 0
    worst = 0.0
    for p, (w, s, st, (nu, th)) in enumerate(zip(wls, scales, states, starts)):
        ref = RP.step_sampled(RP.Cost(s, 1.0, x=w.x, y=w.y), w.r, w.c, lam[t], nu, th, OL.Params(eta=1e-3),
                              1.0, np.arange(w.m))
        calpha = w.c + 0.01 / w.m
        lim_bar = 1e-14 + (COL_RTOL * ref["colA"] + COL_FLOOR) / calpha
        lim_hat = 1e-14 + (COL_RTOL * ref["colB"] + COL_FLOOR) / calpha
        d_nu = np.abs(to_np(st.nu) - ref["nu"])
        d_th = np.abs(to_np(st.theta) - ref["theta"])
        wgt = 0.5 / ref["lam_next"]
        ratio = max(np.max(d_nu / (1e-14 + wgt * lim_bar)), np.max(d_th / lim_hat))
        worst = max(worst, ratio)
        assert st.t == t + 1 and st.inv_eta == ref["lam_next"], p
        assert ratio <= 1.0, (p, w.n, w.m, w.d, ratio)
    _say(f"batch64: all 64 problems within the bounds, worst error / bound {worst:.3f}")


def test_batch64_stop_iterations():
    """The 64-problem batch solved to ||col(X^t) - c||_1 <= 1e-4 in one batched solve: the four
    smallest problems (by n m) stop at the oracle's iteration, every problem converges, and a
    problem's stop does not depend on the others (each equals its own single solve)."""
    wls, scales, probs = _batch(64)
    params = P.make_params(eta=1e-3, tol=1e-4, max_iter=20000, check_every=32)
    states, reps, status = P.solve_batched(probs, params)
    assert status == 0 and all(r["converged"] == 1 for r in reps)
    order = sorted(range(64), key=lambda p: wls[p].n * wls[p].m)
    for p in order[:4]:
        w = wls[p]
        run = RP.solve(RP.Cost(scales[p], 1.0, x=w.x, y=w.y), w.r, w.c, OL.Params(eta=1e-3), 1.0, 20000,
                       tol=1e-4)
        single, srep, _ = P.solve(probs[p], params)
        _say(f"problem {p} ({w.n} x {w.m}, d = {w.d}): batched t {states[p].t}, single t {single.t}, "
             f"oracle t {run['t']}")
        assert states[p].t == run["t"] == single.t
