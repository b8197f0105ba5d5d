"""GPU parity of the D_t tracking (Proposition infeas_bound(b), def:sum_condition) against the
FP64 oracle, which evaluates every summand from its definition on the dense couplings
(oracle.lamp.dt_sequence).  Through the C ABI: lamp_step / lamp_solve with track_dt, and
lamp_certificate, which adds the telescoped normaliser term and the midpoint bound.

Tolerance of one summand (the part the iterations accumulate, without <r, log Z^{t+1} - log Z^t>),
from the error of the terms it is made of rather than from the parity tolerances of its inputs.
Every coupling entry is an FP32 exponential of an FP64 argument; for the entries that carry the
mass (argument within a few units of the row's largest) that is a relative error
delta <= 3 x 2^-24 = 1.8e-7 (rounding of the argument, the exponential's ulp, FP32 partial sums of
8 terms).  A column marginal and a row normaliser then carry 2 delta at most, and:
  the column term K <col(Xbar), lam' nu' - lam nu> (|lam' nu' - lam nu| <= 2 tau1 = 1) moves by
  K 2 delta = 4 delta; the cost term (lam' - lam) <C, Xbar> (lam' - lam <= tau1, <C, Xbar> <= 1) by
  2 tau1 delta = delta; each Bregman term, a c^alpha-weighted Bernoulli KL of the steps' natural
  parameters a_j, whose errors are kappa 2 delta col_j / c^alpha_j, by at most
  sum_j 2 |a_j - b_j| kappa 2 delta col_j <= 4 delta max_j |a_j - b_j|, under 1 here: 4 delta.
In all <= 13 delta = 2.3e-6; the entries carrying the mass are the ones that matter, so
DT_STEP_TOL = 1e-6 (measured: 2e-9 to 8e-8).  Along a trajectory of T iterations the summands'
errors are independent in sign: sqrt(T) DT_STEP_TOL, and the bound's constant 2 ||C||_inf / T
on top for the midpoint bound.
"""
import math
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from paper_2511_11359_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

DT_STEP_TOL = 1e-6


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
    return wl, C, prob


@pytest.mark.parametrize("shape,kind,steps", [((70, 53, 2), "sqeuclid", [0, 1, 10, 60]),
                                              ((64, 64, 3), "l1", [0, 5, 40]),
                                              ((50, 61, 2), "linf", [0, 9]),
                                              ((45, 38, 20), "sqeuclid", [0, 7]),
                                              ((300, 1100, 20), "sqeuclid", [0, 2]),
                                              ((200, 530, 64), "sqeuclid", [0, 3]),
                                              ((90, 170, 100), "sqeuclid", [0, 1]),
                                              ((40, 50, 6), "l1", [0, 3]),
                                              ((30, 40, 150), "sqeuclid", [0, 2]),
                                              ((1, 9, 2), "sqeuclid", [0, 3]),
                                              ((300, 1100, 3), "sqeuclid", [0, 2]),
                                              ((260, 900, 2), "l1", [0, 1])])
def test_dt_summand_of_one_step_matches_oracle(shape, kind, steps):
    """One GPU step from the oracle's FP64 state at s, dt_partial starting at 0: the increment is
    the summand of D_{s+1} without its normaliser telescope.  Covers the D_t sums fused into the
    vector-ALU row sweep (d = 2, 3; 300 x 1100 and 260 x 900 split the columns 9 and 8 ways with
    a ragged last split) and into the FP64 matrix-core row sweep (d = 20, 64, 100: operand widths
    32, 64 and 128; 1100 and 530 columns are 69 and 34 tiles of 16 with ragged last tiles over
    several splits, 300 rows a ragged last wave), the separate cost pass of the dimensions
    without either (l1 at d = 6, squared Euclidean at d = 150), each ground cost and a single
    row."""
    n, m, d = shape
    wl, C, prob = _problem(n, m, d, kind, seed=300 + n)
    _say("case", wl.name, kind)
    prm = OL.Params(eta=wl.eta)
    T = max(steps) + 1
    D, _, traces = OL.dt_sequence(C, wl.r, wl.c, prm, T, 1.0)
    lam = OL.inv_eta_schedule(T, 0.5, wl.eta)
    params = P.make_params(eta=wl.eta, track_dt=True)
    for s in steps:
        nu = np.zeros(m) if s == 0 else traces[s - 1].nu[0]
        th = np.zeros(m) if s == 0 else traces[s - 1].theta[0]
        nu_n = traces[s].nu[0]
        telescope = float(wl.r @ (OL.log_normaliser(C, nu_n, lam[s + 1], 1.0)
                                  - OL.log_normaliser(C, nu, lam[s], 1.0)))
        ref = (D[s] - (D[s - 1] if s else 0.0)) - telescope
        st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), s, float(lam[s]), 0.0)
        P.step(prob, params, st)
        err = abs(st.dt_partial - ref)
        _say(f"  s={s} gpu {st.dt_partial:.9e} oracle {ref:.9e} err {err:.2e}")
        assert st.t == s + 1
        assert err <= DT_STEP_TOL * max(1.0, abs(ref))


@pytest.mark.parametrize("kind,eta", [("sqeuclid", 1e-2), ("l1", 1e-2), ("sqeuclid", 0.0)])
def test_dt_along_a_solve_and_midpoint_bound(kind, eta):
    """T iterations of the graph-captured loop with tracking (several replayed chunks), then the
    certificate: D_T and 2||C||_inf (log m + (1 + alpha) log 2 + D_T)/T against the oracle's;
    eta = 0 is the setting of Proposition infeas_bound."""
    wl, C, prob = _problem(96, 80, 2, kind, seed=71, eta=eta)
    T = 80
    D, _, _ = OL.dt_sequence(C, wl.r, wl.c, OL.Params(eta=eta), T, 1.0)
    params = P.make_params(eta=eta, tol=0.0, max_iter=T, check_every=16, track_dt=True)
    st, rep, status = P.solve(prob, params)
    assert status == 0 and st.t == T
    cert = P.certificate(prob, params, st)
    ref_bound = OL.midpoint_bound(D[-1], T, 80, 0.01, 1.0)
    tol = math.sqrt(T) * DT_STEP_TOL
    _say(kind, f"D_T gpu {cert['dt']:.9e} oracle {D[-1]:.9e} err {abs(cert['dt'] - D[-1]):.2e} (tol {tol:.1e})",
         f"bound gpu {cert['midpoint_bound']:.6e} oracle {ref_bound:.6e}")
    assert abs(cert["dt"] - D[-1]) <= tol
    assert abs(cert["midpoint_bound"] - ref_bound) <= 2.0 * tol / T + 1e-12


@pytest.mark.parametrize("d,tau1", [(2, 100.0), (24, 40.0)])
def test_dt_summands_at_recomputed_rows(d, tau1):
    """tau1 = 100 (40) at eta = 0 (lam grows by tau1 per iteration): in a two-iteration solve
    from an oracle state the row offsets, taken from the previous iteration, leave rows outside
    [2^-60, 2^60]; row_finish recomputes their normalisers exactly (row_fallbacks > 0) and the
    D_t pass of the tracked row sweep evaluates their <C, Xbar> share again in FP64 where its
    B sums left that range (d = 2: the vector-ALU sweep's finish; d = 24: the FP64 matrix-core
    sweep's, dimension at run time).  The two summands (without the normaliser telescope)
    against the oracle's (at d = 24 and tau1 = 100 the oracle's dense FP64 couplings underflow
    inside its Bregman terms; that case is pinned through the duals below)."""
    wl, C, prob = _problem(64, 80, d, "sqeuclid", seed=71, eta=0.0)
    prm = OL.Params(eta=0.0, tau1=tau1)
    k = 5
    T = k + 2
    D, _, traces = OL.dt_sequence(C, wl.r, wl.c, prm, T, 1.0)
    lam = OL.inv_eta_schedule(T, tau1, 0.0)
    nu, th, nu_n = traces[k - 1].nu[0], traces[k - 1].theta[0], traces[k + 1].nu[0]
    telescope = float(wl.r @ (OL.log_normaliser(C, nu_n, lam[k + 2], 1.0) - OL.log_normaliser(C, nu, lam[k], 1.0)))
    ref = (D[k + 1] - D[k - 1]) - telescope
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), k, float(lam[k]), 0.0)
    params = P.make_params(eta=0.0, tau1=tau1, max_iter=2, check_every=2, track_dt=True)
    st, rep, status = P.solve(prob, params, st)
    err = abs(st.dt_partial - ref)
    _say(f"d = {d}, tau1 = {tau1}: fallbacks {rep['row_fallbacks']}, gpu {st.dt_partial:.9e} oracle {ref:.9e} err {err:.2e}")
    assert status == 0 and st.t == k + 2
    assert rep["row_fallbacks"] > 0
    assert err <= 2.0 * DT_STEP_TOL * max(1.0, abs(ref))


def test_matrix_core_row_weights_at_large_tau1():
    """d = 24 (FP64 matrix-core sweeps), tau1 = 100 at eta = 0: the A coupling's row factor
    2^ew, |ew| up to LOG2E (K tau1 max|theta - nu| + ln m) (about 144 here), exceeds FP32 as a
    weight of the matrix-core column sweep; row_finish shares it between both couplings'
    weights by moving that sweep's offset for rows with |ew| > 100.  Two iterations from the
    oracle's state at t = 5, the duals against the oracle's.  The columns carry FP32 sums of
    relative error ~1e-6 and c^alpha_j ~ 1/m, so a dual moves by ~1e-6 (columns whose mass
    underflows FP32 read 0 against ~1e-245 in FP64, which moves their duals by less)."""
    wl, C, prob = _problem(64, 80, 24, "sqeuclid", seed=71, eta=0.0)
    prm = OL.Params(eta=0.0, tau1=100.0)
    k = 5
    _, _, traces = OL.dt_sequence(C, wl.r, wl.c, prm, k + 2, 1.0)
    lam = OL.inv_eta_schedule(k + 2, 100.0, 0.0)
    st = P.State(torch.tensor(traces[k - 1].nu[0], device="cuda"),
                 torch.tensor(traces[k - 1].theta[0], device="cuda"), k, float(lam[k]), 0.0)
    params = P.make_params(eta=0.0, tau1=100.0, max_iter=2, check_every=2)
    st, rep, status = P.solve(prob, params, st)
    e_nu = np.max(np.abs(st.nu.cpu().numpy() - traces[k + 1].nu[0]))
    e_th = np.max(np.abs(st.theta.cpu().numpy() - traces[k + 1].theta[0]))
    _say(f"d = 24, tau1 = 100: fallbacks {rep['row_fallbacks']}, nu err {e_nu:.2e}, theta err {e_th:.2e}")
    assert status == 0 and st.t == k + 2
    assert rep["row_fallbacks"] > 0
    assert e_nu <= 1e-5 and e_th <= 1e-5


def test_dt_resume_untracked_and_rejected_forms():
    """A tracked run split in two calls accumulates the same D_t as one call, to the trajectory
    tolerance (the second call starts from exact row offsets, which changes the FP32 rounding of
    the sums, as for the duals of a resumed solve); an untracked iteration makes the partial sum
    NaN (so the certificate reports NaN); the matrix-core forms and the batching form reject
    tracking."""
    wl, _, prob = _problem(120, 100, 3, "sqeuclid", seed=73)
    params = P.make_params(eta=wl.eta, max_iter=60, check_every=16, track_dt=True)
    whole, _, _ = P.solve(prob, params)
    half = P.make_params(eta=wl.eta, max_iter=30, check_every=16, track_dt=True)
    st, _, _ = P.solve(prob, half)
    st, _, _ = P.solve(prob, half, st)
    assert st.t == whole.t == 60
    _say(f"split {st.dt_partial:.12e} whole {whole.dt_partial:.12e}")
    assert abs(st.dt_partial - whole.dt_partial) <= math.sqrt(30) * DT_STEP_TOL
    assert math.isfinite(P.certificate(prob, params, st)["dt"])
    untracked = P.make_params(eta=wl.eta, max_iter=1)
    st2, _, _ = P.solve(prob, untracked, st)
    assert st2.t == 61 and math.isnan(st2.dt_partial)
    assert math.isnan(P.certificate(prob, untracked, st2)["dt"])
    with pytest.raises(P.LampError):
        P.solve(prob, P.make_params(eta=wl.eta, max_iter=5, precision="bf16_mfma", track_dt=True))
    with pytest.raises(P.LampError):
        P.solve_batched([prob, prob], P.make_params(eta=wl.eta, max_iter=5, track_dt=True))
