"""Full-size GPU checks in the launch configuration the benchmark times.

At n = m = 2^16 (d = 64) and n = m = 2^18 (d = 3) one GPU iteration from a seeded
synthetic state is checked element by element against the oracle's full-size C pass
(oracle/rowpass.c, FP64, threaded over the host's cores): the row log-normalisers of
both couplings on every row, and on at least 64 sampled columns (tile and range ends
included) both column marginals, both dual mirror steps and the updated duals.  Beside
those, properties that hold at any size (each column marginal sums to sum(r) = 1, duals
stay in (-1, 1)), gradient rows, and the certificate.  The cost normalisation comes from
tests/golden/cost_scales.json, written by the oracle's exact C routine.

Tolerances.  FP32 form (FP64 exponent arguments): row log-normalisers 2e-6 absolute; a
column marginal is a sum of terms r_i exp(a_ij - log Z_i), so its relative error is at
most the normalisers' error plus the per-term error of an FP32 exponential of an FP64
argument of magnitude <= 30 (30 x 2^-24 x ln 2 = 1.2e-6) plus FP32 partial sums of 8 terms
(8 x 2^-24): 4e-6 per column.  Matrix-core forms: per-term bound of
tests.gpu_util.mfma_term_bound (FP32 exponent assembly) plus the FP32 sums of a split; a
column marginal twice that.  A dual step moves with its column: |d thetabar_j| <=
kappa |d col_j| / c^alpha_j (def:closed_form_opt), and nu^{t+1}_j by w times that.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

from oracle import cmax
from oracle import lamp as OL
from oracle import rowpass as RP
from oracle import stream as OS
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import (U32, mfma_term_bound, rel_dual, rel_inf, round_to_type, sample_columns,
                            split_fp16, split_fp16_scale,
                            to_np)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cost_scales.json")))
SAMPLE = np.array([0, 1, 31, 32, 4095, 12345, 33333, 65535])



def _operands(dtype, xc, yc):
    """The operands whose FP64 inner products give the cost a matrix-core form computes, and the
    operand width: each centred coordinate rounded once to the operand type; for the split FP16
    form ("fp16x3") the three-part vectors [x_hi, x_hi, x_lo] and [y_hi, y_lo, y_hi] of the
    range-scaled points, divided back by the scale (exact, a power of two)."""
    if dtype == "fp16x3":
        sc = split_fp16_scale(xc, yc)
        xh, xl = split_fp16(xc, sc)
        yh, yl = split_fp16(yc, sc)
        d = xc.shape[1]
        kp = next(k for k in (16, 64, 128, 192) if 3 * d <= k)
        return np.hstack([xh, xh, xl]) / sc, np.hstack([yh, yl, yh]) / sc, kp
    return round_to_type(xc, dtype), round_to_type(yc, dtype), 64

def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _synthetic_state(wl, t, seed):
    nu, th = W.synthetic_duals(wl.m, seed)
    lam = OL.inv_eta_schedule(t + 1, 1.0 / 2.0, wl.eta)
    return nu, th, lam[t], lam[t + 1]


def _check_step(wl, key, precision, t, cost, logz_tol, col_tol, with_trace=False, with_ref=False):
    """One GPU iteration at t from the seeded synthetic state, against the oracle's full-size
    pass over `cost` (every row, sampled columns), plus size-independent properties."""
    s = GOLD[key]["cost_scale"]
    nu, th, lam_t, lam_t1 = _synthetic_state(wl, t, seed=77)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam_t)
    _say("case", key, precision, "t", t, "lam", lam_t)
    res, tr = P.step(prob, P.make_params(eta=wl.eta, precision=precision), st, trace=True)
    torch.cuda.synchronize()
    cols = sample_columns(wl.m)
    t0 = time.time()
    ref = RP.step_sampled(cost, wl.r, wl.c, lam_t, nu, th, OL.Params(eta=wl.eta), 1.0, cols)
    _say(f"  oracle full-size pass {time.time() - t0:.1f} s")
    assert ref["lam_next"] == pytest.approx(lam_t1, rel=1e-15)
    assert res == pytest.approx(float(np.abs(to_np(tr["col_a"]) - wl.c).sum()), rel=1e-12)
    _full_parity(f"{key} {precision}", st, tr, ref, cols, wl.c, 0.01, logz_tol, col_tol, 0.5 / lam_t1)
    ca, cb = to_np(tr["col_a"]), to_np(tr["col_b"])
    _say(key, precision, f"sum colA-1 {ca.sum() - 1:.2e} sum colB-1 {cb.sum() - 1:.2e} res {res:.3e}")
    assert abs(ca.sum() - 1.0) <= 1e-6 and abs(cb.sum() - 1.0) <= 1e-6
    # marginals are non-negative; a column whose every term lies below FP32's range reads 0
    assert np.all(ca >= 0) and np.all(cb >= 0)
    assert np.all(np.abs(to_np(st.theta)) < 1) and np.all(np.abs(to_np(st.nu)) < 1)
    if with_ref:
        return prob, st, ref
    return (prob, st, tr) if with_trace else (prob, st)


FP32_LOGZ_ATOL = 2e-6
FP32_COL_RTOL = 4e-6
COL_FLOOR = 1e-30


def _full_parity(tag, st, tr, ref, cols, c, alpha, logz_tol, col_tol, w):
    """GPU iteration (state after the step, trace) against the oracle's full-size pass `ref`
    (rowpass.step_sampled): every row's log-normalisers, and the sampled columns."""
    m = c.shape[0]
    ea = np.max(np.abs(to_np(tr["log_za"]) - ref["logZA"]))
    eb = np.max(np.abs(to_np(tr["log_zb"]) - ref["logZB"]))
    got = dict(colA=to_np(tr["col_a"])[cols], colB=to_np(tr["col_b"])[cols],
               theta_bar=to_np(tr["theta_bar"])[cols], theta_hat=to_np(tr["theta_hat"])[cols],
               nu=to_np(st.nu)[cols], theta=to_np(st.theta)[cols])
    # a column whose every term lies below FP32's normal range sums to (nearly) zero on the GPU:
    # its mass is below n 2^-126 < COL_FLOOR, an absolute allowance beside the relative one
    rc = {k: np.max(np.abs(got[k] - ref[k]) / np.maximum(ref[k], COL_FLOOR / col_tol)) for k in ("colA", "colB")}
    calpha = c[cols] + alpha / m
    kappa = 1.0                                   # 2 tau2 ||C||_inf at the default tau2
    lim_bar = 1e-14 + kappa * (col_tol * ref["colA"] + COL_FLOOR) / calpha
    lim_hat = 1e-14 + kappa * (col_tol * ref["colB"] + COL_FLOOR) / calpha
    d = {k: np.abs(got[k] - ref[k]) for k in ("theta_bar", "theta_hat", "nu", "theta")}
    plain = {k: rel_inf(got[k], ref[k]) for k in d}
    floored = {k: rel_dual(got[k], ref[k]) for k in d}
    _say(tag, f"rows: logZA {ea:.2e} logZB {eb:.2e} (tol {logz_tol:.1e}); {len(cols)} columns: "
              f"colA {rc['colA']:.2e} colB {rc['colB']:.2e} (tol {col_tol:.1e}); duals plain rel "
         + " ".join(f"{k} {v:.2e}" for k, v in plain.items())
         + "; floored " + " ".join(f"{k} {v:.2e}" for k, v in floored.items())
         + f"; worst dual / bound {max(np.max(d['theta_bar'] / lim_bar), np.max(d['theta_hat'] / lim_hat)):.3f}")
    assert ea <= logz_tol and eb <= logz_tol, (ea, eb)
    assert rc["colA"] <= col_tol and rc["colB"] <= col_tol, rc
    assert np.all(d["theta_bar"] <= lim_bar)
    assert np.all(d["theta_hat"] <= lim_hat)
    assert np.all(d["nu"] <= 1e-14 + w * lim_bar)
    assert np.all(d["theta"] <= lim_hat)


def _check_certificate(prob, params, nu, th, t, lam_t, col_a, c):
    """Certificate of the iterate X^t a step started from (the state before the step), at full
    size, by properties that hold at any size: its column residual equals ||col(X^t) - c||_1
    from the sweep's own column marginal of the same iterate (a different kernel path), the
    row residual vanishes (row feasibility, eq:row_feasible), weak duality puts D(theta) and
    D(nu) below the cost of the feasible plan Round(X^t), and Round moves the cost by at most
    ||C||_inf ||X - Round(X)||_1 <= K (row_res + col_res) (Algorithm 3 guarantee)."""
    st0 = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam_t)
    cert = P.certificate(prob, params, st0)
    ref_col = float(np.abs(col_a - c).sum())
    _say("certificate", {k: cert[k] for k in ["col_res", "row_res", "cost", "rounded_cost", "dual_theta",
                                              "dual_nu", "primal_penalized"]}, "sweep col_res", ref_col)
    assert abs(cert["col_res"] - ref_col) <= 1e-6 * max(1.0, ref_col)
    assert cert["row_res"] <= 1e-6
    assert max(cert["dual_theta"], cert["dual_nu"]) <= cert["rounded_cost"] + 1e-12
    assert cert["rounded_cost"] <= cert["primal_penalized"] + 1e-12


def test_sphere_cube_262144_step_and_gradient():
    """2^18 x 2^18, d = 3: one FP32-form iteration at t = 400 (every row, sampled columns); then the adjoint
    at the resulting state: 16 random gradient coordinates against the oracle's per-row
    envelope gradient and against central finite differences of the row term (h = 1e-4); and
    the adjoint with respect to y at the state the step started from, on 34 columns (the 16
    of largest gradient, both ends, 16 random ones), against the oracle's column gradient
    over every row, with the row log-normalisers of that state from the oracle's full-size
    pass; and the transport cost of that state against the oracle's full-size row costs."""
    key = "sphere_cube_262144"
    wl = W.sphere_cube()
    s = GOLD[key]["cost_scale"]
    prob, st, ref = _check_step(wl, key, "fp32", 400, RP.Cost(s, 1.0, x=wl.x, y=wl.y), FP32_LOGZ_ATOL,
                                FP32_COL_RTOL, with_ref=True)
    nu0, th0, lam0, _ = _synthetic_state(wl, 400, seed=77)
    st0 = P.State(torch.tensor(nu0, device="cuda"), torch.tensor(th0, device="cuda"), 400, lam0)
    gy = to_np(P.backward_y(prob, P.make_params(eta=wl.eta), st0, grad_out=1.0))
    # most target points far from the sphere carry no mass at this temperature (gradient 0 on
    # both sides): the sample takes the 16 columns of largest gradient, both ends and 16
    # random ones
    big = np.argsort(-np.linalg.norm(gy, axis=1))[:16]
    ycols = np.concatenate([[0, wl.m - 1], big, np.random.default_rng(9).integers(0, wl.m, 16)])
    gy_or = OL.envelope_grad_y_columns(wl.x.astype(np.float64), wl.y.astype(np.float64), wl.r, s, nu0, lam0,
                                       1.0, ycols, ref["logZA"])
    yscale = np.maximum(np.abs(gy_or), 1e-3 * np.max(np.abs(gy)))
    yerr = np.abs(gy[ycols] - gy_or) / yscale
    _say(f"y-gradient on {len(ycols)} columns: |g| up to {np.max(np.abs(gy_or)):.3e}, "
         f"max scaled error {np.max(yerr):.2e} (on the 16 largest {np.max(yerr[2:18]):.2e})")
    assert np.max(np.abs(gy_or[2:18])) > 0.1 * np.max(np.abs(gy))
    assert np.max(yerr) <= 1e-5
    # the transport cost <C, X^t> of the same state (the autograd forward's value): every row's
    # expected cost from the oracle's full-size pass; relative tolerance 2e-6, the per-row
    # bound of the transport-cost tests (FP32 exponentials of FP64 arguments, FP32 block sums)
    E = RP.Cost(s, 1.0, x=wl.x, y=wl.y).row_costs([nu0], [lam0], ref["logZA"][None, :])[0]
    ref_cost = float(wl.r @ E)
    got_cost = float(P.transport_cost(prob, P.make_params(eta=wl.eta), st0))
    _say(f"transport cost gpu {got_cost:.12e} oracle {ref_cost:.12e} rel {abs(got_cost / ref_cost - 1):.2e}")
    assert abs(got_cost - ref_cost) <= 2e-6 * abs(ref_cost)
    g = to_np(P.backward(prob, P.make_params(eta=wl.eta), st, grad_out=1.0))
    rng = np.random.default_rng(5)
    coords = [(int(rng.integers(0, wl.n)), int(rng.integers(0, 3))) for _ in range(16)]
    nu = to_np(st.nu)
    lam = st.inv_eta
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    for (i, k) in coords:
        gi = OL.envelope_grad_x(x[i:i + 1], y, wl.r[i:i + 1], s, nu, lam, 1.0)[0, k]
        h = 1e-4
        xp, xm = x[i:i + 1].copy(), x[i:i + 1].copy()
        xp[0, k] += h
        xm[0, k] -= h
        fd = (OL.envelope_value_rows(xp, y, wl.r[i:i + 1], s, nu, lam, 1.0)[0]
              - OL.envelope_value_rows(xm, y, wl.r[i:i + 1], s, nu, lam, 1.0)[0]) / (2 * h)
        scale = max(abs(gi), 1e-3 * np.max(np.abs(g)))
        _say(f"grad[{i},{k}] gpu {g[i, k]:.9e} oracle {gi:.9e} fd {fd:.9e}")
        assert abs(g[i, k] - gi) <= 1e-5 * scale + 1e-12
        assert abs(fd - gi) <= 1e-4 * scale + 1e-12


def test_gmm64_65536_fp32_step():
    """2^16 x 2^16, d = 64: one FP32-form (FP64 argument) iteration at t = 300 (every row, sampled
    columns);
    the certificate of the iterate the step started from."""
    wl = W.gmm64()
    s = GOLD["gmm64d_65536"]["cost_scale"]
    prob, st, tr = _check_step(wl, "gmm64d_65536", "fp32", 300, RP.Cost(s, 1.0, x=wl.x, y=wl.y),
                               FP32_LOGZ_ATOL, FP32_COL_RTOL, with_trace=True)
    nu, th, lam_t, _ = _synthetic_state(wl, 300, seed=77)
    _check_certificate(prob, P.make_params(eta=wl.eta), nu, th, 300, lam_t, to_np(tr["col_a"]), wl.c)


@pytest.mark.parametrize("form,dtype,kstep", [("bf16_mfma", "bfloat16", 16), ("fp16_mfma", "float16", 16),
                                              ("fp32_mfma", "float32", 2), ("fp16x3_mfma", "fp16x3", 16)])
def test_gmm64_65536_mfma_step(form, dtype, kstep):
    """2^16 x 2^16, d = 64: one matrix-core iteration at t = 300 (every row, sampled columns)
    against the oracle evaluated on the cost the form computes: each centred coordinate rounded
    once to the operand type (for the split FP16 form: its three-part operands), FP64 inner
    products of the operands, unrounded squared norms, C_ij = s (|x~_i|^2 + |y~_j|^2 - 2 xr_i . yr_j)."""
    key = "gmm64d_65536"
    wl = W.gmm64()
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    xr, yr, kp = _operands(dtype, xc, yc)
    nx, ny = np.sum(xc * xc, axis=1), np.sum(yc * yc, axis=1)
    s = GOLD[key]["cost_scale"]
    nu, th, lam_t, lam_t1 = _synthetic_state(wl, 300, seed=77)
    term = mfma_term_bound(xr, yr, ny, s, lam_t1, [nu, th], kp, kstep)
    logz_tol = term + (wl.m / 256 + 6) * U32
    col_tol = logz_tol + term + (wl.n / 256 + 6) * U32
    _say(form, f"per-term bound {term:.2e}: logZ tol {logz_tol:.2e}, column tol {col_tol:.2e}")
    _check_step(wl, key, form, 300, RP.Cost(s, 1.0, gram=(xr, yr, nx, ny)), logz_tol, col_tol)


def test_sphere_cube_262144_bf16_step():
    """2^18 x 2^18, d = 3: one BF16 matrix-core iteration at t = 400 (every row, sampled columns)
    against the oracle's pass over the cost the form computes (centred coordinates rounded to
    BF16, FP64 inner products, unrounded squared norms); tolerances from the FP32-assembly bound."""
    key = "sphere_cube_262144"
    wl = W.sphere_cube()
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    xr, yr = round_to_type(xc, "bfloat16"), round_to_type(yc, "bfloat16")
    nx, ny = np.sum(xc * xc, axis=1), np.sum(yc * yc, axis=1)
    s = GOLD[key]["cost_scale"]
    nu, th, lam_t, lam_t1 = _synthetic_state(wl, 400, seed=77)
    term = mfma_term_bound(xr, yr, ny, s, lam_t1, [nu, th], 16, 16)
    logz_tol = term + (wl.m / 256 + 6) * U32
    col_tol = logz_tol + term + (wl.n / 256 + 6) * U32
    _say(f"per-term bound {term:.2e}: logZ tol {logz_tol:.2e}, column tol {col_tol:.2e}")
    _check_step(wl, key, "bf16_mfma", 400, RP.Cost(s, 1.0, gram=(xr, yr, nx, ny)), logz_tol, col_tol)


def test_sphere_cube_bf16_forward_then_fp32_adjoint():
    """The differentiation workload end to end: 2^18 x 2^18, d = 3, BF16-MFMA forward from the
    start until ||col(X^t) - c||_1 <= 1e-4, then the FP32 adjoint at the final state; 16 random
    gradient coordinates against the oracle's envelope gradient (exact cost) and against
    central finite differences of the row term (h = 1e-4)."""
    key = "sphere_cube_262144"
    wl = W.sphere_cube()
    s = GOLD[key]["cost_scale"]
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    st, rep, status = P.solve(prob, P.make_params(eta=wl.eta, tol=1e-4, max_iter=20000,
                                                  precision="bf16_mfma"))
    _say("bf16 forward", rep)
    assert status == 0 and rep["converged"] == 1 and rep["final_res"] <= 1e-4
    g = to_np(P.backward(prob, P.make_params(eta=wl.eta), st, grad_out=1.0))
    nu = to_np(st.nu)
    lam = st.inv_eta
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    rng = np.random.default_rng(7)
    coords = [(int(rng.integers(0, wl.n)), int(rng.integers(0, 3))) for _ in range(16)]
    for (i, k) in coords:
        gi = OL.envelope_grad_x(x[i:i + 1], y, wl.r[i:i + 1], s, nu, lam, 1.0)[0, k]
        h = 1e-4
        xp, xm = x[i:i + 1].copy(), x[i:i + 1].copy()
        xp[0, k] += h
        xm[0, k] -= h
        fd = (OL.envelope_value_rows(xp, y, wl.r[i:i + 1], s, nu, lam, 1.0)[0]
              - OL.envelope_value_rows(xm, y, wl.r[i:i + 1], s, nu, lam, 1.0)[0]) / (2 * h)
        scale = max(abs(gi), 1e-3 * np.max(np.abs(g)))
        _say(f"grad[{i},{k}] gpu {g[i, k]:.9e} oracle {gi:.9e} fd {fd:.9e}")
        assert abs(g[i, k] - gi) <= 1e-5 * scale + 1e-12
        assert abs(fd - gi) <= 1e-4 * scale + 1e-12


def test_images_256_explicit_cost_step():
    """The cost-matrix benchmark at n = m = 2^16 (two 256 x 256 images, squared Euclidean grid
    cost, 16 GiB FP32 on the device): the cost maximum against its closed form 2 (k - 1)^2;
    one iteration at t = 300 from a synthetic state in the launch configuration the benchmark
    times, sampled rows' log-normalisers against the oracle (cost rows from the pixel
    coordinates), each column marginal summing to 1."""
    k = 256
    wl = W.image_pair_device(k, "sqeuclid", device="cuda")
    prob = P.Problem.from_cost(wl.cost, wl.r, wl.c)
    s, cmax = P.cost_scale(prob)
    assert cmax == 2.0 * (k - 1) ** 2 and s == 1.0 / cmax
    prob.cost_scale, prob.cost_norm = s, 1.0
    n = k * k
    t = 300
    nu, th = W.synthetic_duals(n, 77)
    lam = OL.inv_eta_schedule(t + 1, 0.5, wl.eta)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam[t])
    res, tr = P.step(prob, P.make_params(eta=wl.eta), st, trace=True)
    yy, xx = np.divmod(np.arange(n), k)
    pts = np.stack([yy, xx], axis=1).astype(np.float64)
    Crows = OL.ground_cost(pts[SAMPLE], pts, s, "sqeuclid")
    nubar = nu + (0.5 / lam[t + 1]) * (th - nu)
    la = OL.log_normaliser(Crows, nu, lam[t], 1.0)
    lb = OL.log_normaliser(Crows, nubar, lam[t + 1], 1.0)
    ea = np.max(np.abs(to_np(tr["log_za"])[SAMPLE] - la))
    eb = np.max(np.abs(to_np(tr["log_zb"])[SAMPLE] - lb))
    ca, cb = to_np(tr["col_a"]), to_np(tr["col_b"])
    _say(f"explicit 2^16: logZA err {ea:.2e} logZB err {eb:.2e} sum colA-1 {ca.sum() - 1:.2e} "
         f"sum colB-1 {cb.sum() - 1:.2e} res {res:.3e}")
    assert ea <= 2e-6 and eb <= 2e-6
    assert abs(ca.sum() - 1.0) <= 1e-6 and abs(cb.sum() - 1.0) <= 1e-6
    assert np.all(ca >= 0) and np.all(cb >= 0)
    assert np.all(np.abs(to_np(st.theta)) < 1) and np.all(np.abs(to_np(st.nu)) < 1)
    _check_certificate(prob, P.make_params(eta=wl.eta), nu, th, t, lam[t], ca, wl.c)


@pytest.mark.parametrize("shape", [(4096, 65536), (65536, 4096)])
@pytest.mark.parametrize("form,dtype,kstep", [("bf16_mfma", "bfloat16", 16), ("fp16_mfma", "float16", 16),
                                              ("fp32_mfma", "float32", 2), ("fp16x3_mfma", "fp16x3", 16)])
def test_gmm64_medium_mfma_step_every_row_and_column(shape, form, dtype, kstep):
    """d = 64 GMM points at n x m = 4096 x 65536 and 65536 x 4096: each split of both sweeps
    streams 16 tiles, so the pipelined tile loop (prefetch two tiles ahead, buffer swap, clamped
    last tile) runs in steady state; one step at t = 300 against the oracle's pass over the
    rounded-operand cost, on every row and every column."""
    n, m = shape
    wl = W.gmm64(n, m)
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    s = 1.0 / cmax.max_sqdist(wl.x, wl.y)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    xr, yr, kp = _operands(dtype, xc, yc)
    nx, ny = np.sum(xc * xc, axis=1), np.sum(yc * yc, axis=1)
    t = 300
    nu, th = W.synthetic_duals(m, 78)
    lam = OL.inv_eta_schedule(t + 1, 0.5, wl.eta)
    term = mfma_term_bound(xr, yr, ny, s, lam[t + 1], [nu, th], kp, kstep)
    logz_tol = term + (m / 256 + 6) * U32
    col_tol = logz_tol + term + (n / 256 + 6) * U32
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam[t])
    _say("case", form, shape, f"per-term bound {term:.2e}")
    res, tr = P.step(prob, P.make_params(eta=wl.eta, precision=form), st, trace=True)
    torch.cuda.synchronize()
    cols = np.arange(m)
    ref = RP.step_sampled(RP.Cost(s, 1.0, gram=(xr, yr, nx, ny)), wl.r, wl.c, lam[t], nu, th,
                          OL.Params(eta=wl.eta), 1.0, cols)
    _full_parity(f"{form} {n}x{m}", st, tr, ref, cols, wl.c, 0.01, logz_tol, col_tol, 0.5 / lam[t + 1])
