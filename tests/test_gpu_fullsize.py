"""Full-size GPU checks in the launch configuration the benchmark times.

At n = m = 2^16 (d = 64) and n = m = 2^18 (d = 3) the oracle cannot run whole
iterations, so one GPU iteration from a seeded synthetic state is checked on
sampled rows the oracle computes one by one (row log-normalisers, gradient
rows), and on properties that hold at any size (each column marginal sums to
sum(r) = 1, duals stay in (-1, 1)).  The cost normalisation comes from
tests/golden/cost_scales.json, written by the oracle's exact C routine.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from oracle import stream as OS
from paper_2511_11359_amd import workloads as W
from tests.gpu_util import rel_inf, round_to_type, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cost_scales.json")))
SAMPLE = np.array([0, 1, 31, 32, 4095, 12345, 33333, 65535])


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _synthetic_state(wl, t, seed):
    nu, th = W.synthetic_duals(wl.m, seed)
    lam = OL.inv_eta_schedule(t + 1, 1.0 / 2.0, wl.eta)
    return nu, th, lam[t], lam[t + 1]


def _check_step(wl, key, precision, t, rows, logz_atol, rounded=None, with_trace=False):
    s = GOLD[key]["cost_scale"]
    nu, th, lam_t, lam_t1 = _synthetic_state(wl, t, seed=77)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), t, lam_t)
    _say("case", key, precision, "t", t, "lam", lam_t)
    res, tr = P.step(prob, P.make_params(eta=wl.eta, precision=precision), st, trace=True)
    x = wl.x.astype(np.float64) if rounded is None else rounded[0]
    y = wl.y.astype(np.float64) if rounded is None else rounded[1]
    w = 1.0 / 2.0 / lam_t1                                  # tau1 * eta_{t+1}
    nubar = nu + w * (th - nu)
    la = OS.row_log_normalisers(x, y, s, 1.0, nu, lam_t, rows)
    lb = OS.row_log_normalisers(x, y, s, 1.0, nubar, lam_t1, rows)
    ea = np.max(np.abs(to_np(tr["log_za"])[rows] - la))
    eb = np.max(np.abs(to_np(tr["log_zb"])[rows] - lb))
    ca, cb = to_np(tr["col_a"]), to_np(tr["col_b"])
    _say(key, precision, f"logZA err {ea:.2e} logZB err {eb:.2e} sum colA-1 {ca.sum() - 1:.2e} "
                         f"sum colB-1 {cb.sum() - 1:.2e} res {res:.3e}")
    assert ea <= logz_atol and eb <= logz_atol
    assert abs(ca.sum() - 1.0) <= 1e-6 and abs(cb.sum() - 1.0) <= 1e-6
    # marginals are non-negative; a column whose every term lies below FP32's range reads 0
    assert np.all(ca >= 0) and np.all(cb >= 0)
    assert np.all(np.abs(to_np(st.theta)) < 1) and np.all(np.abs(to_np(st.nu)) < 1)
    return (prob, st, tr) if with_trace else (prob, st)


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
    """2^18 x 2^18, d = 3: one FP32-form iteration at t = 400, sampled rows; then the adjoint
    at the resulting state: 16 random gradient coordinates against the oracle's per-row
    envelope gradient and against central finite differences of the row term (h = 1e-4)."""
    key = "sphere_cube_262144"
    wl = W.sphere_cube()
    rows = np.array([0, 1, 63, 64, 100000, 200001, 262143])
    prob, st = _check_step(wl, key, "fp32", 400, rows, 2e-6)
    s = GOLD[key]["cost_scale"]
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
    """2^16 x 2^16, d = 64: one FP32-form (FP64 argument) iteration at t = 300, sampled rows;
    the certificate of the iterate the step started from."""
    wl = W.gmm64()
    prob, st, tr = _check_step(wl, "gmm64d_65536", "fp32", 300, SAMPLE, 2e-6, with_trace=True)
    nu, th, lam_t, _ = _synthetic_state(wl, 300, seed=77)
    _check_certificate(prob, P.make_params(eta=wl.eta), nu, th, 300, lam_t, to_np(tr["col_a"]), wl.c)


@pytest.mark.parametrize("form,dtype", [("bf16_mfma", torch.bfloat16), ("fp16_mfma", torch.float16),
                                        ("fp32_mfma", torch.float32)])
def test_gmm64_65536_mfma_step(form, dtype):
    """2^16 x 2^16, d = 64: one matrix-core iteration at t = 300, sampled rows against the
    oracle evaluated on the rounded operands the form uses (exponent assembled in FP32)."""
    wl = W.gmm64()
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    mu = 0.5 * (x[0] + y[0])
    xc, yc = x - mu, y - mu
    xr = round_to_type(xc, str(dtype).replace("torch.", ""))
    yr = round_to_type(yc, str(dtype).replace("torch.", ""))
    # the rounded dot products with the unrounded norms are the cost of points whose
    # difference form reproduces them: feed the oracle the exact cost through an offset
    # representation, C_ij = s (|xc_i|^2 + |yc_j|^2 - 2 xr_i . yr_j)
    s = GOLD["gmm64d_65536"]["cost_scale"]
    nu, th, lam_t, lam_t1 = _synthetic_state(wl, 300, seed=77)
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
    st = P.State(torch.tensor(nu, device="cuda"), torch.tensor(th, device="cuda"), 300, lam_t)
    res, tr = P.step(prob, P.make_params(eta=wl.eta, precision=form), st, trace=True)
    nx = np.sum(xc * xc, axis=1)
    ny = np.sum(yc * yc, axis=1)
    w = 0.5 / lam_t1
    nubar = nu + w * (th - nu)
    errs = []
    for i in SAMPLE:
        Ci = s * (nx[i] + ny - 2.0 * yr @ xr[i])
        la = np.logaddexp.reduce(-lam_t * (Ci + 2.0 * nu))
        lb = np.logaddexp.reduce(-lam_t1 * (Ci + 2.0 * nubar))
        errs.append(max(abs(to_np(tr["log_za"])[i] - la), abs(to_np(tr["log_zb"])[i] - lb)))
    ca = to_np(tr["col_a"])
    _say(form, "max logZ err on sampled rows", max(errs), "sum colA - 1", ca.sum() - 1)
    # FP32 exponent assembly: |e| carries ~ c * 2^-24 * (|h| + |x.y|) + ulp(g)/2; at lam ~ 150,
    # c ~ 0.37 and |h|, |x.y| ~ 1e3 this is ~1e-4 per term
    assert max(errs) <= 2e-3
    assert abs(ca.sum() - 1.0) <= 1e-5


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
