"""Helpers shared by the GPU tests: build problems from workloads, run the oracle
on the same inputs, compare with the tolerances derived in the design doc."""
from __future__ import annotations

import numpy as np

from oracle import lamp as OL


def oracle_problem(wl):
    """FP64 copy of the FP32 points, the cost scale s = 1/max ||x - y||^2 and C (dense)."""
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    s = 1.0 / OL.max_sqdist(x, y)
    C = OL.sqeuclid_cost(x, y, s)
    return x, y, s, C


def gpu_problem(wl, s):
    import paper_2511_11359_amd as P
    return P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)


def rel_inf(a, ref, floor=0.0):
    """Norm-wise relative error ||a - ref||_inf / max(||ref||_inf, floor)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = max(float(np.max(np.abs(ref))), floor)
    num = np.max(np.abs(a - ref))
    return num / den if den > 0 else num


# Duals live in [-1, 1] (theta is clipped to the radius tanh(beta/2) = 0.50052).  Their FP32
# error is absolute (~1e-7: kappa (col_j error)/c^alpha_j with col_j carrying the ~1e-7
# relative error of FP32 exponentials), so "relative" is taken against the larger of the
# reference's norm and the clip radius.
DUAL_SCALE = 0.5


def rel_dual(a, ref):
    return rel_inf(a, ref, DUAL_SCALE)


def rel_l1(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(a - ref).sum() / np.abs(ref).sum()


def to_np(t):
    return t.detach().cpu().numpy()


# (significant bits, smallest normal exponent) of the operand types of the matrix-core forms
_FORMATS = {"float32": (24, -126), "bfloat16": (8, -126), "float16": (11, -14)}


def round_to_type(a, name):
    """Round FP64 values once, to nearest with ties to even, onto the grid of the named
    binary format (subnormals included): the rounding the library applies to each centred
    coordinate when it writes the matrix-core operands.  Written out from the definition of
    the format (p significant bits, exponent floor emin): the quantum of |a| in
    [2^e, 2^(e+1)) is 2^(max(e, emin) - p + 1), and a / quantum is exact in FP64."""
    p, emin = _FORMATS[name]
    a = np.asarray(a, dtype=np.float64)
    _, e = np.frexp(a)                      # a = f 2^e with 1/2 <= |f| < 1
    q = np.ldexp(1.0, np.maximum(e - 1, emin) - (p - 1))
    return np.rint(a / q) * q


def fp32_trajectory_allowance(C, r, c, prm, T, cnorm=1.0, eps=2.0 ** -24, seeds=(0, 1)):
    """How far the oracle's duals after T iterations move when every column marginal it
    computes carries an independent relative perturbation of size eps (half an FP32 ulp,
    the least any FP32 evaluation of the marginals carries).  The dual update adds
    kappa (col - c) / c^alpha to atanh(theta) every iteration, so such errors accumulate
    along a trajectory; a multi-iteration comparison allows for it.  Returns the largest
    rel_dual deviation of theta or nu over the seeded perturbations."""
    ref, _ = OL.lamp_dense(C, r, c, prm, T, cnorm, trace=False)
    orig = OL.col_r
    worst = 0.0
    try:
        for sd in seeds:
            rng = np.random.default_rng(sd)
            OL.col_r = lambda p, rr, rng=rng: orig(p, rr) * (1.0 + eps * rng.standard_normal(p.shape[1]))
            st, _ = OL.lamp_dense(C, r, c, prm, T, cnorm, trace=False)
            OL.col_r = orig
            worst = max(worst, rel_dual(st.theta, ref.theta), rel_dual(st.nu, ref.nu))
    finally:
        OL.col_r = orig
    return worst


U32 = 2.0 ** -24        # unit roundoff of FP32
LOG2E = 1.4426950408889634


def sample_columns(m, seed=11, extra=64):
    """Columns for full-size parity: the ends of 32- and 128-column tiles at both ends of the
    range, around m/2 and 4096, plus `extra` seeded random ones (at least 64 in all)."""
    fixed = [0, 1, 31, 32, 63, 64, 127, 128, 255, 256, 4095, 4096, m // 2 - 1, m // 2,
             m - 129, m - 128, m - 33, m - 32, m - 2, m - 1]
    rng = np.random.default_rng(seed)
    cols = np.concatenate([[j for j in fixed if 0 <= j < m], rng.choice(m, min(extra, m), replace=False)])
    return np.unique(cols)


def mfma_term_bound(xr, yr, yn2, s, lam, duals, kp, kstep, cnorm=1.0, erange=64.0):
    """Worst-case relative error of one exponential term of a matrix-core form, from its FP32
    exponent assembly: the dot product x~_i . y~_j of operands rounded to the form's type is
    accumulated in FP32 onto an offset of magnitude up to Q (kp / kstep matrix instructions, each
    rounding once, plus the offset's own rounding), multiplied by c = 2 s lam log2(e) rounded to
    FP32, and added to a column term of magnitude c Q rounded to FP32 (three such roundings: the
    table entry, its A/B correction and the row term), with a final rounding of the exponent
    itself (|e| <= erange).  Every FP32 rounding moves a value v by at most U32 |v|, so the base-2
    exponent moves by at most
        U32 (c A (kp / kstep + 3) + 3 c Q + erange),   A = Q + 2 max|x~| max|y~|,
    Q = max_j (|y~_j|^2 / 2 + 2 ||C||_inf max|v_j| / (2 s)), and the term by ln 2 times that."""
    X = float(np.max(np.sqrt(np.sum(np.asarray(xr) ** 2, axis=1))))
    Y = float(np.max(np.sqrt(np.sum(np.asarray(yr) ** 2, axis=1))))
    vmax = max(float(np.max(np.abs(v))) for v in duals)
    Q = float(np.max(yn2)) / 2.0 + 2.0 * cnorm * vmax / (2.0 * s)
    A = Q + 2.0 * X * Y
    c = 2.0 * s * lam * LOG2E
    de = U32 * (c * A * (kp // kstep + 3) + 3.0 * c * Q + erange)
    return float(np.log(2.0) * de)


def split_fp16_scale(xc, yc):
    """Range scale of the split FP16 form (a power of two): 2^(7 - e) with 2^e <= max |coordinate|
    < 2^(e+1) over both centred clouds, 1 when every coordinate is zero."""
    mx = max(float(np.max(np.abs(xc))), float(np.max(np.abs(yc))))
    if mx == 0.0:
        return 1.0
    _, e = np.frexp(mx)                      # mx = f 2^e, 1/2 <= f < 1: floor(log2 mx) = e - 1
    return float(np.ldexp(1.0, 7 - (int(e) - 1)))


def split_fp16(v, scale):
    """(hi, lo) of the split FP16 form for FP64 values v: hi = fp16(v scale), lo = fp16(v scale - hi),
    each one rounding to nearest even (the scaled value and the difference are exact in FP64)."""
    vs = np.asarray(v, dtype=np.float64) * scale
    hi = round_to_type(vs, "float16")
    lo = round_to_type(vs - hi, "float16")
    return hi, lo
