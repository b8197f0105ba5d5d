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
