"""ctypes loader for oracle/rowpass.c (test infrastructure only; see oracle/__init__).

One LAMP iteration at full size, for sampled parity checks: the C routine evaluates the
row log-normalisers of every row (Section 4.1, first display) and the column marginals
col_r(p^{1/lam}(v)) of listed columns (second display) in FP64; the dual steps of those
columns then follow Algorithm 2 coordinate by coordinate (they only need their own
column's marginal).  ``build()`` compiles the C file with gcc into ``oracle/_rowpass.so``;
the loader compiles it on first use if the library is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .lamp import Params, dual_mirror_map, tclip

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rowpass.c")
_LIB = os.path.join(_HERE, "_rowpass.so")
_lib = None
_vp = ctypes.c_void_p


class _CostDef(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("d", ctypes.c_int32), ("n", ctypes.c_int64),
                ("m", ctypes.c_int64), ("x", _vp), ("y", _vp), ("xr", _vp), ("yr", _vp),
                ("nx", _vp), ("ny", _vp), ("s", ctypes.c_double), ("K", ctypes.c_double)]


def build() -> str:
    subprocess.run(["gcc", "-O3", "-ffast-math", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, _SRC,
                    "-lm"], check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_log_normalisers.restype = None
        lib.oracle_log_normalisers.argtypes = [ctypes.POINTER(_CostDef), ctypes.c_int32, _vp, _vp, _vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_sampled_columns.restype = None
        lib.oracle_sampled_columns.argtypes = [ctypes.POINTER(_CostDef), ctypes.c_int32, _vp, _vp, _vp,
                                               _vp, _vp, ctypes.c_int64, _vp]
        lib.oracle_row_costs.restype = None
        lib.oracle_row_costs.argtypes = [ctypes.POINTER(_CostDef), ctypes.c_int32, _vp, _vp, _vp, _vp]
        _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the C routines run on (OpenMP)."""
    return int(_load().oracle_num_threads())


class Cost:
    """C_ij = s * ||x_i - y_j||^2 from FP32 points (difference form), or, with ``gram``,
    C_ij = s * (nx_i + ny_j - 2 xr_i . yr_j) from FP64 arrays; K = 2 ||C||_inf."""

    def __init__(self, s: float, cnorm: float, x=None, y=None, gram=None):
        self._keep = []
        if gram is None:
            x = np.ascontiguousarray(x, dtype=np.float32)
            y = np.ascontiguousarray(y, dtype=np.float32)
            self.n, self.m, d = x.shape[0], y.shape[0], x.shape[1]
            self._keep += [x, y]
            self.cd = _CostDef(0, d, self.n, self.m, x.ctypes.data, y.ctypes.data, None, None, None,
                               None, s, 2.0 * cnorm)
        else:
            xr, yr, nx, ny = (np.ascontiguousarray(a, dtype=np.float64) for a in gram)
            self.n, self.m, d = xr.shape[0], yr.shape[0], xr.shape[1]
            self._keep += [xr, yr, nx, ny]
            self.cd = _CostDef(1, d, self.n, self.m, None, None, xr.ctypes.data, yr.ctypes.data,
                               nx.ctypes.data, ny.ctypes.data, s, 2.0 * cnorm)

    def log_normalisers(self, duals, lams) -> np.ndarray:
        """log Z^q_i = LSE_j(-lam_q (C_ij + K v_q,j)) for every row i, one row per coupling q."""
        v = np.ascontiguousarray(np.stack(duals), dtype=np.float64)
        lam = np.ascontiguousarray(lams, dtype=np.float64)
        out = np.empty((v.shape[0], self.n))
        _load().oracle_log_normalisers(ctypes.byref(self.cd), v.shape[0], v.ctypes.data, lam.ctypes.data,
                                       out.ctypes.data)
        return out

    def sampled_columns(self, duals, lams, logZ, r, cols) -> np.ndarray:
        """col_r(p^{1/lam_q}(v_q))_j = sum_i r_i exp(-lam_q (C_ij + K v_q,j) - log Z^q_i) for the
        listed columns j, one row per coupling q."""
        v = np.ascontiguousarray(np.stack(duals), dtype=np.float64)
        lam = np.ascontiguousarray(lams, dtype=np.float64)
        lz = np.ascontiguousarray(logZ, dtype=np.float64)
        rr = np.ascontiguousarray(r, dtype=np.float64)
        cj = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty((v.shape[0], cj.shape[0]))
        _load().oracle_sampled_columns(ctypes.byref(self.cd), v.shape[0], v.ctypes.data, lam.ctypes.data,
                                       lz.ctypes.data, rr.ctypes.data, cj.ctypes.data, cj.shape[0],
                                       out.ctypes.data)
        return out


    def row_costs(self, duals, lams, logZ) -> np.ndarray:
        """E^q_i = sum_j p^{1/lam_q}(v_q)_ij C_ij for every row i, one row per coupling q, given the
        row log-normalisers; <C, diag(r) p> = r . E."""
        v = np.ascontiguousarray(np.stack(duals), dtype=np.float64)
        lam = np.ascontiguousarray(lams, dtype=np.float64)
        lz = np.ascontiguousarray(logZ, dtype=np.float64)
        out = np.empty((v.shape[0], self.n))
        _load().oracle_row_costs(ctypes.byref(self.cd), v.shape[0], v.ctypes.data, lam.ctypes.data,
                                 lz.ctypes.data, out.ctypes.data)
        return out


def step_sampled(cost: Cost, r, c, lam, nu, theta, prm: Params, cnorm: float, cols):
    """One iteration t -> t+1 of Algorithm 2 from (lam_t, nu^t, theta^t): log Z of both couplings
    on every row, and on the listed columns colA, colB, thetabar, thetahat, nu^{t+1}, theta^{t+1}
    (steps step:eta_update to tclip; the dual steps act coordinate by coordinate).
    Returns a dict of arrays (row quantities over all rows, column quantities over ``cols``)."""
    prm = prm.resolved(cnorm)
    m = c.shape[0]
    cols = np.asarray(cols, dtype=np.int64)
    lam_next = prm.tau1 + lam * (1.0 - prm.tau1 * prm.eta)
    w = prm.tau1 / lam_next
    nubar = nu + w * (theta - nu)
    logZ = cost.log_normalisers([nu, nubar], [lam, lam_next])
    colA, colB = cost.sampled_columns([nu, nubar], [lam, lam_next], logZ, r, cols)
    cJ = c[cols]
    calpha = cJ + prm.alpha / m
    th = theta[cols]
    theta_bar = dual_mirror_map(th, colA, cJ, calpha, prm.tau2, cnorm)
    nu_next = nu[cols] + w * (theta_bar - nu[cols])
    theta_hat = dual_mirror_map(th, colB, cJ, calpha, prm.tau2, cnorm)
    return dict(logZA=logZ[0], logZB=logZ[1], colA=colA, colB=colB, theta_bar=theta_bar,
                theta_hat=theta_hat, nu=nu_next, theta=tclip(theta_hat, prm.beta), lam_next=lam_next)


def solve(cost: Cost, r, c, prm: Params, cnorm: float, T: int, tol: float | None = None, keep=()):
    """Algorithm 2 from its start (theta^0 = nu^0 = 0, eta_0 = infinity) with full steps of
    ``step_sampled`` over every column, for at most T iterations.  Stopping reading as
    ``oracle.lamp.lamp_dense``: before iteration t >= 1 the residual ||col(X^t) - c||_1 is
    measured (the step from t computes col(X^t) as its colA) and, if it is <= tol, the run stops
    with the state holding nu^t.  ``keep``: iterations t whose starting state (lam_t, nu^t,
    theta^t) is returned in ``saved[t]``.  Returns a dict (t, lam, nu, theta, res, saved)."""
    m = c.shape[0]
    cols = np.arange(m)
    t, lam = 0, 0.0
    nu, theta = np.zeros(m), np.zeros(m)
    saved, res = {}, None
    for _ in range(T):
        if t in keep:
            saved[t] = (lam, nu.copy(), theta.copy())
        out = step_sampled(cost, r, c, lam, nu, theta, prm, cnorm, cols)
        res = float(np.abs(out["colA"] - c).sum())
        if tol is not None and t >= 1 and res <= tol:
            break
        t, lam, nu, theta = t + 1, out["lam_next"], out["nu"], out["theta"]
    return dict(t=t, lam=lam, nu=nu, theta=theta, res=res, saved=saved)
