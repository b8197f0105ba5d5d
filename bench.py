"""Benchmark of the LAMP iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision P]
                    [--compare FORMS] [--time-to-tol FORMS] [--no-cpu] [--metric sqeuclid|l1|linf]
                    [--track-dt] [--mode batch|grad|cost|peak]

A step is one LAMP iteration t -> t+1 (Algorithm 2: both marginal sweeps of
Section 4.1, the dual mirror steps, averaging, clipping and the residual) over
the whole problem.  One iteration evaluates 4 n m coupling entries (two row
log-sum-exp sweeps and two column sums): the pair-eval count.  The timed
region is one lamp_solve call that runs exactly K iterations from a warmed-up
state, inputs resident in HBM.

The default workload is n = m = 2^16 points in d = 64 (8-component Gaussian
mixture), eta = 1e-3, in the BF16 matrix-core form; the other forms of the same
workload (FP32 matrix-core tiles, and the reference-accuracy form with FP64 dot
products) are measured beside it, and the BF16 and reference-accuracy forms are
each solved from the start to ||col(X^t) - c||_1 <= 1e-4 (time to tolerance).
`roofline.traffic` is the HBM bytes per launch of the dominant kernel from the
committed counter summaries under profiles/, when they match the current kernel
sources.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures: 256 CUs at 2.4 GHz, 4 SIMD16 per CU.  v_exp_f32 issues at half
# the full VALU rate on CDNA4 (32 lanes per clock per CU).  Dense matrix peaks: FP64 78.6,
# FP32 157.3, BF16/FP16 2500 TFLOP/s.
CUS, CLOCK = 256, 2.4e9
EXP_PEAK = CUS * 32 * CLOCK          # 1.966e13 exp/s
HBM_PEAK = 8.0e12                    # bytes/s, HBM3E
MFMA_PEAK = {"fp32": 78.6e12, "fp32_mfma": 157.3e12, "bf16_mfma": 2500e12, "fp16_mfma": 2500e12}
FORM_DTYPE = {"fp32": "f64/f32", "fp32_mfma": "f32", "bf16_mfma": "bf16/f32", "fp16_mfma": "f16/f32",
              "fp16x3_mfma": "f16x3/f32"}
FORM_DESC = {
    "fp32": "x.y and exponent arguments in FP64, exponentials and sums FP32, duals FP64",
    "fp32_mfma": "x.y tiles on FP32 matrix cores, exponent assembled in FP32, duals FP64",
    "bf16_mfma": "x.y tiles from BF16 points on matrix cores (FP32 accumulate), FP32 exponent "
                 "and sums, FP64 duals",
    "fp16_mfma": "x.y tiles from FP16 points on matrix cores (FP32 accumulate), FP32 exponent "
                 "and sums, FP64 duals",
    "fp16x3_mfma": "x.y as x_hi.y_hi + x_hi.y_lo + x_lo.y_hi from split FP16 points on matrix cores "
                   "(FP32 accumulate), FP32 exponent and sums, FP64 duals",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(wl, s, seconds_target: float = 12.0):
    """The FP64 oracle timed on a bounded sample of rows of the same workload (row log-sum-exp over
    all m columns and the rows' column terms: one marginal pass), pair-evals counted like the
    GPU's.  Main figure: the oracle's C pass (oracle/rowpass.c) on every host core it gets;
    beside it the NumPy row-block form on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import rowpass as RP
    from oracle import stream as OS
    nu = np.zeros(wl.m)
    cols = np.arange(wl.m)
    rows = 16
    while True:
        cost = RP.Cost(s, 1.0, x=wl.x[:rows], y=wl.y)
        t0 = time.perf_counter()
        L = cost.log_normalisers([nu], [10.0])
        cost.sampled_columns([nu], [10.0], L, wl.r[:rows], cols)
        dt_c = time.perf_counter() - t0
        if dt_c >= seconds_target / 3 or rows >= wl.n:
            break
        rows = min(wl.n, rows * 4)
    threads = RP.num_threads()
    allcore = 2.0 * rows * wl.m / dt_c
    # NumPy form on one thread (the BLAS pool limited to one)
    x = wl.x.astype(np.float64)
    y = wl.y.astype(np.float64)
    nrows = 0
    block = 4 if wl.d > 16 else 16
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds_target / 2 and nrows < wl.n:
            idx = np.arange(nrows, min(wl.n, nrows + block))
            OS.marginal_pass(x, y, wl.r, s, 1.0, nu, 10.0, rows=idx, block=block)
            nrows += len(idx)
        dt_n = time.perf_counter() - t0
    single = 2.0 * nrows * wl.m / dt_n
    log(f"cpu oracle: C pass {allcore:.3e} pair-evals/s on {threads} threads ({rows} rows, {dt_c:.1f} s); "
        f"NumPy {single:.3e} on 1 thread ({nrows} rows, {dt_n:.1f} s); host cpus {os.cpu_count()}")
    return {"value": allcore, "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"one marginal pass (row LSE + column terms) over {rows} of {wl.n} rows x {wl.m} columns, "
                      f"d={wl.d}, FP64, the oracle's C pass (oracle/rowpass.c) on {threads} OpenMP threads, "
                      f"{dt_c:.1f} s",
            "host_cpus": os.cpu_count(),
            "numpy_single_thread": {"value": single, "cores": 1,
                                    "sample": f"{nrows} rows, oracle/stream.py row blocks, {dt_n:.1f} s"}}


def measure_form(P, prob, wl, form, steps, warmup, reps, track_dt=False):
    """Throughput of `steps` iterations of one precision form, and its sweep kernel times.
    track_dt: the iterations also accumulate the D_t summands (FP32 form)."""
    import torch
    dev = prob.device
    st = P.State.fresh(wl.m, dev)
    if warmup:
        st, _, _ = P.solve(prob, P.make_params(eta=wl.eta, max_iter=warmup, check_every=max(1, warmup // 2),
                                               precision=form, track_dt=track_dt), st)
    params = P.make_params(eta=wl.eta, tol=0.0, max_iter=steps, check_every=max(1, steps // 2),
                           precision=form, track_dt=track_dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep, _ = P.solve(prob, params, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert rep["iters"] == steps, rep
    row_ms, col_ms = P.sweep_times(prob, params, st, reps=reps)
    log(f"{form}{' (D_t tracked)' if track_dt else ''}: {steps} iterations in {dt:.3f} s "
        f"({dt * 1e3 / steps:.3f} ms/iteration), row sweep {row_ms:.3f} ms, column sweep {col_ms:.3f} ms, "
        f"residual {rep['final_res']:.3e}")
    return {"pair_evals_per_s": 4.0 * wl.n * wl.m * steps / dt, "ms_per_step": dt * 1e3 / steps,
            "row_sweep_ms": row_ms, "col_sweep_ms": col_ms, "residual_after": rep["final_res"],
            "t_after": st.t}


def kernel_sources_sha256():
    """SHA-256 of the kernel headers' code: comments, blank lines and trailing blanks removed,
    so that a counter summary stays valid across edits that change no kernel."""
    h = hashlib.sha256()
    for f in ("lamp_mfma.hpp", "lamp_kernels.hpp", "lamp_cost.hpp"):
        with open(os.path.join(ROOT, "paper_2511_11359_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(workload, form, kernel):
    """HBM bytes per launch from the committed counter summaries (profiles/*.md lines
    'traffic workload=... form=... kernel=... bytes=... kernel_sources_sha256=...'), or None
    when no summary covers this kernel or the kernel sources changed since it was taken."""
    want = {"workload": workload, "form": form, "kernel": kernel,
            "kernel_sources_sha256": kernel_sources_sha256()}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic "):
                    continue
                kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
                if all(kv.get(k) == v for k, v in want.items()):
                    return int(kv["bytes"])
    return None


def roofline(wl, form, m, probe=None):
    """Roofline of the slower sweep kernel of a form: the exponential (VALU) bound for the
    vector-ALU and half-precision forms, the matrix-core bound where the dot products dominate."""
    dom_name, dom_ms = ("row_sweep", m["row_sweep_ms"])
    if m["col_sweep_ms"] > dom_ms:
        dom_name, dom_ms = ("col_sweep", m["col_sweep_ms"])
    mfma_bound = (form == "fp32" and wl.d > 16) or form == "fp32_mfma"
    if mfma_bound:
        flops = 2.0 * wl.n * wl.m * wl.d          # one d-dimensional dot product per pair
        ach = flops / (dom_ms * 1e-3)
        return {"bound": "mfma", "kernel": dom_name, "achieved": ach / 1e12,
                "peak": MFMA_PEAK[form] / 1e12, "unit": "TFLOP/s", "frac": ach / MFMA_PEAK[form],
                "traffic": measured_traffic(wl.name, form, dom_name), "per_launch": f"2*n*m*d = {flops:.3e} flop",
                "row_sweep_ms": m["row_sweep_ms"], "col_sweep_ms": m["col_sweep_ms"]}
    exps = 2.0 * wl.n * wl.m                      # both couplings, one exponential per pair each
    ach = exps / (dom_ms * 1e-3)
    out = {"bound": "alu", "kernel": dom_name, "achieved": ach / 1e12, "peak": EXP_PEAK / 1e12,
           "unit": "Texp/s", "frac": ach / EXP_PEAK, "traffic": measured_traffic(wl.name, form, dom_name),
           "per_launch": f"2*n*m = {exps:.3e} exponentials",
           "row_sweep_ms": m["row_sweep_ms"], "col_sweep_ms": m["col_sweep_ms"]}
    if probe:
        out["probe_exp_per_s"] = probe
        out["frac_of_probe"] = ach / probe
    return out


def fresh_problem(P, wl, dev, metric="sqeuclid"):
    """The workload's problem with the cost scale left to the solve (cost_scale = 0): a timed
    solve then includes the device pass that computes the largest ground cost."""
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, device=dev, metric=metric)
    return prob


def time_to_tol(P, prob, wl, form, tol, max_iter, start=None):
    """Wall time of lamp_solve from `start` (default: the beginning, the cost-scale pass included
    when prob.cost_scale is 0) until ||col(X^t) - c||_1 <= tol, then the certificate of the
    returned iterate on the exact cost (row and column residuals, <C, X^t>, D(theta), D(nu), gap)."""
    import torch
    params = P.make_params(eta=wl.eta, tol=tol, max_iter=max_iter, check_every=64, precision=form)
    prob.workspace(params)                       # allocate outside the timed region
    st0 = start.clone() if start is not None else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep, status = P.solve(prob, params, st0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    cert = P.certificate(prob, P.make_params(eta=wl.eta, precision=form), st)
    dt_cert = time.perf_counter() - t1
    log(f"{form}: time to ||col - c||_1 <= {tol}: {rep['iters']} iterations, {dt:.2f} s, "
        f"converged={rep['converged']}, final residual {rep['final_res']:.3e}; certificate on the exact "
        f"cost: col_res {cert['col_res']:.3e} row_res {cert['row_res']:.3e} cost {cert['cost']:.9e} "
        f"D(theta) {cert['dual_theta']:.6e} D(nu) {cert['dual_nu']:.6e} gap {cert['gap']:.4e} ({dt_cert:.2f} s)")
    out = {"tol": tol, "iters": rep["iters"], "t": st.t, "seconds": dt, "converged": bool(rep["converged"]),
           "final_res": rep["final_res"], "cost_scale_in_timing": prob.cost_scale <= 0,
           "cert": {k: cert[k] for k in ("col_res", "row_res", "cost", "dual_theta", "dual_nu",
                                         "primal_penalized", "gap", "rounded_cost", "prop_bound")},
           "cert_seconds": dt_cert}
    return out, st


def polish(P, prob, wl, st, tol, max_iter):
    """The FP32 reference form resumed from a matrix-core form's iterate until its own residual
    (exact cost) meets tol: the certified-gap comparison of the precision forms."""
    out, st2 = time_to_tol(P, prob, wl, "fp32", tol, max_iter, start=st)
    return out, st2


def batch_mode(args):
    """The 64-problem batch (n, m log-uniform in [512, 8192], d in {2, 3, 16}): batched solve to
    the tolerance against the same problems solved one after another."""
    import torch

    import paper_2511_11359_amd as P
    from paper_2511_11359_amd import workloads as W
    dev = torch.device("cuda:0")
    wls = [W.batch_problem(p) for p in range(args.batch_count)]
    probs = [P.Problem(w.x, w.y, w.r, w.c, device=dev) for w in wls]
    pairs = sum(w.n * w.m for w in wls)
    params = P.make_params(eta=1e-3, tol=args.tol, max_iter=args.max_iter, check_every=32)
    P.solve_batched(probs, P.make_params(eta=1e-3, max_iter=4, check_every=2))   # tune + warm up
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()                                 # the batched solve runs on torch's current stream
    states, reps, status = P.solve_batched(probs, params)
    ev1.record()
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    dev_s = ev0.elapsed_time(ev1) * 1e-3
    iters = [r["iters"] for r in reps]
    evals_b = sum(4.0 * w.n * w.m * r["iters"] for w, r in zip(wls, reps))
    ach = evals_b / dev_s                        # one exponential per pair-eval
    log(f"batched: {args.batch_count} problems, {dt_b:.3f} s, iterations min/max "
        f"{min(iters)}/{max(iters)}, converged {sum(r['converged'] for r in reps)}")
    t0 = time.perf_counter()
    seq = []
    for prob in probs:
        _, rep, _ = P.solve(prob, params)
        seq.append(rep)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    log(f"sequential: {dt_s:.3f} s")
    out = {"metric": "pair-evals/s", "value": evals_b / dt_b, "unit": "pair-evals/s", "n_gpus": 1,
           "steps": max(iters), "warmup": 4, "ms_per_step": dt_b * 1e3 / max(1, max(iters)),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32",
           "data": "synthetic",
           "config": {"workload": f"batch{args.batch_count}", "pairs_per_iteration": 4 * pairs,
                      "eta": 1e-3, "tol": args.tol, "form": "fp32"},
           "roofline": {"bound": "alu", "kernel": "batched iterations (row and column sweeps of all problems, "
                                                   "row finish, dual update; graph replays)",
                        "achieved": ach / 1e12, "peak": EXP_PEAK / 1e12, "unit": "Texp/s", "frac": ach / EXP_PEAK,
                        "traffic": None, "per_launch": "4 n_p m_p exponentials per problem iteration",
                        "device_seconds": dev_s},
           "batched_seconds": dt_b, "sequential_seconds": dt_s,
           "converged": int(sum(r["converged"] for r in reps)),
           "iterations": {"min": min(iters), "max": max(iters)}}
    print(json.dumps(out), flush=True)


def grad_mode(args):
    """The differentiation workload: n = m = 2^18, d = 3 (sphere vs cube), BF16-MFMA forward
    from the start to ||col(X^t) - c||_1 <= tol, then the FP32 adjoint (envelope gradient
    with respect to x) at the final state.  Reports both times and the adjoint's rate."""
    import torch

    import paper_2511_11359_amd as P
    from paper_2511_11359_amd import workloads as W
    wl = W.sphere_cube()
    dev = torch.device("cuda:0")
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, device=dev)
    s, _ = P.cost_scale(prob)
    prob.cost_scale, prob.cost_norm = s, 1.0
    fwd, st = time_to_tol(P, prob, wl, "bf16_mfma", args.tol, args.max_iter)
    params = P.make_params(eta=wl.eta)
    P.backward(prob, params, st)                 # warm-up (workspace, code paths)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 10)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()                                 # the library launches on torch's current stream
    for _ in range(reps):
        g = P.backward(prob, params, st)
    ev1.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    dev_ms = ev0.elapsed_time(ev1) / reps
    pairs = float(wl.n) * wl.m
    ach = pairs / (dev_ms * 1e-3)
    log(f"adjoint: {dt * 1e3:.3f} ms per gradient (device {dev_ms:.3f} ms, {ach:.3e} exp/s), "
        f"|g|_max {float(g.abs().max()):.3e}")
    # the gradient with respect to y (column side)
    P.backward_y(prob, params, st)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        gy = P.backward_y(prob, params, st)
    ev1.record()
    torch.cuda.synchronize()
    dev_ms_y = ev0.elapsed_time(ev1) / reps
    log(f"adjoint with respect to y: {dev_ms_y:.3f} ms per gradient (device, {2.0 * pairs / (dev_ms_y * 1e-3):.3e} "
        f"exp/s: a row-sum pass and a column pass, one exponential per pair each), "
        f"|g|_max {float(gy.abs().max()):.3e}")
    # the autograd forward's value: <C, X^t> in one pass (lamp_transport_cost)
    cost = P.transport_cost(prob, params, st)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        cost = P.transport_cost(prob, params, st)
    ev1.record()
    torch.cuda.synchronize()
    cost_ms = ev0.elapsed_time(ev1) / reps
    log(f"transport cost: {cost_ms:.3f} ms per call (device), <C, X> = {float(cost):.9e}")
    out = {"metric": "pair-evals/s", "value": pairs / dt, "unit": "pair-evals/s", "n_gpus": 1,
           "steps": reps, "warmup": 1, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
           "config": {"workload": wl.name + "_gradient", "n": wl.n, "m": wl.m, "d": wl.d,
                      "eta": wl.eta, "forward": "bf16_mfma", "adjoint": "fp32"},
           "roofline": {"bound": "alu", "kernel": "adjoint (backward call: column term, adjoint sweep, finish)",
                        "achieved": ach / 1e12, "peak": EXP_PEAK / 1e12, "unit": "Texp/s",
                        "frac": ach / EXP_PEAK, "traffic": None,
                        "per_launch": f"n*m = {pairs:.3e} exponentials", "device_ms": dev_ms},
           "forward_time_to_tol": fwd, "adjoint_ms": dt * 1e3, "adjoint_y_ms": dev_ms_y,
           "transport_cost_ms": cost_ms}
    print(json.dumps(out), flush=True)


def calibration_copy(mib, dev):
    """One device copy of `mib` MiB (bytes known exactly), the reference the HBM counters of
    a profiled run are scaled by."""
    if not mib:
        return
    import torch
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cost_mode(args):
    """Explicit-cost input at n = m = 2^16: transport between two random 256 x 256 images over
    the squared Euclidean grid cost, a 16 GiB FP32 matrix built on the device (the image
    benchmarks of Section 5 use explicit grid costs, at up to 64 x 64 pixels).  Both sweeps
    stream the matrix once per launch, so the roofline is HBM bandwidth at 4 bytes per pair (2
    with --cost-dtype bfloat16, the matrix rounded once); time to the tolerance is capped at
    --cost-max-iter iterations."""
    import types

    import torch

    import paper_2511_11359_amd as P
    from paper_2511_11359_amd import workloads as W
    dev = torch.device("cuda:0")
    calibration_copy(args.calib_copy_mib, dev)
    cw = W.image_pair_device(256, "sqeuclid", device=dev)
    cost = cw.cost if args.cost_dtype == "float32" else cw.cost.to(torch.bfloat16)
    prob = P.Problem.from_cost(cost, cw.r, cw.c, device=dev)
    s, cmax = P.cost_scale(prob)
    prob.cost_scale, prob.cost_norm = s, 1.0
    esize = cost.element_size()
    name = cw.name if args.cost_dtype == "float32" else cw.name + "_bf16"
    wl = types.SimpleNamespace(name=name, n=prob.n, m=prob.m, d=1, eta=cw.eta)
    log(f"{wl.name}: n=m={wl.n}, max cost {cmax:g}, s={s:.9e}")
    mm = measure_form(P, prob, wl, "fp32", args.steps, args.warmup, args.reps)
    dom_name, dom_ms = ("row_sweep", mm["row_sweep_ms"])
    if mm["col_sweep_ms"] > dom_ms:
        dom_name, dom_ms = ("col_sweep", mm["col_sweep_ms"])
    nbytes = float(esize) * wl.n * wl.m
    ach = nbytes / (dom_ms * 1e-3) / 1e9
    ttt = time_to_tol(P, prob, wl, "fp32", args.tol, args.cost_max_iter)[0] if args.cost_max_iter > 0 else None
    out = {"metric": "pair-evals/s", "value": mm["pair_evals_per_s"], "unit": "pair-evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": mm["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32",
           "data": "synthetic",
           "config": {"workload": wl.name, "n": wl.n, "m": wl.m, "input": "explicit cost matrix",
                      "cost_dtype": args.cost_dtype, "eta": wl.eta, "form": "fp32"},
           "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": ach, "peak": HBM_PEAK / 1e9,
                        "unit": "GB/s", "frac": ach * 1e9 / HBM_PEAK,
                        "traffic": measured_traffic(wl.name, "fp32", dom_name),
                        "per_launch": f"{esize}*n*m = {nbytes:.3e} bytes",
                        "row_sweep_ms": mm["row_sweep_ms"], "col_sweep_ms": mm["col_sweep_ms"]},
           "time_to_tol": {"fp32": ttt}}
    print(json.dumps(out), flush=True)


def peak_mode(args):
    """The exponential probe alone (lamp_exp_rate): issue rate of the base-2 exponential at a few
    launch sizes, against the derived 256 CUs x 32 lanes per clock x 2.4 GHz."""
    import torch

    import paper_2511_11359_amd as P
    dev = torch.device("cuda:0")
    rates = {}
    for blocks in (1024, 2048, 4096, 8192, 16384):
        rates[blocks] = P.exp_rate(dev, blocks=blocks, iters=4096, reps=args.reps)
        log(f"probe {blocks} blocks x 256 threads: {rates[blocks]:.4e} exp/s ({rates[blocks] / EXP_PEAK:.3f})")
    best = max(rates.values())
    out = {"metric": "exp/s", "value": best, "unit": "exp/s", "n_gpus": 1, "steps": args.reps, "warmup": 1,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": "exp_probe", "chains": 8, "iters": 4096},
           "derived_peak": EXP_PEAK, "frac_of_derived": best / EXP_PEAK,
           "by_blocks": {str(k): v for k, v in rates.items()}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="single", choices=["single", "batch", "grad", "cost", "peak"])
    ap.add_argument("--cost-dtype", default="float32", choices=["float32", "bfloat16"],
                    help="element type of the explicit cost matrix in --mode cost")
    ap.add_argument("--cost-max-iter", type=int, default=3000,
                    help="iteration cap of the time to tolerance in --mode cost (0: skip it)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="gmm64d_65536")
    ap.add_argument("--metric", default="sqeuclid", choices=["sqeuclid", "l1", "linf"],
                    help="ground cost generated from the points (l1 / linf: FP32 form only)")
    ap.add_argument("--track-dt", action="store_true",
                    help="also time the primary form with D_t tracking (FP32 form)")
    ap.add_argument("--precision", default="bf16_mfma",
                    choices=["fp32", "fp32_mfma", "bf16_mfma", "fp16_mfma", "fp16x3_mfma"])
    ap.add_argument("--compare", default="fp16x3_mfma,fp32_mfma,fp32",
                    help="other forms measured beside the primary one (comma list, '' for none)")
    ap.add_argument("--compare-steps", type=int, default=10)
    ap.add_argument("--time-to-tol", default="bf16_mfma,fp16_mfma,fp16x3_mfma,fp32_mfma,fp32",
                    help="forms solved from the start to the tolerance (comma list, '' for none)")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--polish", default="bf16_mfma",
                    help="matrix-core forms whose time to tolerance is followed by an FP32-form polish "
                         "to the same tolerance on the exact cost (comma list, '' for none)")
    ap.add_argument("--reps", type=int, default=5, help="launches per kernel for the roofline timing")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "DESIGN.md describes how the path would shard", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        batch_mode(args)
        return
    if args.mode == "grad":
        grad_mode(args)
        return
    if args.mode == "cost":
        cost_mode(args)
        return
    if args.mode == "peak":
        peak_mode(args)
        return

    import torch

    import paper_2511_11359_amd as P
    from paper_2511_11359_amd import workloads as W

    wl = W.WORKLOADS[args.workload]()
    dev = torch.device("cuda:0")
    calibration_copy(args.calib_copy_mib, dev)
    if args.metric != "sqeuclid":
        if args.precision != "fp32":
            print("bench.py: the l1 / linf costs run in the FP32 form only (--precision fp32)", file=sys.stderr)
            sys.exit(2)
        wl.name = f"{wl.name}_{args.metric}"
    prob = P.Problem(wl.x, wl.y, wl.r, wl.c, device=dev, metric=args.metric)   # cost scale on the device
    s, _ = P.cost_scale(prob)
    prob.cost_scale, prob.cost_norm = s, 1.0
    log(f"{wl.name}: n={wl.n} m={wl.m} d={wl.d} eta={wl.eta} metric={args.metric} s={s:.9e}")

    main_m = measure_form(P, prob, wl, args.precision, args.steps, args.warmup, args.reps)
    dt_track = None
    if args.track_dt:
        tr = measure_form(P, prob, wl, args.precision, args.steps, args.warmup, args.reps, track_dt=True)
        dt_track = {"ms_per_step": tr["ms_per_step"], "overhead_ms": tr["ms_per_step"] - main_m["ms_per_step"]}
        log(f"D_t tracking: {tr['ms_per_step']:.3f} ms per iteration, "
            f"{dt_track['overhead_ms']:.3f} ms more than untracked")
    others = {}
    for form in [f for f in args.compare.split(",") if f and f != args.precision]:
        others[form] = measure_form(P, prob, wl, form, args.compare_steps, 2, max(2, args.reps // 2))
        others[form]["roofline"] = roofline(wl, form, others[form])
    ttt = None
    forms_ttt = [f for f in args.time_to_tol.split(",") if f]
    if forms_ttt:
        ttt = {}
        for f in forms_ttt:
            prob_f = fresh_problem(P, wl, dev, args.metric)
            res, st_f = time_to_tol(P, prob_f, wl, f, args.tol, args.max_iter)
            if f != "fp32" and f in args.polish.split(","):
                pol, _ = polish(P, prob_f, wl, st_f, args.tol, args.max_iter)
                res["fp32_polish"] = pol
                res["seconds_with_polish"] = res["seconds"] + pol["seconds"]
            ttt[f] = res
    cpu = None if (args.no_cpu or args.metric != "sqeuclid") else cpu_baseline(wl, s)   # C pass: squared Euclidean
    probe = P.exp_rate(dev)
    log(f"exponential probe: {probe:.4e} exp/s ({probe / EXP_PEAK:.3f} of the derived {EXP_PEAK:.4e})")

    out = {
        "metric": "pair-evals/s",
        "value": main_m["pair_evals_per_s"],
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORM_DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "m": wl.m, "d": wl.d, "eta": wl.eta, "metric": args.metric,
                   "form": args.precision, "precision": FORM_DESC[args.precision]},
        "roofline": roofline(wl, args.precision, main_m, probe),
        "cpu_baseline": cpu,
        "forms": others,
        "time_to_tol": ttt,
    }
    if dt_track is not None:
        out["dt_tracking"] = dt_track
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
