"""Python binding of the LAMP C ABI.  PyTorch provides device memory and the
stream; every step of the method runs in the HIP kernels of liblamp.so, and a
missing library raises (there is no fallback path)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


class LampError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int) -> int:
    if status < 0:
        lib = L.load()
        raise LampError(status, lib.lamp_last_error().decode(errors="replace"))
    return status


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


class Problem:
    """Device-resident problem data (Section 1): x (n x d) and y (m x d) FP32 point clouds,
    r and c FP64 marginals, the ground cost (metric: "sqeuclid", "l1" or "linf"), and the
    workspace the library works in.  Problem.from_cost gives the cost as an n x m matrix
    instead (metric "explicit")."""

    def __init__(self, x, y, r, c, cost_scale: float = 0.0, cost_norm: float = 0.0,
                 device: str | torch.device = "cuda", metric: str = "sqeuclid", cost=None):
        dev = torch.device(device)
        self.device = dev
        self.r = torch.as_tensor(r, dtype=torch.float64).to(dev).contiguous()
        self.c = torch.as_tensor(c, dtype=torch.float64).to(dev).contiguous()
        if metric == "explicit":
            self.x = self.y = None
            cost = torch.as_tensor(cost)
            keep = cost.dtype in (torch.bfloat16, torch.float16)   # 2-byte storage is kept as given
            self.cost = cost.to(dev, dtype=cost.dtype if keep else torch.float32).contiguous()
            assert self.cost.dim() == 2
            self.n, self.m = self.cost.shape
            self.d = 1
        else:
            self.cost = None
            self.x = torch.as_tensor(x, dtype=torch.float32).to(dev).contiguous()
            self.y = torch.as_tensor(y, dtype=torch.float32).to(dev).contiguous()
            assert self.x.dim() == 2 and self.y.dim() == 2 and self.x.shape[1] == self.y.shape[1]
            self.n, self.d = self.x.shape
            self.m = self.y.shape[0]
        self.cost_scale = float(cost_scale)
        self.cost_norm = float(cost_norm)
        self.metric = metric
        self._ws = None

    @classmethod
    def from_cost(cls, cost, r, c, cost_scale: float = 0.0, cost_norm: float = 0.0,
                  device: str | torch.device = "cuda") -> "Problem":
        """C_ij = cost_scale * cost[i, j] from an n x m matrix, row-major: bfloat16 and float16
        matrices are used as given (2 bytes per entry), any other dtype is stored as float32."""
        return cls(None, None, r, c, cost_scale, cost_norm, device, metric="explicit", cost=cost)

    def struct(self) -> L.Problem:
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        cost_type = L.COST_TYPES[str(self.cost.dtype).replace("torch.", "")] if self.cost is not None else 0
        return L.Problem(self.n, self.m, self.d, L.METRICS[self.metric], ptr(self.x), ptr(self.y),
                         self.r.data_ptr(), self.c.data_ptr(), self.cost_scale, self.cost_norm, ptr(self.cost),
                         cost_type, 0)

    def workspace(self, params: L.Params) -> tuple[int, int]:
        lib = L.load()
        prob = self.struct()
        need = int(lib.lamp_workspace_bytes(ctypes.byref(prob), ctypes.byref(params)))
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        return aligned, need


def make_params(eta: float = 0.0, tol: float = 0.0, max_iter: int = 1000, alpha: float = 0.0,
                beta: float = 0.0, tau1: float = 0.0, tau2: float = 0.0,
                check_every: int = 64, precision: str = "fp32", track_dt: bool = False) -> L.Params:
    """Algorithm 2 parameters; zeros select the defaults of Appendix E.  precision is one of
    fp32 (FP64 arguments, FP32 exponentials), fp32_mfma, bf16_mfma, fp16_mfma, fp16x3_mfma.  track_dt
    accumulates the partial sums D_t of Proposition infeas_bound(b) in the state (fp32 only)."""
    return L.Params(eta, tol, int(max_iter), alpha, beta, tau1, tau2, L.PRECISIONS[precision],
                    int(check_every), int(bool(track_dt)), 0)


@dataclass
class State:
    """O(n + m) state: nu^t, theta^t (FP64 device), t, lam_t = 1/eta_t and the D_t summands
    accumulated so far (NaN unless every iteration tracked them)."""
    nu: torch.Tensor
    theta: torch.Tensor
    t: int = 0
    inv_eta: float = 0.0
    dt_partial: float = 0.0

    @staticmethod
    def fresh(m: int, device="cuda") -> "State":
        z = torch.zeros(m, dtype=torch.float64, device=device)
        return State(z, z.clone(), 0, 0.0, 0.0)

    def struct(self) -> L.State:
        return L.State(self.nu.data_ptr(), self.theta.data_ptr(), self.t, self.inv_eta, self.dt_partial)

    def update(self, s: L.State) -> None:
        self.t = int(s.t)
        self.inv_eta = float(s.inv_eta)
        self.dt_partial = float(s.dt_partial)

    def clone(self) -> "State":
        return State(self.nu.clone(), self.theta.clone(), self.t, self.inv_eta, self.dt_partial)


def cost_scale(prob: Problem) -> tuple[float, float]:
    """(s, max_ij ||x_i - y_j||^2) with s = 1/max: the normalisation ||C||_inf = 1."""
    lib = L.load()
    params = make_params()
    ws, nb = prob.workspace(params)
    s = ctypes.c_double()
    md = ctypes.c_double()
    p = prob.struct()
    _check(lib.lamp_cost_scale(ctypes.byref(p), ws, nb, _stream_handle(prob.device), ctypes.byref(s),
                               ctypes.byref(md)))
    return s.value, md.value


def _trace_buffers(prob: Problem, trace: bool):
    if not trace:
        return None, None
    dd = dict(device=prob.device, dtype=torch.float64)
    tr = dict(log_za=torch.empty(prob.n, **dd), log_zb=torch.empty(prob.n, **dd),
              col_a=torch.empty(prob.m, **dd), col_b=torch.empty(prob.m, **dd),
              theta_bar=torch.empty(prob.m, **dd), theta_hat=torch.empty(prob.m, **dd))
    trs = L.Trace(*(tr[k].data_ptr() for k in ["log_za", "log_zb", "col_a", "col_b",
                                                "theta_bar", "theta_hat"]))
    return tr, trs


def step(prob: Problem, params: L.Params, state: State, trace: bool = False):
    """One iteration of Algorithm 2 in place.  Returns (||col(X^t) - c||_1, trace dict or None)."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    tr, trs = _trace_buffers(prob, trace)
    p = prob.struct()
    s = state.struct()
    res = ctypes.c_double()
    _check(lib.lamp_step(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), ws, nb,
                         _stream_handle(prob.device), ctypes.byref(trs) if trs is not None else None,
                         ctypes.byref(res)))
    state.update(s)
    return res.value, tr


def step_noalloc(prob: Problem, params: L.Params, state: State, trace: bool = False):
    """step() through lamp_step_noalloc: the library's fixed device scratch replaces the
    workspace (problems up to LAMP_NOALLOC_WS_BYTES of workspace).  The trace buffers, when asked
    for, are the caller's outputs and are allocated here, before the call."""
    lib = L.load()
    tr, trs = _trace_buffers(prob, trace)
    p = prob.struct()
    s = state.struct()
    res = ctypes.c_double()
    _check(lib.lamp_step_noalloc(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s),
                                 _stream_handle(prob.device),
                                 ctypes.byref(trs) if trs is not None else None, ctypes.byref(res)))
    state.update(s)
    return res.value, tr


def solve(prob: Problem, params: L.Params, state: State | None = None):
    """Runs Algorithm 2 (resuming from `state` if given).  Returns (state, report dict, status)."""
    lib = L.load()
    if state is None:
        state = State.fresh(prob.m, prob.device)
    ws, nb = prob.workspace(params)
    p = prob.struct()
    s = state.struct()
    rep = L.Report()
    st = _check(lib.lamp_solve(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), ws, nb,
                               _stream_handle(prob.device), ctypes.byref(rep)))
    state.update(s)
    report = {k: getattr(rep, k) for k, _ in L.Report._fields_}
    return state, report, st


def certificate(prob: Problem, params: L.Params, state: State) -> dict:
    """Certificate of X^t (Proposition infeas_bound, def:dual_spp)."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    p = prob.struct()
    s = state.struct()
    cert = L.Cert()
    _check(lib.lamp_certificate(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), ws, nb,
                                _stream_handle(prob.device), ctypes.byref(cert)))
    return {k: getattr(cert, k) for k, _ in L.Cert._fields_}


def transport_cost(prob: Problem, params: L.Params, state: State) -> torch.Tensor:
    """<C, X^t> of the state's iterate in one pass over the pairs, as a 0-dim FP64 device tensor
    (written stream-ordered; no host synchronisation)."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    out = torch.empty((), dtype=torch.float64, device=prob.device)
    p = prob.struct()
    s = state.struct()
    _check(lib.lamp_transport_cost(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), ws, nb,
                                   _stream_handle(prob.device), out.data_ptr()))
    return out


def backward(prob: Problem, params: L.Params, state: State, grad_out: float = 1.0) -> torch.Tensor:
    """grad_out * sum_j X_ij dC_ij/dx_i at the state's iterate (envelope gradient), n x d FP32."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    g = torch.empty(prob.n, prob.d, dtype=torch.float32, device=prob.device)
    p = prob.struct()
    s = state.struct()
    _check(lib.lamp_backward(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), float(grad_out),
                             g.data_ptr(), ws, nb, _stream_handle(prob.device)))
    return g


def backward_y(prob: Problem, params: L.Params, state: State, grad_out: float = 1.0) -> torch.Tensor:
    """grad_out * sum_i X_ij dC_ij/dy_j at the state's iterate (envelope gradient with respect
    to the target points), m x d FP32."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    g = torch.empty(prob.m, prob.d, dtype=torch.float32, device=prob.device)
    p = prob.struct()
    s = state.struct()
    _check(lib.lamp_backward_y(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), float(grad_out),
                               g.data_ptr(), ws, nb, _stream_handle(prob.device)))
    return g


def sweep_times(prob: Problem, params: L.Params, state: State, reps: int = 10) -> tuple[float, float]:
    """Average device milliseconds of one row sweep and one column sweep (HIP events)."""
    lib = L.load()
    ws, nb = prob.workspace(params)
    p = prob.struct()
    s = state.struct()
    a = ctypes.c_double()
    b = ctypes.c_double()
    _check(lib.lamp_sweep_times(ctypes.byref(p), ctypes.byref(params), ctypes.byref(s), ws, nb,
                                _stream_handle(prob.device), int(reps), ctypes.byref(a),
                                ctypes.byref(b)))
    return a.value, b.value


def exp_rate(device="cuda", blocks: int = 8192, iters: int = 4096, reps: int = 5) -> float:
    """Measured issue rate of the base-2 exponential on this GPU (exponentials per second), from
    the library's probe kernel (measurement support)."""
    lib = L.load()
    out = ctypes.c_double()
    _check(lib.lamp_exp_rate(_stream_handle(torch.device(device)), int(blocks), int(iters), int(reps),
                             ctypes.byref(out)))
    return out.value


def solve_batched(probs: list, params: L.Params, states: list | None = None):
    """Batching form: all problems advance together, one launch per phase for the whole batch.
    Returns (states, reports, status)."""
    lib = L.load()
    count = len(probs)
    dev = probs[0].device
    if states is None:
        states = [State.fresh(p.m, dev) for p in probs]
    parr = (L.Problem * count)(*[p.struct() for p in probs])
    sarr = (L.State * count)(*[s.struct() for s in states])
    rarr = (L.Report * count)()
    need = int(lib.lamp_batch_workspace_bytes(parr, count, ctypes.byref(params)))
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    base = (ws.data_ptr() + 255) & ~255
    st = _check(lib.lamp_solve_batched(parr, count, ctypes.byref(params), sarr, base, need,
                                       _stream_handle(dev), rarr))
    for s, sc in zip(states, sarr):
        s.update(sc)
    reports = [{k: getattr(r, k) for k, _ in L.Report._fields_} for r in rarr]
    return states, reports, st


class LampOT(torch.autograd.Function):
    """Transport cost <C, X^T> of the LAMP iterate as a differentiable function of the source
    and target points x, y (envelope gradients at fixed duals and fixed cost scale)."""

    @staticmethod
    def forward(ctx, x, y, r, c, eta: float, tol: float, max_iter: int, cost_scale: float,
                metric: str = "sqeuclid"):
        prob = Problem(x.detach(), y.detach(), r, c, cost_scale=cost_scale, device=x.device, metric=metric)
        if cost_scale <= 0:
            prob.cost_scale, _ = cost_scale_of(prob)
            prob.cost_norm = 1.0
        params = make_params(eta=eta, tol=tol, max_iter=max_iter)
        state, report, _ = solve(prob, params)
        ctx.lamp = (prob, params, state)
        return transport_cost(prob, params, state)

    @staticmethod
    def backward(ctx, g):
        prob, params, state = ctx.lamp
        gx = backward(prob, params, state, float(g)) if ctx.needs_input_grad[0] else None
        gy = backward_y(prob, params, state, float(g)) if ctx.needs_input_grad[1] else None
        return gx, gy, None, None, None, None, None, None, None


cost_scale_of = cost_scale
