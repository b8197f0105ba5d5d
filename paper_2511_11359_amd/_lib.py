"""ctypes declarations of the C ABI in include/lamp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblamp.so")

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_size_t, ctypes.c_void_p)

LAMP_OK = 0
LAMP_NOT_CONVERGED = 1
LAMP_EINVAL = -1
LAMP_EDOMAIN = -2
LAMP_ENOMEM = -3
LAMP_EDEVICE = -4
LAMP_ENUMERIC = -5
LAMP_FP32 = 0
LAMP_FP32_MFMA = 1
LAMP_BF16_MFMA = 2
LAMP_FP16_MFMA = 3
PRECISIONS = {"fp32": 0, "fp32_mfma": 1, "bf16_mfma": 2, "fp16_mfma": 3, "fp16x3_mfma": 4}
LAMP_SQEUCLID = 0
LAMP_L1 = 1
LAMP_LINF = 2
METRICS = {"sqeuclid": 0, "l1": 1, "linf": 2, "explicit": 3}
COST_TYPES = {"float32": 0, "bfloat16": 1, "float16": 2}
NOALLOC_WS_BYTES = 64 << 20        # LAMP_NOALLOC_WS_BYTES: the fixed scratch of lamp_step_noalloc

STATUS_NAMES = {0: "LAMP_OK", 1: "LAMP_NOT_CONVERGED", -1: "LAMP_EINVAL", -2: "LAMP_EDOMAIN",
                -3: "LAMP_ENOMEM", -4: "LAMP_EDEVICE", -5: "LAMP_ENUMERIC"}


class Problem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("m", c_int64), ("d", c_int32), ("metric", c_int32),
                ("x", c_void_p), ("y", c_void_p), ("r", c_void_p), ("c", c_void_p),
                ("cost_scale", c_double), ("cost_norm", c_double), ("cost", c_void_p),
                ("cost_type", c_int32), ("reserved", c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("eta", c_double), ("tol", c_double), ("max_iter", c_int64),
                ("alpha", c_double), ("beta", c_double), ("tau1", c_double), ("tau2", c_double),
                ("precision", c_int32), ("check_every", c_int32),
                ("track_dt", c_int32), ("reserved", c_int32)]


class State(ctypes.Structure):
    _fields_ = [("nu", c_void_p), ("theta", c_void_p), ("t", c_int64), ("inv_eta", c_double),
                ("dt_partial", c_double)]


class Trace(ctypes.Structure):
    _fields_ = [("log_za", c_void_p), ("log_zb", c_void_p), ("col_a", c_void_p),
                ("col_b", c_void_p), ("theta_bar", c_void_p), ("theta_hat", c_void_p)]


class Cert(ctypes.Structure):
    _fields_ = [("col_res", c_double), ("row_res", c_double), ("cost", c_double),
                ("dual_theta", c_double), ("dual_nu", c_double), ("primal_penalized", c_double),
                ("gap", c_double), ("prop_bound", c_double), ("cost_scale", c_double),
                ("cost_norm", c_double), ("t", c_int64), ("rounded_cost", c_double),
                ("dt", c_double), ("midpoint_bound", c_double), ("dual_eta_theta", c_double),
                ("dual_eta_nu", c_double)]


class Report(ctypes.Structure):
    _fields_ = [("iters", c_int64), ("t", c_int64), ("seconds", c_double), ("final_res", c_double),
                ("cost_scale", c_double), ("cost_norm", c_double), ("converged", c_int32),
                ("row_fallbacks", c_int32)]


SYMBOLS = {
    "lamp_workspace_bytes": (c_size_t, [ctypes.POINTER(Problem), ctypes.POINTER(Params)]),
    "lamp_cost_scale": (c_int32, [ctypes.POINTER(Problem), c_void_p, c_size_t, c_void_p,
                                  ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "lamp_step": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(State),
                            c_void_p, c_size_t, c_void_p, ctypes.POINTER(Trace),
                            ctypes.POINTER(c_double)]),
    "lamp_step_noalloc": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                    ctypes.POINTER(State), c_void_p, ctypes.POINTER(Trace),
                                    ctypes.POINTER(c_double)]),
    "lamp_solve": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(State),
                             c_void_p, c_size_t, c_void_p, ctypes.POINTER(Report)]),
    "lamp_certificate": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                   ctypes.POINTER(State), c_void_p, c_size_t, c_void_p,
                                   ctypes.POINTER(Cert)]),
    "lamp_backward": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                ctypes.POINTER(State), c_double, c_void_p, c_void_p, c_size_t,
                                c_void_p]),
    "lamp_transport_cost": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                      ctypes.POINTER(State), c_void_p, c_size_t, c_void_p, c_void_p]),
    "lamp_backward_y": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                  ctypes.POINTER(State), c_double, c_void_p, c_void_p, c_size_t,
                                  c_void_p]),
    "lamp_sweep_times": (c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                   ctypes.POINTER(State), c_void_p, c_size_t, c_void_p, c_int32,
                                   ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "lamp_exp_rate": (c_int32, [c_void_p, c_int32, c_int32, c_int32, ctypes.POINTER(c_double)]),
    "lamp_batch_workspace_bytes": (c_size_t, [ctypes.POINTER(Problem), c_int32, ctypes.POINTER(Params)]),
    "lamp_solve_batched": (c_int32, [ctypes.POINTER(Problem), c_int32, ctypes.POINTER(Params),
                                     ctypes.POINTER(State), c_void_p, c_size_t, c_void_p,
                                     ctypes.POINTER(Report)]),
    "lamp_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads liblamp.so and declares every exported symbol.  Raises if the library is missing:
    there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2511_11359_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
