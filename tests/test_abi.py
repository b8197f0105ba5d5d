"""The C-ABI library loads and exports every function include/lamp.h declares, the
ctypes structures have the C layout, and the host-side argument checks return their
status codes (they run before any device call: no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2511_11359_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lamp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lamp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["lamp_solve", "lamp_step", "lamp_certificate", "lamp_backward",
                     "lamp_workspace_bytes", "lamp_last_error", "lamp_cost_scale"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblamp.so not built")
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SYMBOLS, f"{name} has no ctypes declaration"


def test_ctypes_layout_matches_c(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lamp.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(lamp_problem), sizeof(lamp_params), sizeof(lamp_state), sizeof(lamp_trace),"
        "sizeof(lamp_cert), sizeof(lamp_report), offsetof(lamp_problem, cost_norm),"
        "offsetof(lamp_params, check_every), offsetof(lamp_report, row_fallbacks),"
        "offsetof(lamp_params, track_dt), offsetof(lamp_state, dt_partial),"
        "offsetof(lamp_cert, dual_eta_nu), offsetof(lamp_problem, cost_type));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(_lib.Problem), ctypes.sizeof(_lib.Params), ctypes.sizeof(_lib.State),
            ctypes.sizeof(_lib.Trace), ctypes.sizeof(_lib.Cert), ctypes.sizeof(_lib.Report),
            _lib.Problem.cost_norm.offset, _lib.Params.check_every.offset,
            _lib.Report.row_fallbacks.offset, _lib.Params.track_dt.offset, _lib.State.dt_partial.offset,
            _lib.Cert.dual_eta_nu.offset, _lib.Problem.cost_type.offset]
    assert got == want


# ---------------------------------------------------------------- host argument checks

FAKE = 0x100000          # non-null, 256-byte aligned; never dereferenced by the failing checks
LAMP_EINVAL, LAMP_ENOMEM = -1, -3


def _problem(**kw):
    f = dict(n=100, m=80, d=3, metric=0, x=FAKE, y=FAKE, r=FAKE, c=FAKE, cost_scale=0.0, cost_norm=0.0,
             cost=None, cost_type=0)
    f.update(kw)
    return _lib.Problem(f["n"], f["m"], f["d"], f["metric"], f["x"], f["y"], f["r"], f["c"],
                        f["cost_scale"], f["cost_norm"], f["cost"], f["cost_type"], 0)


def _params(**kw):
    f = dict(eta=1e-2, tol=0.0, max_iter=10, alpha=0.0, beta=0.0, tau1=0.0, tau2=0.0, precision=0,
             check_every=8, track_dt=0, reserved=0)
    f.update(kw)
    return _lib.Params(f["eta"], f["tol"], f["max_iter"], f["alpha"], f["beta"], f["tau1"], f["tau2"],
                       f["precision"], f["check_every"], f["track_dt"], f["reserved"])


def _step(prob, params, state=None, ws=FAKE, ws_bytes=1 << 40):
    lib = _lib.load()
    st = state if state is not None else _lib.State(FAKE, FAKE, 0, 0.0, 0.0)
    return lib.lamp_step(ctypes.byref(prob), ctypes.byref(params), ctypes.byref(st), ws, ws_bytes, None,
                         None, None)


@pytest.mark.parametrize("case,kw", [("n = 0", dict(n=0)), ("m = 0", dict(m=0)), ("d = 0", dict(d=0)),
                                     ("x NULL", dict(x=None)), ("c NULL", dict(c=None)),
                                     ("unknown ground cost", dict(metric=7)),
                                     ("cost matrix NULL", dict(metric=3, cost=None)),
                                     ("unknown cost element type", dict(metric=3, cost=FAKE, cost_type=5)),
                                     ("explicit cost wider than 2^30 columns",
                                      dict(metric=3, cost=FAKE, m=(1 << 30) + 1))])
def test_invalid_problem_is_rejected(case, kw):
    lib = _lib.load()
    assert _step(_problem(**kw), _params()) == LAMP_EINVAL, case
    assert lib.lamp_last_error()


@pytest.mark.parametrize("case,kw", [("eta < 0", dict(eta=-1.0)), ("eta inf", dict(eta=float("inf"))),
                                     ("tol NaN", dict(tol=float("nan"))), ("max_iter < 0", dict(max_iter=-1)),
                                     ("unknown precision", dict(precision=9)), ("track_dt = 2", dict(track_dt=2)),
                                     ("tracking in BF16", dict(track_dt=1, precision=_lib.PRECISIONS["bf16_mfma"]))])
def test_invalid_params_are_rejected(case, kw):
    assert _step(_problem(), _params(**kw)) == LAMP_EINVAL, case


def test_workspace_and_form_checks():
    lib = _lib.load()
    prob, params = _problem(), _params()
    need = lib.lamp_workspace_bytes(ctypes.byref(prob), ctypes.byref(params))
    assert need > 0
    big = _problem(n=1000, m=800)
    assert lib.lamp_workspace_bytes(ctypes.byref(big), ctypes.byref(params)) > need
    assert _step(prob, params, ws=None) == LAMP_EINVAL
    assert _step(prob, params, ws=FAKE + 8) == LAMP_EINVAL          # not 256-byte aligned
    assert _step(prob, params, ws_bytes=need - 1) == LAMP_ENOMEM
    bf16 = _params(precision=_lib.PRECISIONS["bf16_mfma"])
    assert _step(_problem(d=200), bf16) == LAMP_EINVAL               # matrix-core forms: d <= 128
    assert _step(_problem(metric=_lib.METRICS["l1"]), bf16) == LAMP_EINVAL   # inner products only


def test_invalid_state_is_rejected():
    prob, params = _problem(), _params()
    assert _step(prob, params, state=_lib.State(None, FAKE, 0, 0.0, 0.0)) == LAMP_EINVAL
    assert _step(prob, params, state=_lib.State(FAKE, FAKE, -1, 0.0, 0.0)) == LAMP_EINVAL
    assert _step(prob, params, state=_lib.State(FAKE, FAKE, 3, -1.0, 0.0)) == LAMP_EINVAL


def test_explicit_cost_checks():
    """A cost-matrix problem needs no point clouds and ignores d; the matrix-core forms and
    the point adjoints reject it before any device work."""
    lib = _lib.load()
    params = _params()
    expl = _problem(metric=_lib.METRICS["explicit"], x=None, y=None, d=0, cost=FAKE)
    assert lib.lamp_workspace_bytes(ctypes.byref(expl), ctypes.byref(params)) > 0
    bf16 = _params(precision=_lib.PRECISIONS["bf16_mfma"])
    assert _step(expl, bf16) == LAMP_EINVAL
    st = _lib.State(FAKE, FAKE, 3, 1.0, 0.0)
    for fn in (lib.lamp_backward, lib.lamp_backward_y):
        assert fn(ctypes.byref(expl), ctypes.byref(params), ctypes.byref(st), 1.0, FAKE, FAKE, 1 << 40,
                  None) == LAMP_EINVAL
        assert b"point clouds" in lib.lamp_last_error()


def _step_noalloc(prob, params):
    lib = _lib.load()
    st = _lib.State(FAKE, FAKE, 0, 0.0, 0.0)
    return lib.lamp_step_noalloc(ctypes.byref(prob), ctypes.byref(params), ctypes.byref(st), None, None,
                                 None)


def test_noalloc_step_host_checks():
    """lamp_step_noalloc rejects bad arguments, and problems whose workspace exceeds the fixed
    device scratch, before any device call."""
    lib = _lib.load()
    params = _params()
    assert _step_noalloc(_problem(n=0), params) == LAMP_EINVAL
    assert _step_noalloc(_problem(), _params(eta=-1.0)) == LAMP_EINVAL
    big = _problem(n=1 << 18, m=1 << 18)
    assert lib.lamp_workspace_bytes(ctypes.byref(big), ctypes.byref(params)) > _lib.NOALLOC_WS_BYTES
    assert _step_noalloc(big, params) == LAMP_ENOMEM
    assert b"fixed device scratch" in lib.lamp_last_error()
    src = open(HEADER).read()
    assert f"#define LAMP_NOALLOC_WS_BYTES ((size_t)64 << 20)" in src
    assert _lib.NOALLOC_WS_BYTES == 64 << 20
