"""The C ABI from a plain C program, without Python in the process: tests/c_abi/solve_example.c
(built by build()) reads a problem, runs lamp_solve for 40 iterations from the fresh state and
lamp_certificate, and writes nu, theta and the certificate's transport cost; these against the
FP64 oracle with the tolerances of the Python-driven parity tests (duals 1e-6, cost 1e-5)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import lamp as OL
from paper_2511_11359_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "solve_example")


def test_plain_c_program_solves_through_the_abi(tmp_path):
    assert os.path.exists(EXE), "tests/c_abi/solve_example is not built: run __graft_entry__.build()"
    wl = W.random_small(96, 80, 2, seed=5, eta=1e-2)
    T = 40
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([wl.n, wl.m], dtype=np.int64).tobytes())
        f.write(np.array([wl.d], dtype=np.int32).tobytes())
        for a, t in ((wl.x, np.float32), (wl.y, np.float32), (wl.r, np.float64), (wl.c, np.float64)):
            f.write(np.ascontiguousarray(a, dtype=t).tobytes())
    print("case", wl.name, "T", T, flush=True)
    sys.stdout.flush()
    run = subprocess.run([EXE, str(src), str(dst), str(T), repr(wl.eta)], capture_output=True, text=True,
                         timeout=120)
    print(run.stdout, run.stderr, flush=True)
    assert run.returncode == 0, run.stderr
    out = np.fromfile(dst, dtype=np.float64, count=2 * wl.m + 1)
    t = int(np.fromfile(dst, dtype=np.int64)[-1])
    nu, th, cost = out[:wl.m], out[wl.m:2 * wl.m], out[-1]
    x, y = wl.x.astype(np.float64), wl.y.astype(np.float64)
    s = 1.0 / OL.max_sqdist(x, y)
    C = OL.sqeuclid_cost(x, y, s)
    prm = OL.Params(eta=wl.eta)
    st_or, _ = OL.lamp_dense(C, wl.r, wl.c, prm, T, 1.0, trace=False)
    cert_or = OL.certificate(C, wl.r, wl.c, st_or, prm.resolved(1.0), 1.0)
    e_nu = np.max(np.abs(nu - st_or.nu)) / max(np.max(np.abs(st_or.nu)), 0.5)
    e_th = np.max(np.abs(th - st_or.theta)) / max(np.max(np.abs(st_or.theta)), 0.5)
    print(f"C program: nu err {e_nu:.2e}, theta err {e_th:.2e}, cost {cost:.12e} oracle {cert_or['cost']:.12e}",
          flush=True)
    assert t == T
    assert e_nu <= 1e-6 and e_th <= 1e-6
    assert abs(cost - cert_or["cost"]) <= 1e-5 * abs(cert_or["cost"])
