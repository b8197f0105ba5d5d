"""lamp_step_noalloc (the workspace taken from the library's fixed device scratch) against
lamp_step with a caller workspace: the same kernels on the same inputs give bitwise equal
results.  Two problems in a row on one device, the second smaller, so the second call runs
on scratch that still holds the first call's contents; each problem takes several steps."""
import sys

import numpy as np
import pytest

from paper_2511_11359_amd import workloads as W
from tests.gpu_util import oracle_problem, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2511_11359_amd as P  # noqa: E402
from paper_2511_11359_amd import _lib as LIB  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [  # (n, m, d, seed, eta, precision): the second smaller than the first
    (2600, 3100, 3, 501, 1e-2, "fp32"),
    (700, 450, 2, 502, 0.0, "fp32"),
    (900, 1100, 16, 503, 0.0, "bf16_mfma"),
    (300, 200, 16, 504, 1e-3, "bf16_mfma"),
]


@pytest.mark.parametrize("pair", [(0, 1), (2, 3)])
def test_noalloc_step_matches_lamp_step(pair):
    for idx in pair:
        n, m, d, seed, eta, prec = CASES[idx]
        _say(f"noalloc case n={n} m={m} d={d} seed={seed} eta={eta} {prec}")
        wl = W.random_small(n, m, d, seed)
        _, _, s, _ = oracle_problem(wl)
        prob = P.Problem(wl.x, wl.y, wl.r, wl.c, cost_scale=s, cost_norm=1.0)
        params = P.make_params(eta=eta, precision=prec)
        assert prob.workspace(params)[1] <= LIB.NOALLOC_WS_BYTES
        sa = P.State.fresh(m)
        sb = P.State.fresh(m)
        for k in range(4):
            ra, ta = P.step(prob, params, sa, trace=True)
            rb, tb = P.step_noalloc(prob, params, sb, trace=True)
            torch.cuda.synchronize()
            assert (sa.t, sa.inv_eta, ra) == (sb.t, sb.inv_eta, rb), (k, ra, rb)
            for key in ta:
                assert np.array_equal(to_np(ta[key]), to_np(tb[key])), (k, key)
            assert np.array_equal(to_np(sa.nu), to_np(sb.nu)), k
            assert np.array_equal(to_np(sa.theta), to_np(sb.theta)), k
        _say("  equal after", sa.t, "steps; res", ra)
