"""CPU checks of the seeded cost-matrix inputs (the explicit-cost workloads): the grid costs of
k x k image pairs have the norms the paper states for 2-D image problems (Appendix, the D_t
experiment: ||C||_inf = 2(sqrt(n) - 1)^2 for l2^2, 2(sqrt(n) - 1) for l1, sqrt(n) - 1 for
l_inf), equal the oracle's ground costs of the pixel coordinates, and the marginals are
full-support probability vectors."""
import numpy as np
import pytest

from oracle import lamp as OL
from paper_2511_11359_amd import workloads as W


@pytest.mark.parametrize("k", [4, 16, 32])
@pytest.mark.parametrize("kind,norm", [("sqeuclid", lambda q: 2 * q * q), ("l1", lambda q: 2 * q),
                                       ("linf", lambda q: q)])
def test_grid_cost_norms_match_the_paper(k, kind, norm):
    cmat = W.grid_cost(k, kind)
    assert cmat.shape == (k * k, k * k) and cmat.dtype == np.float32
    assert float(cmat.max()) == norm(k - 1)
    assert float(cmat.min()) == 0.0 and np.all(np.diag(cmat) == 0.0)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1", "linf"])
def test_grid_cost_is_the_ground_cost_of_the_pixel_grid(kind):
    k = 7
    yy, xx = np.divmod(np.arange(k * k), k)
    pts = np.stack([yy, xx], axis=1).astype(np.float64)
    ref = OL.ground_cost(pts, pts, 1.0, kind)
    assert np.array_equal(W.grid_cost(k, kind).astype(np.float64), ref)


def test_cost_workload_marginals():
    for wl in (W.image_pair(9, seed=3), W.random_cost(40, 25, seed=4)):
        assert wl.cost.dtype == np.float32 and np.all(wl.cost >= 0)
        for v in (wl.r, wl.c):
            assert np.all(v > 0) and abs(v.sum() - 1.0) < 1e-12
        assert wl.cost.shape == (wl.r.size, wl.c.size)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1", "linf"])
def test_device_grid_cost_generator_matches(kind):
    """The chunked torch generator of the large image pairs gives the same matrix (on the CPU)."""
    torch = pytest.importorskip("torch")
    got = W.grid_cost_device(6, kind, torch.device("cpu"), rows_per_chunk=5).numpy()
    assert np.array_equal(got, W.grid_cost(6, kind))
