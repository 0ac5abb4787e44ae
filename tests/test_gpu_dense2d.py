"""The 2D dense baselines (section 4's standard Sinkhorn product on tensor
meshes) against the oracle: the per-axis matrix products on the matrix cores
and the full (NM)^2 product, each compared entry by entry with the oracle's
dense definitions (per axis, eq. 2d-kron, and through the full kernel) and
with its recurrence-based 2D product, on grids that span several 64 x 64
tiles with ragged edges and at the 1024 x 1024 tanh workload's size."""
import numpy as np
import pytest

from oracle import clib, dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

pytestmark = pytest.mark.gpu


def _grids(seed, n1, m1, n2, m2):
    rng = np.random.default_rng(seed)
    s = lambda k: np.sort(rng.uniform(0, 1, k))
    return s(n1), s(m1), s(n2), s(m2), rng.normal(scale=0.05, size=(n2, m2))


@pytest.mark.parametrize("shape", [(37, 29, 41, 33), (130, 70, 100, 90), (1, 64, 65, 1), (64, 64, 64, 64)])
@pytest.mark.parametrize("full", [False, True])
def test_dense_2d_against_the_oracle(shape, full):
    from paper_2605_26659_amd import dense_matvec_2d
    n1, m1, n2, m2 = shape
    x1, y1, x2, y2, G = _grids(sum(shape), n1, m1, n2, m2)
    eps = 0.03
    print(f"dense 2D shape={shape} full={full}", flush=True)
    out = host(dense_matvec_2d(dev(x1), dev(y1), dev(x2), dev(y2), eps, dev(G.ravel(order="F")), full=full))
    out = out.reshape((n1, m1), order="F")
    want = dense.logmatvec_2d(x1, y1, x2, y2, G, eps)
    assert np.max(np.abs(out - want)) / eps <= 1e-12
    if n1 * m1 * n2 * m2 <= 2e7:
        want_full = dense.logmatvec_2d_full(x1, y1, x2, y2, G, eps)
        assert np.max(np.abs(out - want_full)) / eps <= 1e-12


@pytest.mark.parametrize("side,full", [(1024, False), (256, True)])
def test_dense_2d_at_the_tanh_workload(side, full):
    """The workload the 2D bench record times (tanh mesh, eps = 5e-3), with
    potentials from a few Sinkhorn iterations, against the oracle's
    recurrence-based 2D product."""
    from paper_2605_26659_amd import dense_matvec_2d
    p = wl.config_tanh_2d(side=side)
    F, G, _, _ = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 3)
    print(f"dense 2D tanh side={side} full={full}", flush=True)
    out = host(dense_matvec_2d(dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2), p.eps, dev(G.ravel(order="F")),
                               full=full)).reshape((side, side), order="F")
    want = clib.finom_logmatvec_2d(p.x1, p.y1, p.x2, p.y2, G, p.eps)
    assert np.max(np.abs(out - want)) / p.eps <= 1e-11


def test_dense_2d_refusals():
    from paper_2605_26659_amd import FinomError, dense_matvec_2d
    x1, y1, x2, y2, G = _grids(1, 4, 4, 4, 4)
    with pytest.raises(FinomError):
        dense_matvec_2d(dev(x1), dev(y1), dev(x2), dev(y2), 0.0, dev(G.ravel(order="F")))
