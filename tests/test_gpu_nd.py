"""sinkhorn_w1_nd (HIP) on d-dimensional tensor meshes against the FP64 oracle.

* d = 3 and d = 4 at fixed iteration counts against the oracle's loop with
  products axis by axis, including axes of one point, unequal grids and a
  checking sweep of more lines than the deciding sweep sums itself;
* d = 1 and d = 2 run sinkhorn_w1_1d / sinkhorn_w1_2d: the same bits;
* d = 3 with FP32-mantissa scans to convergence;
* argument errors.
"""
import numpy as np
import pytest

from oracle import dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

pytestmark = pytest.mark.gpu


def _case(seed, ns, nt):
    rng = np.random.default_rng(seed)
    xs = [np.sort(rng.uniform(0, 1, k)) for k in ns]
    xt = [np.sort(rng.uniform(0, 1, k)) for k in nt]
    u = wl.normalise(rng.uniform(0.1, 1, tuple(ns)))
    v = wl.normalise(rng.uniform(0.1, 1, tuple(nt)))
    return xs, xt, u, v


def _solve(xs, xt, u, v, eps, tol, itr_max, precision=0):
    from paper_2605_26659_amd import sinkhorn_w1_nd
    res, F, G = sinkhorn_w1_nd([dev(a) for a in xs], [dev(a) for a in xt], dev(u.ravel(order="F")),
                               dev(v.ravel(order="F")), eps, tol, itr_max, precision=precision)
    return res, host(F).reshape(u.shape, order="F"), host(G).reshape(v.shape, order="F")


@pytest.mark.parametrize("ns,nt", [((6, 5, 4), (5, 7, 3)), ((9, 1, 8), (7, 3, 1)), ((3, 4, 2, 3), (2, 3, 4, 2)),
                                   ((40, 30, 20), (35, 25, 30)), ((3, 2, 4, 2, 3), (2, 3, 2, 3, 2)),
                                   ((2,) * 8, (2, 3, 2, 1, 2, 2, 2, 2)),
                                   # 44 x 36 = 1584 checked lines: their partial errors are
                                   # summed once ahead of the deciding sweep
                                   ((48, 40, 24), (44, 36, 30))])
def test_nd_fixed_iterations(ns, nt):
    xs, xt, u, v = _case(sum(ns) * 7 + sum(nt), ns, nt)
    eps, L = 0.05, 15
    res, F, G = _solve(xs, xt, u, v, eps, 0.0, L)
    ref = dense.sinkhorn_nd(xs, xt, u, v, eps, 0.0, L)
    assert res["iters"] == ref.iters == L
    assert np.max(np.abs(F - ref.f)) / eps <= 1e-9
    assert np.max(np.abs(G - ref.g)) / eps <= 1e-9
    assert abs(res["marginal_err"] - ref.err) <= 1e-10 * max(1.0, ref.err)
    assert abs(res["w1"] - ref.w1) <= 1e-10 * ref.w1


def test_nd_d1_and_d2_match_the_1d_and_2d_entry_points():
    from paper_2605_26659_amd import sinkhorn_w1_1d, sinkhorn_w1_2d
    xs, xt, u, v = _case(51, (300,), (257,))
    r1, f1, g1 = sinkhorn_w1_1d(dev(xs[0]), dev(xt[0]), dev(u), dev(v), 0.02, 0.0, 40, precision=0)
    rn, fn, gn = _solve(xs, xt, u, v, 0.02, 0.0, 40)
    # one and two axes run the 1D and 2D entry points: the same bits
    assert rn["iters"] == r1["iters"] == 40
    assert np.array_equal(fn, host(f1)) and np.array_equal(gn, host(g1))
    assert rn["w1"] == r1["w1"]
    p = wl.paper_random_2d(24, iters=30)
    r2, F2, G2 = sinkhorn_w1_2d(dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2), dev(p.u.ravel(order="F")),
                                dev(p.v.ravel(order="F")), p.eps, 0.0, 30)
    rn, Fn, Gn = _solve([p.x1, p.y1], [p.x2, p.y2], p.u, p.v, p.eps, 0.0, 30)
    assert rn["iters"] == r2["iters"] == 30
    assert np.array_equal(Fn.ravel(order="F"), host(F2))
    assert np.array_equal(Gn.ravel(order="F"), host(G2))
    assert rn["w1"] == r2["w1"]


def test_nd_fp32_to_convergence():
    xs, xt, u, v = _case(52, (20, 18, 16), (17, 21, 15))
    eps, tol = 0.05, 1e-6
    res, F, G = _solve(xs, xt, u, v, eps, tol, 5000, precision=1)
    ref = dense.sinkhorn_nd(xs, xt, u, v, eps, tol, 5000)
    assert res["converged"] and ref.converged
    assert abs(res["w1"] - ref.w1) <= 1e-6 * ref.w1
    assert abs(res["iters"] - ref.iters) <= max(3, ref.iters // 100)


def test_nd_argument_errors():
    from paper_2605_26659_amd import FINOM_E_ARG, FINOM_E_UNSORTED, FinomError, sinkhorn_w1_nd
    xs, xt, u, v = _case(53, (4, 3, 2), (3, 3, 2))
    args = (dev(u.ravel(order="F")), dev(v.ravel(order="F")), 0.05, 1e-6, 10)
    with pytest.raises(FinomError) as e:
        sinkhorn_w1_nd([], [], *args)
    assert e.value.status == FINOM_E_ARG
    nine = [dev(np.array([0.5]))] * 9
    with pytest.raises(FinomError) as e:
        sinkhorn_w1_nd(nine, nine, dev(np.ones(1)), dev(np.ones(1)), 0.05, 1e-6, 10)
    assert e.value.status == FINOM_E_ARG
    bad = [dev(a) for a in xs]
    bad[1] = dev(xs[1][::-1].copy())
    with pytest.raises(FinomError) as e:
        sinkhorn_w1_nd(bad, [dev(a) for a in xt], *args)
    assert e.value.status == FINOM_E_UNSORTED
