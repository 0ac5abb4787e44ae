"""sinkhorn_w1_2d (HIP) against the FP64 oracle (Algorithm 2).

* the paper's 2D workload (section 4.3: sorted uniform node vectors, masses
  U[0,1]) at fixed iteration counts against Algorithm 2 on the CPU and the
  full (NM)x(NM) dense definition;
* product measures: the 2D iterate equals the product of the two 1D
  iterates and the cost splits into the 1D costs;
* unequal grids (n1 != n2, m1 != m2), FP32 scans at convergence;
* the 1024 x 1024 tanh-stretched workload at a fixed iteration count;
* the FP32 loop on extended-number state for every line shape and both
  in-line scans, with small eps and zero masses, and on degenerate grids.
"""
import numpy as np
import pytest

from oracle import clib, closed_form as cf, dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import check_slack, dev, host

pytestmark = pytest.mark.gpu


def _solve(p, precision=0, tol=None, itr_max=None):
    from paper_2605_26659_amd import sinkhorn_w1_2d
    res, F, G = sinkhorn_w1_2d(dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2),
                               dev(p.u.ravel(order="F")), dev(p.v.ravel(order="F")), p.eps,
                               p.tol if tol is None else tol,
                               p.itr_max if itr_max is None else itr_max, precision=precision)
    F = host(F).reshape(p.u.shape, order="F")
    G = host(G).reshape(p.v.shape, order="F")
    return res, F, G


@pytest.mark.parametrize("side", [10, 20, 40])
def test_paper_2d_workload_fixed_iterations(side):
    p = wl.paper_random_2d(side, iters=60)
    res, F, G = _solve(p, tol=0.0, itr_max=60)
    Fo, Go, ito, erro = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 60)
    assert res["iters"] == ito == 60
    assert np.max(np.abs(F - Fo)) / p.eps <= 1e-9
    assert np.max(np.abs(G - Go)) / p.eps <= 1e-9
    assert abs(res["marginal_err"] - erro) <= 1e-9 * erro
    w1o = dense.transport_cost_2d_full(p.x1, p.y1, p.x2, p.y2, Fo, Go, p.eps)
    assert abs(res["w1"] - w1o) <= 1e-10 * w1o


def test_matches_full_dense_definition_tiny():
    p = wl.paper_random_2d(6, iters=25)
    res, F, G = _solve(p, tol=0.0, itr_max=25)
    r = dense.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 25, full=True)
    assert np.max(np.abs(F - r.f)) / p.eps <= 1e-9
    assert np.max(np.abs(G - r.g)) / p.eps <= 1e-9
    assert abs(res["w1"] - r.w1) <= 1e-10 * r.w1


@pytest.mark.parametrize("precision", [0, 1])
def test_product_measures_factorise(precision):
    rng = np.random.default_rng(3)
    n1, n2, m1, m2 = 37, 29, 23, 41
    x1, x2 = np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, n2))
    y1, y2 = np.sort(rng.uniform(0, 1, m1)), np.sort(rng.uniform(0, 1, m2))
    ux, vx = wl.normalise(rng.uniform(.1, 1, n1)), wl.normalise(rng.uniform(.1, 1, n2))
    uy, vy = wl.normalise(rng.uniform(.1, 1, m1)), wl.normalise(rng.uniform(.1, 1, m2))
    eps, L = 0.02, 40
    p = wl.Problem2D(x1, y1, x2, y2, np.outer(ux, uy), np.outer(vx, vy), eps, 0.0, L)
    res, F, G = _solve(p, precision=precision, tol=0.0, itr_max=L)
    fx, gx, _, _ = clib.sinkhorn_1d(x1, x2, ux, vx, eps, 0.0, L)
    fy, gy, _, _ = clib.sinkhorn_1d(y1, y2, uy, vy, eps, 0.0, L)
    tol = 1e-9 if precision == 0 else 2e-5
    assert np.max(np.abs(F - (fx[:, None] + fy[None, :]))) / eps <= tol
    assert np.max(np.abs(G - (gx[:, None] + gy[None, :]))) / eps <= tol
    wx = clib.dense_cost_1d(x1, x2, fx, gx, eps)
    wy = clib.dense_cost_1d(y1, y2, fy, gy, eps)
    assert abs(res["w1"] - (wx + wy)) <= (1e-10 if precision == 0 else 1e-6) * (wx + wy)


@pytest.mark.parametrize("precision", [0, 1])
def test_unequal_grids_to_tolerance(precision):
    rng = np.random.default_rng(5)
    n1, m1, n2, m2 = 33, 20, 25, 31
    p = wl.Problem2D(np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1)),
                     np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2)),
                     wl.normalise(rng.uniform(.1, 1, (n1, m1))),
                     wl.normalise(rng.uniform(.1, 1, (n2, m2))), 0.03, 1e-6, 20000)
    res, F, G = _solve(p, precision=precision)
    assert res["converged"]
    Fo, Go, ito, erro = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 1e-6, 20000)
    w1o = dense.transport_cost_2d_full(p.x1, p.y1, p.x2, p.y2, Fo, Go, p.eps)
    assert abs(res["w1"] - w1o) <= 1e-6 * w1o
    if precision == 0:
        assert res["iters"] == ito
    # plan marginals recomputed by the oracle from the returned potentials
    T = dense.logmatvec_2d(p.x2, p.y2, p.x1, p.y1, F, p.eps)
    # the stop is decided (FP32: confirmed) by the FP64 check of the returned
    # pair: the oracle's recomputed error is within tol and equals the reported one
    err_o = np.sum(np.abs(np.exp((G + T) / p.eps) - p.v))
    slack = check_slack(G, T, p.eps, p.v)
    assert err_o <= 1e-6 + slack, err_o
    assert abs(res["marginal_err"] - err_o) <= slack
    S = dense.logmatvec_2d(p.x1, p.y1, p.x2, p.y2, G, p.eps)
    assert np.sum(np.abs(np.exp((F + S) / p.eps) - p.u)) <= (1e-12 if precision == 0 else 1e-6)


def test_lp_bounds_tiny_to_tolerance():
    rng = np.random.default_rng(9)
    p = wl.Problem2D(np.sort(rng.uniform(0, 1, 3)), np.sort(rng.uniform(0, 1, 3)),
                     np.sort(rng.uniform(0, 1, 3)), np.sort(rng.uniform(0, 1, 2)),
                     wl.normalise(rng.uniform(.1, 1, (3, 3))),
                     wl.normalise(rng.uniform(.1, 1, (3, 2))), 0.01, 1e-11, 200000)
    res, F, G = _solve(p)
    XR, YR = np.meshgrid(p.x1, p.y1, indexing="ij"); XC, YC = np.meshgrid(p.x2, p.y2, indexing="ij")
    w = cf.w1_lp_points(XR.ravel("F"), YR.ravel("F"), p.u.ravel("F"),
                        XC.ravel("F"), YC.ravel("F"), p.v.ravel("F"))
    gap = p.eps * min(cf.entropy(p.u), cf.entropy(p.v))
    assert w - 2 * res["marginal_err"] <= res["w1"] <= w + gap + 2 * res["marginal_err"]


@pytest.mark.parametrize("precision", [0, 1])
def test_tanh_1024_fixed_iterations(precision):
    """The 1024 x 1024 stretched workload (same mesh for source and target:
    ties on every node), 6 iterations against Algorithm 2 on the CPU."""
    p = wl.config_tanh_2d(1024)
    L = 6
    res, F, G = _solve(p, precision=precision, tol=0.0, itr_max=L)
    Fo, Go, ito, erro = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, L)
    assert res["iters"] == L
    tol = 1e-9 if precision == 0 else 2e-5
    assert np.max(np.abs(F - Fo)) / p.eps <= tol
    assert np.max(np.abs(G - Go)) / p.eps <= tol
    assert abs(res["marginal_err"] - erro) <= (1e-9 if precision == 0 else 1e-5) * erro


def test_error_statuses_2d():
    from paper_2605_26659_amd import FINOM_E_MASS, FINOM_E_UNSORTED, FinomError
    p = wl.paper_random_2d(8, iters=5)
    bad = wl.Problem2D(p.x1[::-1].copy(), p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 5)
    with pytest.raises(FinomError) as e:
        _solve(bad)
    assert e.value.status == FINOM_E_UNSORTED
    bad = wl.Problem2D(p.x1, p.y1, p.x2, p.y2, p.u * 2, p.v, p.eps, 0.0, 5)
    with pytest.raises(FinomError) as e:
        _solve(bad)
    assert e.value.status == FINOM_E_MASS


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n1,m1,n2,m2", [(1, 5, 7, 1), (5, 1, 1, 6), (1, 1, 4, 3), (6, 4, 1, 1), (2, 300, 3, 257),
                                         (300, 2, 257, 3)])
def test_degenerate_and_thin_grids(n1, m1, n2, m2, precision):
    """Grids of one row or one column and thin grids: psi is row-major inside
    the solver, so these are the cases where its transposes and the strides
    of the intermediates degenerate. Some of these problems are solved
    exactly by one iteration (the error left is rounding, ~1e-16), so the
    loop runs to tol 1e-12 rather than to a fixed count."""
    rng = np.random.default_rng(n1 * 1000 + m1 * 100 + n2 * 10 + m2)
    x1, y1 = np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1))
    x2, y2 = np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2))
    u = wl.normalise(rng.uniform(0.1, 1, (n1, m1))); v = wl.normalise(rng.uniform(0.1, 1, (n2, m2)))
    if precision == 0:
        p = wl.Problem2D(x1, y1, x2, y2, u, v, 0.05, 1e-12, 12)
        res, F, G = _solve(p)
        ref = dense.sinkhorn_2d(x1, y1, x2, y2, u, v, 0.05, 1e-12, 12)
        assert res["iters"] == ref.iters
        tol, wtol = 1e-9, 1e-10
    else:
        # FP32 (the extended-state loop: lines of one point and thin lines):
        # a fixed count, as its error floor is far above 1e-12 (the oracle
        # stops early where one iteration solves the problem exactly: its
        # error is then 0, and later iterations keep that fixed point)
        p = wl.Problem2D(x1, y1, x2, y2, u, v, 0.05, 0.0, 12)
        res, F, G = _solve(p, precision=1)
        assert res["fast"] == 4 and res["iters"] == 12
        ref = dense.sinkhorn_2d(x1, y1, x2, y2, u, v, 0.05, 0.0, 12)
        assert ref.iters == 12 or ref.err == 0.0
        tol, wtol = 2e-5, 1e-6
    assert np.max(np.abs(F - ref.f)) / 0.05 <= tol
    assert np.max(np.abs(G - ref.g)) / 0.05 <= tol
    assert abs(res["w1"] - ref.w1) <= wtol * ref.w1


@pytest.mark.parametrize("scan", ["f64", "ext"])
@pytest.mark.parametrize("shape", [None, 0, 1, 2, 3, 4])
def test_extended_state_loop_against_algorithm2(shape, scan, monkeypatch):
    """The FP32 loop on extended-number state (result fast = 4) for every line
    shape and both in-line scans (FP64 mantissas against a reference per wave,
    and extended numbers), on unequal ragged grids (several waves per line, a
    partial last one), at a fixed iteration count against Algorithm 2 in C."""
    if shape is not None:
        monkeypatch.setenv("FINOM_LINE_SHAPE", str(shape))
    if scan == "ext":
        monkeypatch.setenv("FINOM_LINE_SCAN", "ext")
    rng = np.random.default_rng(17)
    n1, m1, n2, m2 = 200, 131, 173, 250
    p = wl.Problem2D(np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1)),
                     np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2)),
                     wl.normalise(rng.uniform(.1, 1, (n1, m1))),
                     wl.normalise(rng.uniform(.1, 1, (n2, m2))), 0.02, 0.0, 40)
    res, F, G = _solve(p, precision=1)
    assert res["fast"] == 4 and res["iters"] == 40
    Fo, Go, ito, erro = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 40)
    assert np.max(np.abs(F - Fo)) / p.eps <= 2e-5
    assert np.max(np.abs(G - Go)) / p.eps <= 2e-5
    # the returned pair's error is the FP64 check's
    assert abs(res["marginal_err"] - erro) <= 1e-5 * erro


def test_extended_state_loop_small_eps():
    """eps small enough that a wave's columns span far more than FP64's range
    of kernel decay (the extended-number scan runs), masses spanning many
    orders of magnitude."""
    rng = np.random.default_rng(19)
    n1, m1, n2, m2 = 300, 90, 120, 280
    u = np.exp(rng.uniform(-40, 0, (n1, m1)))
    v = np.exp(rng.uniform(-40, 0, (n2, m2)))
    p = wl.Problem2D(np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1)),
                     np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2)),
                     wl.normalise(u), wl.normalise(v), 2e-3, 0.0, 30)
    res, F, G = _solve(p, precision=1)
    assert res["fast"] == 4 and res["iters"] == 30
    Fo, Go, ito, erro = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, 30)
    assert np.max(np.abs(F - Fo)) / p.eps <= 2e-5
    assert np.max(np.abs(G - Go)) / p.eps <= 2e-5
    assert abs(res["marginal_err"] - erro) <= 1e-5 * erro
