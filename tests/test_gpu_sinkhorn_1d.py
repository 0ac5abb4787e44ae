"""sinkhorn_w1_1d (HIP) against the FP64 oracle (Algorithm 1).

* The small correctness workload (n = m = 512, eps = 0.01, tol 1e-9, cap 2000)
  in FP64: same iteration count, potentials, marginal error and cost as the
  dense oracle; cost inside the closed-form entropic bounds.
* FP32-mantissa scans: cost and marginals within 1e-6 of the FP64 oracle.
* Iterate identity at fixed l against Algorithm 1 on the CPU, up to 2^20
  graded meshes.
* Edge cases: itr_max 0 and 1, n != m, single points, error statuses (a marginal
  error beyond the FP64 range included).
"""
import numpy as np
import pytest

from oracle import clib, closed_form as cf, dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import check_slack, dev, host, rand_meshes, torch_cuda

pytestmark = pytest.mark.gpu


def _solve(p, precision=0, tol=None, itr_max=None, **kw):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps,
                               p.tol if tol is None else tol,
                               p.itr_max if itr_max is None else itr_max,
                               precision=precision, **kw)
    return res, host(f), host(g)


def test_small_config_fp64_matches_dense_oracle():
    p = wl.config_small_1d()
    res, f, g = _solve(p)
    fo, go, ito, erro = clib.dense_sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, p.tol, p.itr_max)
    assert res["iters"] == ito
    assert np.max(np.abs(f - fo)) / p.eps <= 1e-9
    assert np.max(np.abs(g - go)) / p.eps <= 1e-9
    assert abs(res["marginal_err"] - erro) <= 1e-9 * erro + 1e-15
    w1o = clib.dense_cost_1d(p.x, p.y, fo, go, p.eps)
    assert abs(res["w1"] - w1o) <= 1e-10 * w1o
    lo, hi = cf.entropic_w1_bounds(p.x, p.u, p.y, p.v, p.eps, res["marginal_err"])
    assert lo <= res["w1"] <= hi


@pytest.mark.parametrize("precision", [0, 1])
def test_fp32_and_fp64_converge_to_the_oracle_plan(precision):
    p = wl.config_small_1d(n=1000)
    tol = 1e-6
    res, f, g = _solve(p, precision=precision, tol=tol, itr_max=20000)
    assert res["converged"]
    fo, go, ito, erro = clib.dense_sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, tol, 20000)
    w1o = clib.dense_cost_1d(p.x, p.y, fo, go, p.eps)
    assert abs(res["w1"] - w1o) <= 1e-6 * w1o
    # marginals of the returned plan recomputed by the oracle
    s = dense.logmatvec(p.x, p.y, g, p.eps)
    t = dense.logmatvec(p.y, p.x, f, p.eps)
    row = np.exp((f + s) / p.eps)
    col = np.exp((g + t) / p.eps)
    assert np.sum(np.abs(row - p.u)) <= (1e-12 if precision == 0 else 1e-6)
    # In both modes the stop is decided (FP32: confirmed) by the FP64 check of
    # the returned pair, so the error the oracle recomputes from (f, g) is
    # within tol (up to the rounding of the oracle's own sum, 1e-9 relative)
    # and equals the reported one.
    err_o = np.sum(np.abs(col - p.v))
    slack = check_slack(g, t, p.eps, p.v)
    assert err_o <= tol + slack, err_o
    assert abs(res["marginal_err"] - err_o) <= slack
    if precision == 0:
        assert res["iters"] == ito
    else:
        assert abs(res["iters"] - ito) <= max(3, 0.01 * ito)


@pytest.mark.parametrize("itr_max", [0, 1, 2, 7])
def test_iteration_cap(itr_max):
    p = wl.config_small_1d(n=300)
    res, f, g = _solve(p, tol=0.0, itr_max=itr_max)
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, itr_max)
    assert res["iters"] == ito == itr_max
    assert not res["converged"]
    assert np.max(np.abs(f - fo)) / p.eps <= 1e-10
    assert np.max(np.abs(g - go)) / p.eps <= 1e-10
    assert abs(res["marginal_err"] - erro) <= 1e-10 * erro


@pytest.mark.parametrize("n,m", [(1, 1), (1, 40), (40, 1), (3000, 700), (700, 3000)])
def test_unequal_and_degenerate_sizes(n, m):
    rng = np.random.default_rng(n * 7 + m)
    x, y = rand_meshes(n + m, n, m)
    u = wl.normalise(rng.uniform(0.1, 1, n)); v = wl.normalise(rng.uniform(0.1, 1, m))
    p = wl.Problem1D(x, y, u, v, 0.02, 1e-8, 4000)
    res, f, g = _solve(p)
    fo, go, ito, erro = clib.sinkhorn_1d(x, y, u, v, 0.02, 1e-8, 4000)
    assert res["iters"] == ito
    assert np.max(np.abs(f - fo)) / 0.02 <= 1e-9
    assert np.max(np.abs(g - go)) / 0.02 <= 1e-9


def test_paper_chebyshev_workload_fixed_iterations():
    """Section 4.1 workload (x = y Chebyshev nodes: every node is a tie),
    1000 iterations as in the paper, eps = 0.01."""
    p = wl.paper_chebyshev_1d(2000)
    res, f, g = _solve(p, tol=0.0, itr_max=1000)
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, 1000)
    assert res["iters"] == 1000
    assert np.max(np.abs(f - fo)) / p.eps <= 1e-9
    assert np.max(np.abs(g - go)) / p.eps <= 1e-9
    w1o = clib.dense_cost_1d(p.x, p.y, fo, go, p.eps)
    assert abs(res["w1"] - w1o) <= 1e-10 * w1o


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_full_size_graded_iterates(eps, precision):
    """n = m = 2^20 graded meshes: 12 iterations against Algorithm 1 on the CPU."""
    p = wl.config_graded_1d(1 << 20, eps)
    L = 12
    res, f, g = _solve(p, precision=precision, tol=0.0, itr_max=L)
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, eps, 0.0, L)
    assert res["iters"] == L
    # n + m = 2^21 merged points: 512 tiles of 4096, the resident solver's
    # full grid in FP32; FP64 runs the streaming general sweeps
    assert res["fast"] == (2 if precision == 1 else 0)
    tol = 1e-9 if precision == 0 else 2e-5
    df = np.max(np.abs(f - fo)) / eps
    dg = np.max(np.abs(g - go)) / eps
    assert df <= tol and dg <= tol, (df, dg)
    # FP64 check of the returned pair in both modes; in FP32 the pair itself
    # differs from the oracle's by the iterates' FP32 rounding (df, dg above)
    assert abs(res["marginal_err"] - erro) <= (1e-9 if precision == 0 else 1e-5) * max(erro, 1e-3)
    t = clib.finom_logmatvec(p.y, p.x, f, eps)
    err_r = np.sum(np.abs(np.exp((g + t) / eps) - p.v))
    assert abs(res["marginal_err"] - err_r) <= check_slack(g, t, eps, p.v)


def test_one_point_past_the_resident_grid():
    """n = 2^20 + 1, m = 2^20: one tile more than the resident grid holds,
    so the FP32 solve takes the streaming fast sweeps; 6 iterations against
    Algorithm 1 on the CPU."""
    q = wl.config_graded_1d(1 << 20, 1e-2)
    rng = np.random.default_rng(41)
    x = np.sort(np.concatenate([q.x, [rng.uniform(q.x[0], q.x[-1])]]))
    u = np.concatenate([q.u, [q.u.mean()]])
    u *= q.v.sum() / u.sum()
    p = wl.Problem1D(x, q.y, u, q.v, q.eps, 0.0, 0)
    L = 6
    res, f, g = _solve(p, precision=1, tol=0.0, itr_max=L)
    assert res["fast"] == 1 and res["iters"] == L
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, L)
    df = np.max(np.abs(f - fo)) / p.eps
    dg = np.max(np.abs(g - go)) / p.eps
    assert df <= 2e-5 and dg <= 2e-5, (df, dg)
    assert abs(res["marginal_err"] - erro) <= 1e-5 * max(erro, 1e-3)


def test_streaming_beyond_the_llc_iterates():
    """n = m = 2^24 graded meshes (a working set of about 1.5 GB, beyond the
    256 MB Infinity Cache; too large for the resident solver, so the streaming
    fast sweeps): 4 iterations against Algorithm 1 on the CPU."""
    p = wl.config_graded_1d(1 << 24, 1e-3)
    L = 4
    print("graded 1D n=2^24 eps=1e-3, 4 iterations", flush=True)
    res, f, g = _solve(p, precision=1, tol=0.0, itr_max=L)
    assert res["fast"] == 1 and res["iters"] == L
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, L)
    df = np.max(np.abs(f - fo)) / p.eps
    dg = np.max(np.abs(g - go)) / p.eps
    assert df <= 2e-5 and dg <= 2e-5, (df, dg)
    assert abs(res["marginal_err"] - erro) <= 1e-5 * max(erro, 1e-3)


def test_full_size_converged_cost_within_closed_form_bounds():
    p = wl.config_graded_1d(1 << 20, 1e-2)
    res, f, g = _solve(p, precision=1, tol=1e-6, itr_max=20000)
    assert res["converged"] and res["marginal_err"] <= 1e-6
    assert res["fast"] == 2   # the resident solver (one cooperative launch)
    lo, hi = cf.entropic_w1_bounds(p.x, p.u, p.y, p.v, p.eps, res["marginal_err"])
    assert lo <= res["w1"] <= hi
    # u-side marginal on sampled rows, recomputed by the oracle from (f, g)
    rows = np.random.default_rng(5).integers(0, len(p.x), 64)
    s = clib.dense_logmatvec(p.x, p.y, g, p.eps, rows=rows)
    np.testing.assert_allclose(np.exp((f[rows] + s) / p.eps), p.u[rows], rtol=2e-6)


def test_error_statuses():
    from paper_2605_26659_amd import FINOM_E_ARG, FINOM_E_MASS, FINOM_E_UNSORTED, FinomError
    p = wl.config_small_1d(n=64)
    xb = p.x.copy(); xb[[10, 11]] = xb[[11, 10]]
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(xb, p.y, p.u, p.v, p.eps, p.tol, 10))
    assert e.value.status == FINOM_E_UNSORTED
    ub = p.u.copy(); ub[3] = 0.0; ub /= ub.sum()
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(p.x, p.y, ub, p.v, p.eps, p.tol, 10))
    assert e.value.status == FINOM_E_MASS
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(p.x, p.y, p.u * 1.01, p.v, p.eps, p.tol, 10))
    assert e.value.status == FINOM_E_MASS
    with pytest.raises(FinomError) as e:
        _solve(p, itr_max=-1)
    assert e.value.status == FINOM_E_ARG
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(p.x, p.y, p.u, p.v, 0.0, p.tol, 10))
    assert e.value.status == FINOM_E_ARG
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(p.x, p.y * 3e4, p.u, p.v, 1e-3, p.tol, 10))
    assert e.value.status == FINOM_E_ARG


@pytest.mark.parametrize("precision,itr_max", [(0, 10), (1, 2)])
def test_marginal_error_beyond_fp64_range(precision, itr_max):
    """Masses of 1.5e308 (balanced and finite) at opposite ends, eps so small
    that the kernel moves no mass between the two points: the loop head's
    error sum_j |psi_j (K^T phi)_j - v_j| is about 2 x 1.5e308, beyond the
    largest FP64 number, in the first iterations (the oracle's Algorithm 1
    shows it), so the solve ends with FINOM_E_NUMERIC. The FP32 loop's own
    estimate caps its terms; its stop at the cap is checked in FP64, which
    sees the same overflow."""
    from paper_2605_26659_amd import FINOM_E_NUMERIC, FinomError
    x = np.array([0.0, 1.0]); y = np.array([0.0, 1.0])
    u = np.array([1.5e308, 1e-300]); v = np.array([1e-300, 1.5e308])
    assert u.sum() == v.sum() and np.isfinite(u.sum())
    *_, trace = clib.sinkhorn_1d(x, y, u, v, 1e-4, 1e-6, itr_max, trace=True)
    assert np.isinf(trace[1:3]).all()
    with pytest.raises(FinomError) as e:
        _solve(wl.Problem1D(x, y, u, v, 1e-4, 1e-6, itr_max), precision=precision)
    assert e.value.status == FINOM_E_NUMERIC


def test_repeated_calls_are_deterministic():
    p = wl.config_small_1d(n=2500)
    r1, f1, g1 = _solve(p, precision=1, tol=1e-7, itr_max=3000)
    r2, f2, g2 = _solve(p, precision=1, tol=1e-7, itr_max=3000)
    r1.pop("loop_ms"); r2.pop("loop_ms")
    assert r1 == r2
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2)
