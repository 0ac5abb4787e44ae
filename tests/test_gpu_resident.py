"""The resident solver: one cooperative launch runs the whole 1D loop with
every tile's points held on chip by one block (FP32; taken by sinkhorn_w1_1d
when the tiles fit the GPU at once). Tiles within the fast sweeps' range bound
run the variant with plain FP32 scans (result fast = 2), the others the
variant with extended-number scans (fast = 3).

* Against Algorithm 1 on the CPU at fixed iteration counts, on the graded
  workload, on uneven meshes (tiles holding only x or only y points) and,
  for the extended variant, on tiles far beyond the FP32 range.
* Against the streaming sweeps at convergence (same plan to rounding), and
  batch members against single calls bit for bit, also with more tiles than
  the persistent grid holds.
* The loop head's edge cases (no iteration, one iteration), determinism, and
  the bounded wait for the other tiles' records (forced from the host with a
  wait bound of zero polls: every block leaves the loop, the call reports a
  HIP failure, the next call is unaffected), alone and in a batch.
"""
import numpy as np
import pytest

from oracle import clib
from paper_2605_26659_amd import workloads as wl

from gpuhelp import check_slack, dev, host

pytestmark = pytest.mark.gpu

TOL_ITER = 2e-5     # |f - f_oracle| / eps after a few dozen FP32 iterations (as for the fast sweeps)


def _solve(p, tol, itr_max, precision=1):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, tol, itr_max,
                               precision=precision)
    return res, host(f), host(g)


def _against_oracle(p, iters):
    res, f, g = _solve(p, 0.0, iters)
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, iters)
    assert res["iters"] == iters
    assert np.max(np.abs(f - fo)) / p.eps <= TOL_ITER
    assert np.max(np.abs(g - go)) / p.eps <= TOL_ITER
    # the reported error is the FP64 check of the returned FP32 pair: equal to
    # the oracle's recomputation from (f, g), and off the oracle's own pair by
    # the FP32 iterates' rounding (a few 2^-24 per term, mass 1: ~3e-7)
    t = clib.finom_logmatvec(p.y, p.x, f, p.eps)
    err_r = np.sum(np.abs(np.exp((g + t) / p.eps) - p.v))
    assert abs(res["marginal_err"] - err_r) <= check_slack(g, t, p.eps, p.v)
    assert abs(res["marginal_err"] - erro) <= 3e-7 + 1e-4 * erro
    return res


def _uneven(seed, n, m, eps):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, n))
    y = np.sort(rng.uniform(0, 1, m))
    u = rng.uniform(0.5, 1.5, n); u /= u.sum()
    v = rng.uniform(0.5, 1.5, m); v *= u.sum() / v.sum()
    return wl.Problem1D(x, y, u, v, eps, 0.0, 0)


@pytest.mark.parametrize("n", [40000, 1 << 18])
def test_resident_matches_oracle_at_fixed_iterations(n):
    p = wl.config_graded_1d(n, 1e-2)
    res = _against_oracle(p, 24)
    assert res["fast"] == 2


@pytest.mark.parametrize("n,m", [(1, 1), (1, 7), (7, 1), (3, 5), (64, 1)])
def test_resident_tiny_problems(n, m):
    """One tile with a handful of points, one side possibly a single point
    (most of the block's slots idle)."""
    p = _uneven(7 * n + m, n, m, 5e-2)
    res = _against_oracle(p, 12)
    assert res["fast"] in (2, 3)


@pytest.mark.parametrize("n,eps,iters", [(300, 1e-3, 30), (3000, 1e-2, 40), (20000, 1e-3, 24)])
def test_extended_variant_matches_oracle(n, eps, iters):
    """Tiles beyond the fast bound (coarse meshes, small eps: terms of one
    tile span hundreds to thousands of binary orders): one tile, and a few."""
    if n == 300:
        q = wl.config_batch_problem(3, n)
        p = wl.Problem1D(q.x, q.y, q.u, q.v, eps, 0.0, 0)
    else:
        p = wl.config_graded_1d(n, eps)
    res = _against_oracle(p, iters)
    assert res["fast"] == 3


def test_extended_variant_and_general_sweeps_converge_to_the_same_plan(monkeypatch):
    p = wl.config_graded_1d(3000, 1e-2)
    rr, fr, gr = _solve(p, 1e-6, 20000)
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    rs, fs, gs = _solve(p, 1e-6, 20000)
    r64, _, _ = _solve(p, 1e-6, 20000, precision=0)
    assert rr["fast"] == 3 and rs["fast"] == 0
    assert rr["converged"] and rs["converged"]
    assert abs(rr["w1"] - rs["w1"]) <= 1e-6 * rs["w1"]
    # each stops where the FP64 check of its own pair passes: the resident
    # variant within max(3, 1 %) of the FP64 loop's count, the general sweeps
    # (FP32-mantissa exp2 / log2, an error floor of about 2.5e-7 on unit mass)
    # within max(8, 3 %)
    assert abs(rr["iters"] - r64["iters"]) <= max(3, 0.01 * r64["iters"]), (rr["iters"], r64["iters"])
    assert abs(rs["iters"] - r64["iters"]) <= max(8, 0.03 * r64["iters"]), (rs["iters"], r64["iters"])
    assert np.max(np.abs(fr - fs)) / p.eps <= 1e-4


@pytest.mark.parametrize("n,m", [(2100, 2000), (30000, 60), (60, 30000), (5000, 9000)])
def test_resident_uneven_meshes(n, m):
    """Few tiles, and tiles with columns of one kind only."""
    p = _uneven(n + m, n, m, 1e-1)
    res = _against_oracle(p, 16)
    assert res["fast"] == 2


def test_resident_and_streaming_converge_to_the_same_plan(monkeypatch):
    p = wl.config_graded_1d(1 << 17, 1e-2)
    rr, fr, gr = _solve(p, 1e-6, 20000)
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    rs, fs, gs = _solve(p, 1e-6, 20000)
    assert rr["fast"] == 2 and rs["fast"] == 1
    assert rr["converged"] and rs["converged"]
    assert abs(rr["w1"] - rs["w1"]) <= 1e-6 * rs["w1"]
    assert abs(rr["iters"] - rs["iters"]) <= max(3, 0.01 * rs["iters"])
    assert np.max(np.abs(fr - fs)) / p.eps <= 1e-4


def test_resident_solve_matches_batch_member():
    """A batch member that fits runs on the resident batch kernel, which runs
    the single-problem kernel's code on the same tiles: bit for bit the
    single call's results."""
    from paper_2605_26659_amd import finom_batch
    from test_gpu_batch import _alone, _assert_same, _desc_1d
    p = wl.config_batch_problem(7, 30000)
    d = _desc_1d(p, tol=1e-6, itr_max=5000)
    st, res = finom_batch([d], precision=1)
    ra, fa, ga = _alone(d, 1, resident=True)
    assert ra["fast"] == 2 and res[0]["fast"] == 2
    _assert_same(res[0], d, ra, fa, ga)


def test_resident_batch_wait_bound_with_both_grids(monkeypatch):
    """Members within and beyond the fast bound: the two persistent grids run
    at the same time (the extended one cooperative, the fast one behind a wait
    for the extended blocks' start). With a bound of zero polls both give up,
    every block leaves and the call reports FINOM_E_HIP; the next call runs
    both grids normally."""
    from paper_2605_26659_amd import FINOM_E_HIP, FINOM_NOT_CONVERGED, FINOM_OK, FinomError, finom_batch
    from test_gpu_batch import _desc_1d
    probs = [wl.config_batch_problem(100 + i, 20000 + 700 * i) for i in range(12)]
    descs = [_desc_1d(p, tol=1e-6, itr_max=300) for p in probs]
    monkeypatch.setenv("FINOM_RESIDENT_SPIN", "0")
    with pytest.raises(FinomError) as e:
        finom_batch(descs, precision=1)
    assert e.value.status == FINOM_E_HIP
    assert "grid wait" in str(e.value)
    monkeypatch.delenv("FINOM_RESIDENT_SPIN")
    st, res = finom_batch(descs, precision=1)
    assert st in (FINOM_OK, FINOM_NOT_CONVERGED)
    kinds = {r["fast"] for r in res}
    assert kinds == {2, 3}, kinds


def test_batch_with_more_tiles_than_the_grid():
    """Forty multi-tile members (about a thousand tiles in all, more than the
    grid holds) share the persistent grid: blocks take tiles in order and wait
    for their problem's other tiles. Members whose tiles fail the fast sweeps'
    range bound (the smallest eps) run on the extended-number variant's grid,
    alone as in the batch. Every member checked equals its single call bit
    for bit."""
    from paper_2605_26659_amd import FINOM_NOT_CONVERGED, FINOM_OK, finom_batch
    from test_gpu_batch import _alone, _assert_same, _desc_1d
    probs = [wl.config_batch_problem(100 + i, 20000 + 700 * i) for i in range(40)]
    descs = [_desc_1d(p, tol=1e-6, itr_max=3000) for p in probs]
    st, res = finom_batch(descs, precision=1)
    assert st in (FINOM_OK, FINOM_NOT_CONVERGED)
    assert all(r["status"] in (FINOM_OK, FINOM_NOT_CONVERGED) for r in res)
    resident = [i for i, r in enumerate(res) if r["fast"] == 2]
    other = [i for i, r in enumerate(res) if r["fast"] != 2]
    assert all(res[i]["fast"] == 3 for i in other)   # beyond the bound: the extended variant
    tiles = sum(-(-(2 * len(probs[i].x)) // wl_tile(len(probs[i].x))) for i in resident)
    assert len(resident) >= 10 and tiles > 512, (len(resident), tiles)
    for i in resident[::max(1, len(resident) // 5)] + other[:2]:
        ra, fa, ga = _alone(descs[i], 1, resident=True)
        _assert_same(res[i], descs[i], ra, fa, ga)


def wl_tile(n):
    """Tile size of a 1D problem of n + n points in FP32 (the tuned table's
    shape: 256 x 4, 256 x 8, 512 x 8, 128 x 4, 512 x 4)."""
    from paper_2605_26659_amd import finom_tile_config
    return {0: 1024, 1: 2048, 2: 4096, 3: 512, 4: 2048}[finom_tile_config(1, 2 * n)]


@pytest.mark.parametrize("itr_max", [0, 1, 2])
def test_resident_loop_head_edge_cases(itr_max, monkeypatch):
    """No iteration: the initial pair and its error; then one and two."""
    p = wl.config_graded_1d(20000, 1e-2)
    rr, fr, gr = _solve(p, 0.0, itr_max)
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    rs, fs, gs = _solve(p, 0.0, itr_max)
    assert rr["fast"] == 2
    assert rr["iters"] == rs["iters"] == itr_max
    assert abs(rr["marginal_err"] - rs["marginal_err"]) <= 1e-6 * rs["marginal_err"]
    assert np.max(np.abs(fr - fs)) / p.eps <= 1e-5
    assert np.max(np.abs(gr - gs)) / p.eps <= 1e-5
    if itr_max == 0:
        assert np.array_equal(fr, fs) and np.array_equal(gr, gs)


def test_resident_is_deterministic():
    p = wl.config_graded_1d(1 << 17, 1e-3)
    r1, f1, g1 = _solve(p, 1e-6, 300)
    r2, f2, g2 = _solve(p, 1e-6, 300)
    assert r1["fast"] == 2
    assert r1["iters"] == r2["iters"] and r1["w1"] == r2["w1"]
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2)


def test_resident_wait_bound(monkeypatch):
    from paper_2605_26659_amd import FINOM_E_HIP, FINOM_OK, FinomError, sinkhorn_w1_1d
    p = wl.config_graded_1d(1 << 17, 1e-2)
    monkeypatch.setenv("FINOM_RESIDENT_SPIN", "0")
    with pytest.raises(FinomError) as e:
        sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, 1e-6, 200, precision=1)
    assert e.value.status == FINOM_E_HIP
    assert "grid wait" in str(e.value)
    monkeypatch.delenv("FINOM_RESIDENT_SPIN")
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, 1e-6, 200, precision=1)
    assert res["fast"] == 2 and res["status"] in (FINOM_OK, 1)


def test_resident_batch_wait_bound(monkeypatch):
    """The batch kernel's waits are bounded the same way: with a bound of
    zero polls some wait gives up, every block leaves, and the call reports
    FINOM_E_HIP; the next call runs normally."""
    from paper_2605_26659_amd import FINOM_E_HIP, FINOM_NOT_CONVERGED, FINOM_OK, FinomError, finom_batch
    from test_gpu_batch import _desc_1d
    descs = [_desc_1d(wl.config_batch_problem(200 + i, 30000), tol=1e-6, itr_max=400) for i in range(6)]
    monkeypatch.setenv("FINOM_RESIDENT_SPIN", "0")
    with pytest.raises(FinomError) as e:
        finom_batch(descs, precision=1)
    assert e.value.status == FINOM_E_HIP
    assert "grid wait" in str(e.value)
    monkeypatch.delenv("FINOM_RESIDENT_SPIN")
    st, res = finom_batch(descs, precision=1)
    assert st in (FINOM_OK, FINOM_NOT_CONVERGED)
    assert all(r["fast"] == 2 for r in res)
