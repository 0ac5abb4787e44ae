"""The resident solver: one cooperative launch runs the whole 1D loop with
every tile's points held on chip by one block (FP32 fast sweeps, tiles of
512 x 8; taken by sinkhorn_w1_1d when the tiles fit the GPU at once).

* Against Algorithm 1 on the CPU at fixed iteration counts, on the graded
  workload and on uneven meshes (tiles holding only x or only y points).
* Against the streaming fast sweeps at convergence (same plan to rounding)
  and against a batch member (the batch runs the streaming sweeps).
* The loop head's edge cases (no iteration, one iteration), determinism, and
  the bounded wait of its grid barrier (forced from the host with a wait
  bound of zero polls: every block leaves the loop, the call reports a HIP
  failure, the next call is unaffected).
"""
import numpy as np
import pytest

from oracle import clib
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

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
    # the check runs in FP32: each term |psi_old (K^T phi) - v| carries an
    # absolute error of a few 2^-24 v (the states themselves are FP32-accurate),
    # so the sum (total mass 1) is good to ~3e-7 absolute
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
    """The batch runs the streaming sweeps: the resident single call agrees
    with its member to rounding (FP32 relative 1e-7 on the cost)."""
    from paper_2605_26659_amd import finom_batch
    from test_gpu_batch import _alone, _desc_1d
    p = wl.config_batch_problem(7, 30000)
    d = _desc_1d(p, tol=1e-6, itr_max=5000)
    st, res = finom_batch([d], precision=1)
    ra, fa, ga = _alone(d, 1, resident=True)
    assert ra["fast"] == 2 and res[0]["fast"] == 1
    assert abs(ra["w1"] - res[0]["w1"]) <= 1e-6 * res[0]["w1"]
    assert abs(ra["iters"] - res[0]["iters"]) <= max(3, 0.01 * res[0]["iters"])


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
