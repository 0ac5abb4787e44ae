"""The FP32 fast sweeps (tiles inside the FP32 exponent range, plain FP32
tile scans) against the oracle and against the general extended-exponent
sweeps.

* Lines that pass the static range bound run the fast sweeps (reported in
  the result), lines that fail it run the general ones; both agree with
  Algorithm 1 on the CPU at a fixed iteration count.
* Carries that dominate a tile (mass far away from the tile) and a single
  tile per line.
* Fast and general sweeps converge to the same plan at tolerance.
"""
import numpy as np
import pytest

from oracle import clib
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

pytestmark = pytest.mark.gpu

TOL_ITER = 2e-5     # |f - f_oracle| / eps after a few dozen FP32 iterations (as the 2^20 test)


def _solve(p, precision=1, tol=None, itr_max=None):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps,
                               p.tol if tol is None else tol,
                               p.itr_max if itr_max is None else itr_max, precision=precision)
    return res, host(f), host(g)


def _against_oracle(p, iters, tol=TOL_ITER):
    res, f, g = _solve(p, tol=0.0, itr_max=iters)
    fo, go, ito, erro = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, iters)
    assert res["iters"] == iters
    df = np.max(np.abs(f - fo)) / p.eps
    dg = np.max(np.abs(g - go)) / p.eps
    assert df <= tol and dg <= tol, (df, dg)
    return res


@pytest.mark.parametrize("n,eps,fast", [(3000, 1e-1, True), (3000, 1e-2, False), (1 << 16, 1e-2, True)])
def test_graded_lines_match_oracle_on_either_path(n, eps, fast, monkeypatch):
    """n = 3000, eps = 1e-2: a tile of ~1000 columns spans ~0.67 near x = 1,
    2 kappa span ~ 193 binary orders > the bound, so the general sweeps run
    (the streaming sweeps: the resident solver is off)."""
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    p = wl.config_graded_1d(n, eps)
    res = _against_oracle(p, 40)
    assert bool(res["fast"]) == fast


def test_dominant_carries():
    """u on [0, 0.1], v on [0.9, 1]: every row's sum is carried in from tiles
    far away, and the tiles' own terms are negligible against the carry."""
    n = 1 << 15
    x = np.linspace(0.0, 1.0, n)
    y = np.linspace(0.0, 1.0, n) + 0.3 / n
    u = np.where(x < 0.1, 1.0, 1e-9); u /= u.sum()
    v = np.where(y > 0.9, 1.0, 1e-9); v /= v.sum()
    p = wl.Problem1D(x, y, u, v, 2e-2, 0.0, 30)
    res = _against_oracle(p, 30)
    assert res["fast"]


def test_ineligible_line_runs_general_sweeps(monkeypatch):
    """Coarse mesh and small eps: a tile spans thousands of binary orders (the
    streaming sweeps: the resident solver is off)."""
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    p = wl.config_batch_problem(3, 300)
    p = wl.Problem1D(p.x, p.y, p.u, p.v, 1e-3, 0.0, 30)
    res = _against_oracle(p, 30)
    assert not res["fast"]


def test_fast_and_general_converge_to_the_same_plan(monkeypatch):
    p = wl.config_graded_1d(1 << 16, 1e-2)
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    r1, f1, g1 = _solve(p, tol=1e-6, itr_max=20000)
    monkeypatch.setenv("FINOM_FAST", "0")
    r0, f0, g0 = _solve(p, tol=1e-6, itr_max=20000)
    r64, f64, g64 = _solve(p, tol=1e-6, itr_max=20000, precision=0)
    assert r1["fast"] == 1 and not r0["fast"]
    assert r1["converged"] and r0["converged"]
    assert abs(r1["w1"] - r0["w1"]) <= 1e-6 * r0["w1"]
    # each FP32 path stops where the FP64 check of its own pair passes. The
    # fast sweeps' pairs track the FP64 loop's error to a few %: within
    # max(3, 1 %) of its count. The general sweeps' FP32-mantissa exp2 / log2
    # leave an error floor of about 2.5e-7 on unit mass, so their FP64 error
    # reaches tol = 1e-6 when the FP64 loop's is near 0.75e-6: ln(1/0.75) / the
    # asymptotic rate more iterations (~5 at eps = 1e-2), within max(8, 3 %).
    assert abs(r1["iters"] - r64["iters"]) <= max(3, 0.01 * r64["iters"]), (r1["iters"], r64["iters"])
    assert abs(r0["iters"] - r64["iters"]) <= max(8, 0.03 * r64["iters"]), (r0["iters"], r64["iters"])
    assert np.max(np.abs(f1 - f0)) / p.eps <= 1e-4


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4])
def test_every_tile_shape_on_the_fast_path(cfg, monkeypatch):
    """Every tile shape against the oracle, on lines of 80000 and 600002
    elements: the second has more tiles than two per thread of a block for
    256 x 4 and 128 x 4 (the kernel variant with remainder loops over the
    carries and the decision partials)."""
    monkeypatch.setenv("FINOM_TILE_CFG", str(cfg))
    monkeypatch.setenv("FINOM_RESIDENT", "0")
    for n in (40000, 300001):
        p = wl.config_graded_1d(n, 1e-2)
        res = _against_oracle(p, 24)
        assert res["fast"]
