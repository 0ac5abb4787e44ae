"""The linear-domain mode with the stored vector representation (precision 2):
section 2.2's r, eta, eta' and the recurrences of eq. p-DP / q-DP run as FP64
scans of affine maps, with no exponential or logarithm per iteration.

* One product against the oracle's instrumented representation product
  (orc_rep_matvec, pinned by the operation counts of section 2.3) and the
  dense definition, on meshes with ties, n != m, several tiles and a ragged
  tail, for every tile shape.
* Algorithm 1 in this mode against the oracle's converged references
  (tests/golden): the small workload (n = m = 512, eps 0.01, cap 2000) and the
  graded 2^20 workload at eps = 1e-2: same iteration count, W1, potentials.
* The refusal where the scalings would leave FP64 (diam / eps > 600).
"""
import json
from pathlib import Path

import numpy as np
import pytest

from oracle import clib, dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import check_slack, dev, host, rand_meshes, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_linear_product_matches_the_representation_oracle(cfg, monkeypatch):
    from paper_2605_26659_amd import finom_matvec
    monkeypatch.setenv("FINOM_TILE_CFG", str(cfg))
    for seed, n, m, eps in ((3, 5000, 3777, 0.05), (4, 777, 9001, 0.02), (5, 1, 300, 0.1), (6, 300, 1, 0.1)):
        print(f"linear product cfg={cfg} seed={seed} n={n} m={m} eps={eps}", flush=True)
        x, y = rand_meshes(seed, n, m, ties=True)
        psi = np.random.default_rng(seed + 10).uniform(0.1, 2.0, m)
        out = host(finom_matvec(dev(x), dev(y), eps, dev(psi), precision=2, domain=0))
        rep, _, _, _ = clib.rep_matvec(x, y, psi, eps)
        assert np.max(np.abs(out - rep) / rep) <= 1e-12
        if n * m <= 4e7:
            want = dense.matvec(x, y, psi, eps)
            assert np.max(np.abs(out - want) / want) <= 1e-12


def _golden(name):
    return json.loads((GOLDEN / name).read_text())


@pytest.mark.parametrize("name", ["small_1d_n512.json", "graded_1d_2p20_eps1e-2.json"])
def test_linear_solve_matches_the_oracle(name):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    gold = _golden(name)
    p = wl.config_small_1d() if name.startswith("small") else wl.config_graded_1d(eps=1e-2)
    assert (gold["n"], gold["eps"], gold["tol"], gold["itr_max"]) == (len(p.x), p.eps, p.tol, p.itr_max)
    print(f"linear solve {name}", flush=True)
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, p.tol, p.itr_max, precision=2)
    f, g = host(f), host(g)
    assert res["iters"] == gold["iters"]
    assert res["converged"] == (gold["err"] <= gold["tol"])
    assert abs(res["w1"] - gold["w1"]) <= 1e-10 * gold["w1"]
    # potentials within 1e-9 eps (below) put every scaling within 1e-9
    # relative, each term psi_j (K^T phi)_j within 2e-9, so the error of the
    # returned pair within 2e-9 sum(v) of the oracle's
    assert abs(res["marginal_err"] - gold["err"]) <= 2e-9 * p.v.sum()
    idx = np.asarray(gold["idx"])
    assert np.max(np.abs(f[idx] - np.asarray(gold["f"]))) / p.eps <= 1e-9
    assert np.max(np.abs(g[idx] - np.asarray(gold["g"]))) / p.eps <= 1e-9
    # marginals of the returned pair, recomputed by the oracle's recurrences
    t = clib.finom_logmatvec(p.y, p.x, f, p.eps)
    err_v = float(np.sum(np.abs(np.exp((g + t) / p.eps) - p.v)))
    assert abs(res["marginal_err"] - err_v) <= check_slack(g, t, p.eps, p.v)
    s = clib.finom_logmatvec(p.x, p.y, g, p.eps)
    assert float(np.sum(np.abs(np.exp((f + s) / p.eps) - p.u))) <= 1e-12


@pytest.mark.parametrize("n,m", [(1, 1), (1, 40), (40, 1), (3000, 700)])
def test_linear_solve_small_and_uneven(n, m):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    rng = np.random.default_rng(n * 7 + m)
    x, y = rand_meshes(n + m, n, m, ties=True)
    u = wl.normalise(rng.uniform(0.1, 1, n)); v = wl.normalise(rng.uniform(0.1, 1, m))
    res, f, g = sinkhorn_w1_1d(dev(x), dev(y), dev(u), dev(v), 0.02, 1e-8, 4000, precision=2)
    fo, go, ito, erro = clib.sinkhorn_1d(x, y, u, v, 0.02, 1e-8, 4000)
    assert res["iters"] == ito
    assert np.max(np.abs(host(f) - fo)) / 0.02 <= 1e-9
    assert np.max(np.abs(host(g) - go)) / 0.02 <= 1e-9


def test_linear_mode_refusals():
    torch = torch_cuda()
    from paper_2605_26659_amd import (FINOM_E_ARG, FinomError, dense_matvec, finom_matvec, sinkhorn_w1_1d,
                                      sinkhorn_w1_2d)
    p = wl.config_graded_1d(1 << 12, 1e-3)   # diam / eps = 1000
    with pytest.raises(FinomError) as e:
        sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, p.tol, 10, precision=2)
    assert e.value.status == FINOM_E_ARG
    x, y = dev(p.x), dev(p.y)
    w = torch.ones(len(p.y), dtype=torch.float64, device="cuda")
    with pytest.raises(FinomError):
        finom_matvec(x, y, 0.1, w, precision=2, domain=1)
    with pytest.raises(FinomError):
        dense_matvec(x, y, 0.1, w, precision=2, domain=0)
    q = wl.config_tanh_2d(side=16, eps=0.05)
    with pytest.raises(FinomError):
        sinkhorn_w1_2d(dev(q.x1), dev(q.y1), dev(q.x2), dev(q.y2), dev(q.u.ravel(order="F")),
                       dev(q.v.ravel(order="F")), q.eps, q.tol, 10, precision=2)
