"""FinomServer (HIP serving loop): continuous batching with admission by
device-memory footprint.

* Every completed request equals the single-problem solve of the same
  problem alone (bit for bit: the tile plan depends only on the problem, and
  1D FP32 requests that fit the resident solver take it, as single calls do),
  whatever else shares its rounds.
* A budget that holds only a few requests at a time: the rest waits in
  arrival order and still completes.
* A request larger than the whole budget is refused at submission; an
  invalid one completes with its validation status.
"""
import time

import numpy as np
import pytest

from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host
from test_gpu_batch import _alone, _assert_same, _desc_1d, _desc_2d

pytestmark = pytest.mark.gpu


def _drain(srv, n, timeout_s=60.0):
    out = []
    t0 = time.time()
    while len(out) < n:
        out += srv.poll(256, wait_ms=50)
        assert time.time() - t0 < timeout_s, f"{len(out)} of {n} completed"
    return out


def _mixed_requests():
    descs = []
    for i, n in enumerate([300, 2500, 9000, 40000, 700, 123]):
        descs.append(_desc_1d(wl.config_batch_problem(50 + i, n), tol=1e-6, itr_max=3000))
    descs.append(_desc_2d(wl.config_tanh_2d(side=64, eps=1e-2), tol=1e-6, itr_max=2000))
    descs.append(_desc_2d(wl.paper_random_2d(16, iters=80), tol=0.0, itr_max=80))
    descs.append(_desc_1d(wl.config_graded_1d(5000, 1e-2), tol=1e-6, itr_max=3000))
    return descs


@pytest.mark.parametrize("precision", [0, 1])
def test_requests_equal_alone_solves(precision):
    from paper_2605_26659_amd import FinomServer
    descs = _mixed_requests()
    with FinomServer(1 << 30, precision=precision) as srv:
        tickets = {}
        for i, d in enumerate(descs):
            tickets[srv.submit(d)] = i
            time.sleep(0.002 * (i % 3))   # staggered arrivals join running rounds
        done = _drain(srv, len(descs))
        st = srv.stats()
    assert st["completed"] == len(descs) and st["submitted"] == len(descs)
    for c in done:
        d = descs[tickets[c["ticket"]]]
        assert c["problem"] is d
        assert 0.0 <= c["queue_ms"] <= c["latency_ms"]
        ra, fa, ga = _alone(d, precision, resident=True)
        _assert_same(c, d, ra, fa, ga)


def test_small_budget_queues_in_arrival_order():
    from paper_2605_26659_amd import FinomServer, finom_footprint
    descs = [_desc_1d(wl.config_batch_problem(200 + i, 4000 + 500 * i), tol=1e-6, itr_max=3000)
             for i in range(8)]
    fp = max(finom_footprint(d, precision=1) for d in descs)
    with FinomServer(int(2.5 * fp), precision=1) as srv:
        tk = [srv.submit(d) for d in descs]
        done = _drain(srv, len(descs))
        st = srv.stats()
    assert sorted(c["ticket"] for c in done) == sorted(tk)
    assert st["admitted"] == len(descs)
    assert st["hbm_used"] == 0
    for c in done:
        d = descs[tk.index(c["ticket"])]
        ra, fa, ga = _alone(d, 1, resident=True)
        _assert_same(c, d, ra, fa, ga)


def test_refusals_and_validation_statuses():
    from paper_2605_26659_amd import (FINOM_E_ADMIT, FINOM_E_UNSORTED, FinomError, FinomServer,
                                      finom_footprint)
    big = _desc_1d(wl.config_batch_problem(1, 60000))
    p = wl.config_batch_problem(2, 500)
    xb = p.x.copy(); xb[[0, 1]] = xb[[1, 0]]
    bad = _desc_1d(wl.Problem1D(xb, p.y, p.u, p.v, p.eps, 1e-6, 100))
    good = _desc_1d(p, tol=1e-6, itr_max=3000)
    budget = 4 * finom_footprint(good)
    assert finom_footprint(big) > budget
    with FinomServer(budget) as srv:
        with pytest.raises(FinomError) as e:
            srv.submit(big)
        assert e.value.status == FINOM_E_ADMIT
        tb = srv.submit(bad)
        tg = srv.submit(good)
        done = {c["ticket"]: c for c in _drain(srv, 2)}
        st = srv.stats()
    assert st["rejected"] == 1
    assert done[tb]["status"] == FINOM_E_UNSORTED
    assert done[tg]["converged"]


def test_2d_requests_finishing_in_different_rounds():
    """2D FP32 requests on the extended-state loop admitted together, with
    iteration counts far apart: the rounds after each completion run without
    a rebuild (no new admission), and the completed requests' memory is freed
    by then. Every result still equals its solve alone."""
    from paper_2605_26659_amd import FinomServer
    descs = [_desc_2d(wl.config_tanh_2d(side=s, eps=e), tol=1e-6, itr_max=it)
             for s, e, it in ((64, 1e-2, 40), (96, 1e-2, 2000), (80, 3e-3, 160), (128, 3e-3, 3000),
                              (72, 1e-2, 8))]
    with FinomServer(1 << 30, precision=1, graph_iters=8) as srv:
        tk = [srv.submit(d) for d in descs]
        done = _drain(srv, len(descs))
        st = srv.stats()
    assert st["completed"] == len(descs) and st["admitted"] == len(descs)
    assert st["rounds"] > 2
    iters = set()
    for c in done:
        d = descs[tk.index(c["ticket"])]
        ra, fa, ga = _alone(d, 1)
        assert ra["fast"] == 4
        _assert_same(c, d, ra, fa, ga)
        iters.add(c["iters"])
    assert len(iters) >= 3
