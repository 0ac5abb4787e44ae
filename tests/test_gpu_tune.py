"""Tile-shape autotuner: every shape gives the same products within rounding
(so tuning never changes what is computed beyond summation order), the
tuner's table is used by later calls, and its cache file round-trips.
Runs after the other GPU tests: tuning changes the process-wide table."""
import os

import numpy as np
import pytest

from oracle import clib
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

pytestmark = pytest.mark.gpu


def test_autotune_table_and_cache(tmp_path):
    from paper_2605_26659_amd import finom_autotune, finom_tile_config, sinkhorn_w1_1d
    path = str(tmp_path / "tune.txt")
    finom_autotune(1, path)
    lines = open(path).read().split("\n")
    assert lines[0] == "finom-tune 1"
    rows = [tuple(map(int, l.split())) for l in lines[1:] if l.strip()]
    table = {c: v for p, c, v in rows if p == 1}
    assert sorted(table) == list(range(13))
    assert all(0 <= v < 5 for v in table.values())   # five tile shapes
    for c in range(13):
        assert finom_tile_config(1, 512 << c) == table[c]
    # a second call reads the cache
    finom_autotune(1, path)
    assert {c: finom_tile_config(1, 512 << c) for c in range(13)} == table
    # solves after tuning still match the oracle
    p = wl.config_batch_problem(7, 3000)
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, 0.0, 30,
                               precision=0)
    fo, go, _, _ = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, 30)
    assert np.max(np.abs(host(f) - fo)) / p.eps <= 1e-9
