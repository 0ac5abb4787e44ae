#!/usr/bin/env python3
"""Throughput benchmark: FINOM Sinkhorn solves on one MI355X.

Workload (one step = one full solve of the hot path: setup, Algorithm 1 loop
to tolerance, <C, Gamma>): 1D entropic W1, n = m = 2^20 graded meshes
(x = t^2, y = Chebyshev-clustered), 3-component Gaussian-mixture masses with a
1e-6 floor, eps = 1e-3, tol 1e-6, FP32-mantissa scans with FP64 state.

Prints one JSON line: grid-point iterations per second (grid points =
(n + m)/2, iterations = completed Sinkhorn iterations), p50/p99 solve
latency, the FP64-scan mode and the dense baseline at the same workload, the
roofline of the dominant kernel and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per grid point per iteration with FP64 state and
# coordinates: the K^T phi half reads f, x, y, v (as log2 v) and g_old and
# writes g (16n + 32m); the K psi half reads g, y, x, u (as log2 u) and
# writes f (24n + 16m).
BYTES_KT = (16, 32)
BYTES_K = (24, 16)

# The resident solver (one cooperative launch per solve, state on chip) is
# bound by arithmetic and latency, not by HBM. Its algorithmic work is counted
# in lane operations per grid point per iteration: every FP32 / FP64 add,
# multiply, fused multiply-add, ldexp, reciprocal, frexp and conversion
# counts once, integer exponent arithmetic does not. An x point costs 3 as a
# column, 4 in the column scan and 17 as a row; a y point the same plus 6 for
# the marginal check: 54 per (x, y) pair, i.e. per grid point.
OPS_PER_PT_ITER = 54
# One lane operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz (packed FP32 instructions are not used).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# HBM traffic measured with rocprofv3 FETCH_SIZE and WRITE_SIZE at
# n = m = 2^20 (KiB per dispatch), each scaled by the counter's reading for a
# plain device copy of known size: for the resident kernel per launch (one
# solve at eps = 1e-3, tol 1e-6), for the streaming sweeps per executed sweep
# (mean of the two variants). The loops replay whole graphs, and the sweeps
# after a stop exit at once, so a dispatch mean is scaled by dispatches /
# executed sweeps of the profiled run. Valid only for the kernel sources whose
# digest is recorded beside them; after any change to those sources the
# traffic is null.
FETCH_SCALE = 262144 / 131084
WRITE_SCALE = 262144 / 262144
TRAFFIC_RESIDENT = {"sources_sha256": "f987251bc05ecf3aa06c84eec559cd50e57b120a468c3c99c9d7d178a6a3581c",
                    "fetch_kib": 452901.0, "write_kib": 188601.0, "n": 1 << 20}
# The resident kernel's instruction counters (rocprofv3 --pmc SQ_INSTS_VALU,
# SQ_WAVES, per launch, same workload and sources as TRAFFIC_RESIDENT) and the
# average launch of that run: VALU wave instructions issued, against one per
# SIMD per 4 clocks (a wave64 instruction occupies a 16-lane SIMD for 4).
RESIDENT_VALU = {"sources_sha256": TRAFFIC_RESIDENT["sources_sha256"], "valu_insts": 1.29069e10,
                 "waves": 4096, "launch_us": 27832.53, "iters": 3117, "n": 1 << 20}
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4     # wave instructions per second
TRAFFIC_STREAM = {"sources_sha256": "897fa852bd2807115cca2e6024c5992448a766042d1bad9cc5a2105c92f2d4de",
                  "fetch_kib": (21545.0 + 17655.4) / 2 * 9936 / 9426,
                  "write_kib": (8146.69 + 8186.06) / 2 * 9936 / 9426, "n": 1 << 20}
# the streaming fast sweeps at n = m = 2^24 (beyond the Infinity Cache), per
# sweep (mean of the two variants, plus the carries pre-pass each sweep runs)
TRAFFIC_STREAM_2P24 = {"sources_sha256": "897fa852bd2807115cca2e6024c5992448a766042d1bad9cc5a2105c92f2d4de",
                       "fetch_kib": ((239037.0 + 191924.0) / 2 + 62.36) * 160 / 104,
                       "write_kib": ((90425.1 + 89067.5) / 2 + 84.02) * 160 / 104, "n": 1 << 24}
# the FP64-scan loop's general sweeps, per sweep (mean of the two variants)
TRAFFIC_FP64 = {"sources_sha256": "897fa852bd2807115cca2e6024c5992448a766042d1bad9cc5a2105c92f2d4de",
                "fetch_kib": (26881.8 + 18799.6) / 2 * 9456 / 9381,
                "write_kib": (8732.28 + 8657.67) / 2 * 9456 / 9381, "n": 1 << 20}
RESIDENT_SOURCES = ("paper_2605_26659_amd/csrc/finom_resident.hpp",
                    "paper_2605_26659_amd/csrc/finom_fast.hpp",
                    "paper_2605_26659_amd/csrc/finom_kernels.hpp",
                    "paper_2605_26659_amd/csrc/finom_device.hpp",
                    "paper_2605_26659_amd/csrc/finom_types.hpp")
STREAM_SOURCES = RESIDENT_SOURCES[1:]
# The plan export (k_plan_export<true>) on the 160 x 160 paper workload, per
# launch; `n` is the plan's row count.
TRAFFIC_PLAN = {"sources_sha256": "81b9b566466ba8e5e64e2344982331be9e619045dded8b616bc7067ae99449a2",
                "fetch_kib": 1701.02, "write_kib": 5120010.0, "n": 25600}
PLAN_SOURCES = ("paper_2605_26659_amd/csrc/finom_plan.hip",)
# The 2D FP32 loop on extended-number state (1024 x 1024 tanh): per iteration
# the two fused launches (k_line_pair_ext: psi rows, phi columns) read the
# intermediate, the masses and (psi rows) the checked psi, and write the new
# state and the next intermediate, 8 bytes each: 40 + 32 bytes per grid point.
BYTES_2D_ITER = 72
# Measured per executed iteration (both launches; 1392 dispatches each for
# 3 x 401 iterations):
TRAFFIC_2D = {"sources_sha256": "bcc64cacd4602208390755fecd1d818826ac16f345f0533ffdc9bbbbc98302b9",
              "fetch_kib": (10830.1 + 7303.75) * 1392 / 1203, "write_kib": (14237.0 + 14159.5) * 1392 / 1203,
              "n": 1 << 20}
LINE2D_SOURCES = ("paper_2605_26659_amd/csrc/finom_line_ext.hpp",) + STREAM_SOURCES


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden(name):
    """A converged reference result of the oracle (tests/golden, written by
    oracle/make_goldens.py), or None if the file is absent."""
    path = os.path.join(GOLDEN_DIR, name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def vs_oracle(res, name):
    """Error of a result against the oracle's converged run of the same
    workload: W1 relative, iteration counts, the oracle's own marginal error."""
    gd = golden(name)
    if gd is None:
        return None
    return {"w1_rel_err": abs(res["w1"] - gd["w1"]) / gd["w1"], "w1_oracle": gd["w1"],
            "iters_oracle": gd["iters"], "iters_diff": int(res["iters"]) - int(gd["iters"]),
            "marginal_err": res["marginal_err"], "marginal_err_oracle": gd["err"],
            "golden": f"tests/golden/{name}"}


def graded_golden(eps):
    """The reference file of the graded 2^20 workload at this eps, if any."""
    return {1e-2: "graded_1d_2p20_eps1e-2.json", 1e-3: "graded_1d_2p20_eps1e-3.json"}.get(eps, "none.json")


def state_repr(res):
    """What the loop kept as its iteration state (result field `fast`)."""
    if res.get("fast", 0) in (1, 2, 3, 4):
        return "ext-f32 scalings (FP32 mantissa + int32 exponent)"
    return "f64 log potentials"


def sources_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(t, paths, n):
    if t["sources_sha256"] is None or n != t["n"] or sources_digest(paths) != t["sources_sha256"]:
        return None
    return 1024.0 * (t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the 4096-problem batch")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the small 1D, eps = 1e-2 and 2D 1024^2 configurations")
    ap.add_argument("--serving", action="store_true",
                    help="full serving sweep (several arrival rates and the nominal 2000/s)")
    ap.add_argument("--no-serving", action="store_true", help="skip the short serving sample")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--random-3d-only", action="store_true",
                    help="only the 3D 128^3 record (two warm-ups and one timed solve)")
    ap.add_argument("--tanh-2d-only", action="store_true",
                    help="only the 2D 1024 x 1024 tanh-mesh record (one warm-up and one timed solve)")
    ap.add_argument("--stream-2p24-only", action="store_true",
                    help="only the 2^24 streaming record (a warm-up and one timed 100-iteration solve)")
    ap.add_argument("--plan-only", action="store_true",
                    help="only the plan export / plan difference record (--steps launches each)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2605_26659_amd", "tune_gfx950.txt"),
                    help="tile-shape table: read if present, else tuned here and written")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized FP64 buffer 10 times (counter calibration)")
    return ap.parse_args()


def cpu_baseline(prob, seconds):
    """The oracle timed on host cores on a bounded sample of the workload.

    kind 'oracle': the dense FP64 definition (eps ln K e^{g/eps}, OpenMP over
    rows) on as many sampled rows as fit the time budget; one Sinkhorn
    iteration needs n + m such rows, so grid-pt*iters/s = rows/s * points /
    (n + m). Also times Algorithm 1 on the CPU (single thread) for a few
    iterations of the full workload.
    """
    from oracle import clib
    clib.build(force=False)
    threads = min(16, os.cpu_count() or 1)
    n, m = len(prob.x), len(prob.y)
    g = prob.eps * np.log(prob.v)
    rows = 64
    t_used = 0.0
    done_rows = 0
    rng = np.random.default_rng(0)
    while t_used < seconds * 0.5:
        idx = np.sort(rng.integers(0, n, rows))
        t0 = time.perf_counter()
        clib.dense_logmatvec(prob.x, prob.y, g, prob.eps, rows=idx, threads=threads)
        dt = time.perf_counter() - t0
        t_used += dt
        done_rows += rows
        rows = min(rows * 2, 1 << 14)
    pts = 0.5 * (n + m)
    dense_rate = done_rows / t_used * pts / (n + m)
    # Algorithm 1 on the CPU: a few iterations on the full problem
    iters = 1
    t0 = time.perf_counter()
    while True:
        clib.sinkhorn_1d(prob.x, prob.y, prob.u, prob.v, prob.eps, 0.0, iters)
        dt = time.perf_counter() - t0
        if dt > seconds * 0.3 or iters >= 64:
            break
        iters *= 2
        t0 = time.perf_counter()
    alg1_rate = pts * iters / dt
    return {
        "value": dense_rate, "unit": "grid-pt*iters/s", "cores": threads, "kind": "oracle",
        "sample": f"dense FP64 oracle, {done_rows} sampled rows x {m} columns of the "
                  f"n=m={n} graded workload in {t_used:.1f} s",
        "cpu_algorithm1": {"value": alg1_rate, "unit": "grid-pt*iters/s", "cores": 1,
                           "sample": f"{iters} iterations of Algorithm 1 (FP64 log-form "
                                     f"recurrences, C) on the full workload in {dt:.2f} s"},
        "cpu_model": _cpu_model(),
        "host_cpu_count": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "threads_used": threads,
    }


def bench_batch(precision):
    """The uneven batch: 4096 problems, n = m log-uniform in [256, 65536],
    eps log-uniform in [1e-3, 1e-1], tol 1e-6, cap 20000, one finom_batch
    call. Throughput = sum over problems of points x iterations / time."""
    import torch
    from paper_2605_26659_amd import finom_batch, problem_1d, workloads as wl
    probs = wl.config_batch()
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    descs = [problem_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, p.tol, p.itr_max)
             for p in probs]
    torch.cuda.synchronize()
    out = {}
    for rep in range(2):      # the first call also warms the workspace
        t0 = time.perf_counter()
        st, res = finom_batch(descs, precision=precision)
        wall = time.perf_counter() - t0
    work = float(sum(0.5 * (len(p.x) + len(p.y)) * r["iters"] for p, r in zip(probs, res)))
    loop_s = max(r["loop_ms"] for r in res) * 1e-3
    its = np.array([r["iters"] for r in res])
    # the same problems solved one by one with the single-problem entry point
    # in FP64 (a fixed sample: every 16th problem)
    from paper_2605_26659_amd import sinkhorn_w1_1d
    idx = list(range(0, len(probs), 16))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w_alone = 0.0
    for i in idx:
        d = descs[i]
        r, _, _ = sinkhorn_w1_1d(d["x1"], d["x2"], d["u"], d["v"], d["eps"], d["tol"], d["itr_max"],
                                 precision=0, want_potentials=False)
        w_alone += 0.5 * (d["x1"].numel() + d["x2"].numel()) * r["iters"]
    alone_rate = w_alone / (time.perf_counter() - t0)
    out = {"value": work / wall, "unit": "grid-pt*iters/s", "problems": len(probs),
           "points": float(sum(len(p.x) for p in probs)), "wall_s": wall,
           "loop_s": loop_s, "loop_rate": work / loop_s,
           "iters_mean": float(its.mean()), "iters_max": int(its.max()),
           "converged": int(sum(r["converged"] for r in res)), "status": st,
           "scan_mantissa": "fp32" if precision == 1 else "fp64",
           "per_problem_fp64_alone": {"value": alone_rate, "unit": "grid-pt*iters/s",
                                      "sample": f"{len(idx)} problems (every 16th), one "
                                                "sinkhorn_w1_1d call each, FP64 scans"},
           "note": "wall time of the call (setup, iteration, costs); loop_rate excludes "
                   "setup and cost"}
    return out


def bench_tanh_2d(precision):
    """The 2D 1024 x 1024 tanh-mesh workload (eps = 5e-3, tol 1e-6): one timed
    solve after two warm-up solves."""
    import torch
    from paper_2605_26659_amd import sinkhorn_w1_2d, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    p = wl.config_tanh_2d(1024)
    args2 = (dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2), dev(p.u.ravel(order="F")),
             dev(p.v.ravel(order="F")), p.eps, p.tol, p.itr_max)
    for _ in range(2):   # as for the headline: the first grows the workspace
        sinkhorn_w1_2d(*args2, precision=precision, want_potentials=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, _, _ = sinkhorn_w1_2d(*args2, precision=precision, want_potentials=False)
    dt = time.perf_counter() - t0
    dense2d = bench_dense_2d(p, r["iters"], p.points * r["iters"] / dt)
    roof = None
    if r["fast"] == 4:
        it_s = r["loop_ms"] * 1e-3 / max(1, r["iters"])
        gbs = BYTES_2D_ITER * p.points / it_s / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "traffic": measured_traffic(TRAFFIC_2D, LINE2D_SOURCES, p.points),
                "kernel": "k_line_pair_ext<256, 4> x 2 per iteration (psi rows with the check, phi columns "
                          "after the decision)", "iteration_us": it_s * 1e6,
                "algorithmic_bytes_per_iteration": BYTES_2D_ITER * p.points}
    return {"value": p.points * r["iters"] / dt, "unit": "grid-pt*iters/s", "roofline": roof,
            "solve_ms": dt * 1e3, "iters": r["iters"], "w1": r["w1"],
            "marginal_err": r["marginal_err"], "converged": r["converged"], "dense_2d": dense2d,
            "loop_ms": r["loop_ms"], "iteration_us": r["loop_ms"] * 1e3 / max(1, r["iters"]),
            "scan_mantissa": "fp32" if precision == 1 else "fp64", "state": state_repr(r),
            "resumes": r["resumes"], "vs_oracle": vs_oracle(r, "tanh_2d_1024_eps5e-3.json"),
            "workload": "1024 x 1024 tanh mesh (beta 2.5), 4-component 2D GMM masses, "
                        "eps=5e-3, tol=1e-6"}


def bench_dense_2d(p, iters, finom_rate):
    """The 2D dense baselines on the same workload: one product timed with HIP
    events on the stream it runs on; an iteration is two products, and the
    iterates equal FINOM's, so time to tolerance = 2 x product x FINOM's
    iteration count. Per axis: two FP64 matrix products on the matrix cores
    (roofline against the FP64 matrix peak); full: the (NM)^2 product with
    one exponential per kernel entry."""
    import torch
    from paper_2605_26659_amd import dense_matvec_2d
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    x1, y1, x2, y2 = dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2)
    g = dev((p.eps * np.log(p.v)).ravel(order="F"))
    out = torch.empty(p.u.size, dtype=torch.float64, device="cuda")
    n1, m1 = p.u.shape
    n2, m2 = p.v.shape
    res = {}
    for full, reps in ((False, 5), (True, 1)):
        dense_matvec_2d(x1, y1, x2, y2, p.eps, g, out, full=full)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            dense_matvec_2d(x1, y1, x2, y2, p.eps, g, out, full=full)
        e1.record(s)
        torch.cuda.synchronize()
        prod_s = e0.elapsed_time(e1) * 1e-3 / reps
        rate = p.points / (2.0 * prod_s)
        rec = {"product_s": prod_s, "per_iteration_s": 2 * prod_s, "time_to_tol_s": 2 * prod_s * iters,
               "value": rate, "unit": "grid-pt*iters/s", "finom_speedup": finom_rate / rate}
        if not full:
            flops = 2.0 * (n1 * n2 * m2 + n1 * m2 * m1)
            tf = flops / prod_s / 1e12
            rec["roofline"] = {"bound": "mfma", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
                               "frac": tf / 78.6, "kernel": "k_dense2d_gemm (FP64 MFMA 16x16x4) x 2 "
                                                            "+ the shift kernels", "flops_per_product": flops}
        res["full_on_the_fly" if full else "per_axis_mfma"] = rec
    return res


def bench_random_3d(precision):
    """d = 3 tensor meshes, 128^3 grid points per side, 200 iterations: one
    timed solve after two warm-ups."""
    import torch
    from paper_2605_26659_amd import sinkhorn_w1_nd, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    xs, xt, u3, v3, eps3, its3 = wl.paper_random_nd((128, 128, 128), (128, 128, 128), iters=200)
    args3 = ([dev(a) for a in xs], [dev(a) for a in xt], dev(u3.ravel(order="F")), dev(v3.ravel(order="F")),
             eps3, 0.0, its3)
    # two warm-up solves, as for the headline (the first grows the stream's
    # workspace; later solves allocate nothing)
    for _ in range(2):
        sinkhorn_w1_nd(*args3, precision=precision, want_potentials=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, _, _ = sinkhorn_w1_nd(*args3, precision=precision, want_potentials=False)
    dt = time.perf_counter() - t0
    pts3 = 0.5 * (u3.size + v3.size)
    return {"value": pts3 * r["iters"] / dt, "unit": "grid-pt*iters/s", "solve_ms": dt * 1e3,
            "iters": r["iters"], "w1": r["w1"], "marginal_err": r["marginal_err"],
            "loop_ms": r["loop_ms"], "sweep_us": r["loop_ms"] * 1e3 / (6 * r["iters"]),
            "scan_mantissa": "fp32" if precision == 1 else "fp64",
            "workload": "3D 128^3 sorted U[0,1] axes, masses U[0,1], eps=0.01, "
                        "200 iterations (section 4.3's recipe in three dimensions)"}


def bench_other_configs(precision):
    """The other single-problem configurations, one timed solve each after a
    warm-up: the headline workload on the streaming sweeps, the small 1D
    correctness case (FP64 scans, tol 1e-9, cap 2000), the graded 1D workload
    at eps = 1e-2, and the 2D 1024 x 1024 tanh mesh (eps = 5e-3, tol 1e-6)."""
    import torch
    from paper_2605_26659_amd import sinkhorn_w1_1d, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = {}

    def run1d(p, prec):
        x, y, u, v = dev(p.x), dev(p.y), dev(p.u), dev(p.v)
        sinkhorn_w1_1d(x, y, u, v, p.eps, p.tol, p.itr_max, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, _, _ = sinkhorn_w1_1d(x, y, u, v, p.eps, p.tol, p.itr_max, precision=prec)
        dt = time.perf_counter() - t0
        return {"value": p.points * r["iters"] / dt, "unit": "grid-pt*iters/s", "solve_ms": dt * 1e3,
                "iters": r["iters"], "w1": r["w1"], "marginal_err": r["marginal_err"],
                "converged": r["converged"], "scan_mantissa": "fp32" if prec == 1 else "fp64",
                "state": state_repr(r), "resumes": r["resumes"],
                "resident": r["fast"] == 2, "loop_ms": r["loop_ms"]}

    # the headline workload on the streaming sweeps (the path taken by
    # problems too large for the resident solver, and by batches)
    if precision == 1:
        old = os.environ.get("FINOM_RESIDENT")
        os.environ["FINOM_RESIDENT"] = "0"
        try:
            p = wl.config_graded_1d(1 << 20, 1e-3)
            r = run1d(p, 1)
        finally:
            if old is None:
                os.environ.pop("FINOM_RESIDENT", None)
            else:
                os.environ["FINOM_RESIDENT"] = old
        n = len(p.x)
        per_sweep = ((BYTES_KT[0] + BYTES_K[0]) * n + (BYTES_KT[1] + BYTES_K[1]) * n) / 2.0
        sweep_s = r.pop("loop_ms") * 1e-3 / (2 * r["iters"] + 1)
        gbs = per_sweep / sweep_s / 1e9
        r["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured_traffic(TRAFFIC_STREAM, STREAM_SOURCES, n),
                         "avg_sweep_us": sweep_s * 1e6, "algorithmic_bytes_per_sweep": per_sweep}
        out["graded_1d_streaming"] = r
    p = wl.config_small_1d()
    out["small_1d_n512"] = run1d(p, 0)
    out["small_1d_n512"]["workload"] = "n=m=512 sorted U(0,1), masses U(0.1,1), eps=0.01, tol=1e-9, cap 2000"
    out["small_1d_n512"]["vs_oracle"] = vs_oracle(out["small_1d_n512"], "small_1d_n512.json")
    p = wl.config_graded_1d(1 << 20, 1e-2)
    out["graded_1d_eps1e-2"] = run1d(p, precision)
    out["graded_1d_eps1e-2"]["vs_oracle"] = vs_oracle(out["graded_1d_eps1e-2"], "graded_1d_2p20_eps1e-2.json")
    out["tanh_2d_1024"] = bench_tanh_2d(precision)
    out["random_3d_128"] = bench_random_3d(precision)
    out["graded_1d_2p24_streaming"] = bench_stream_2p24(precision)
    out.update(bench_linear())
    return out


def bench_stream_2p24(precision, iters=100):
    """The graded 1D workload at n = m = 2^24 (eps = 1e-3): too large for the
    resident solver, so it runs the streaming sweeps, with a working set of
    about 1.5 GB, far beyond the 256 MB Infinity Cache. A fixed count of
    iterations (tol 0) after a warm-up solve; the HBM roofline of its sweeps
    from the loop's HIP events."""
    import torch
    from paper_2605_26659_amd import sinkhorn_w1_1d, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    n = 1 << 24
    p = wl.config_graded_1d(n, 1e-3, tol=0.0, itr_max=iters)
    x, y, u, v = dev(p.x), dev(p.y), dev(p.u), dev(p.v)
    del p
    sinkhorn_w1_1d(x, y, u, v, 1e-3, 0.0, 4, precision=precision, want_potentials=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, _, _ = sinkhorn_w1_1d(x, y, u, v, 1e-3, 0.0, iters, precision=precision, want_potentials=False)
    dt = time.perf_counter() - t0
    per_sweep = ((BYTES_KT[0] + BYTES_K[0]) * n + (BYTES_KT[1] + BYTES_K[1]) * n) / 2.0
    sw_s = r["loop_ms"] * 1e-3 / max(1, r["sweeps"])
    gbs = per_sweep / sw_s / 1e9
    return {"value": n * r["iters"] / dt, "unit": "grid-pt*iters/s", "solve_ms": dt * 1e3,
            "iters": r["iters"], "w1": r["w1"], "marginal_err": r["marginal_err"], "state": state_repr(r),
            "fast": r["fast"], "loop_ms": r["loop_ms"],
            "workload": "graded 1D n=m=2^24 (x=t^2, y=Chebyshev), 3-GMM masses, eps=1e-3, "
                        f"{iters} iterations (tol 0)",
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured_traffic(TRAFFIC_STREAM_2P24, STREAM_SOURCES, n),
                         "kernel": "k_sweep_fast, both half-iteration variants, averaged over the loop",
                         "avg_sweep_us": sw_s * 1e6, "algorithmic_bytes_per_sweep": per_sweep}}


def bench_linear():
    """The linear-domain mode (precision 2: the stored vector representation,
    FP64 affine-map scans, no exponential per iteration) on the small 1D case
    and on the graded 2^20 workload at eps = 1e-2 (diam / eps = 100; at
    eps = 1e-3 the mode refuses the mesh). One timed solve after a warm-up."""
    import torch
    from paper_2605_26659_amd import sinkhorn_w1_1d, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = {}
    for key, p, gold in (("small_1d_n512_linear", wl.config_small_1d(), "small_1d_n512.json"),
                         ("graded_1d_eps1e-2_linear", wl.config_graded_1d(1 << 20, 1e-2),
                          "graded_1d_2p20_eps1e-2.json")):
        x, y, u, v = dev(p.x), dev(p.y), dev(p.u), dev(p.v)
        sinkhorn_w1_1d(x, y, u, v, p.eps, p.tol, p.itr_max, precision=2, want_potentials=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, _, _ = sinkhorn_w1_1d(x, y, u, v, p.eps, p.tol, p.itr_max, precision=2, want_potentials=False)
        dt = time.perf_counter() - t0
        n, m = len(p.x), len(p.y)
        # per iteration: K^T phi reads phi, eta, eta' (columns x) and r, v,
        # psi_old (rows y) and writes psi; K psi reads psi, eta, eta'
        # (columns y) and r, u (rows x) and writes phi: 48 n + 56 m bytes
        per_sweep = (48.0 * n + 56.0 * m) / 2.0
        sw_s = r["loop_ms"] * 1e-3 / max(1, r["sweeps"])
        gbs = per_sweep / sw_s / 1e9
        out[key] = {"value": p.points * r["iters"] / dt, "unit": "grid-pt*iters/s", "solve_ms": dt * 1e3,
                    "iters": r["iters"], "w1": r["w1"], "marginal_err": r["marginal_err"],
                    "converged": r["converged"], "mode": "linear domain, stored representation, FP64",
                    "loop_ms": r["loop_ms"], "vs_oracle": vs_oracle(r, gold),
                    "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                                 "kernel": "k_lin_aggregate + k_lin_sweep per half-iteration",
                                 "avg_sweep_us": sw_s * 1e6, "algorithmic_bytes_per_sweep": per_sweep}}
    return out


def bench_plan(reps=10):
    """Plan export and plan difference on the paper's largest plan: the 2D
    160 x 160 workload of section 4.3 (four sorted U[0,1] node vectors,
    masses U[0,1], eps = 0.01, 1000 iterations), whose plan has 25600 x 25600
    FP64 entries (5.2 GB). Potentials from FINOM solves with FP64 and FP32
    scans; the export of the FP64 plan and ||Gamma_fp32 - Gamma_fp64||_F are
    timed with HIP events on the stream the kernels run on."""
    import torch
    from paper_2605_26659_amd import finom_plan_2d, finom_plan_diff_2d, sinkhorn_w1_2d, workloads as wl
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    p = wl.paper_random_2d(160)
    mesh = (dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2))
    uv = (dev(p.u.ravel(order="F")), dev(p.v.ravel(order="F")))
    pot = {}
    for prec in (0, 1):
        r, F, G = sinkhorn_w1_2d(*mesh, *uv, p.eps, 0.0, p.itr_max, precision=prec)
        pot[prec] = (F, G)
    rows, cols = p.u.size, p.v.size
    gamma = torch.empty((rows, cols), dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    F64, G64 = pot[0]
    F32, G32 = pot[1]
    finom_plan_2d(*mesh, F64, G64, p.eps, gamma)
    finom_plan_diff_2d(*mesh, F32, G32, F64, G64, p.eps, out)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(s)
    for _ in range(reps):
        finom_plan_2d(*mesh, F64, G64, p.eps, gamma)
    ev[1].record(s)
    for _ in range(reps):
        finom_plan_diff_2d(*mesh, F32, G32, F64, G64, p.eps, out)
    ev[2].record(s)
    torch.cuda.synchronize()
    export_ms = ev[0].elapsed_time(ev[1]) / reps
    diff_ms = ev[1].elapsed_time(ev[2]) / reps
    total = float(gamma.sum())
    del gamma
    # algorithmic bytes of one export: the plan written once, the potentials
    # and coordinates read once
    bytes_export = 8.0 * rows * cols + 8.0 * 2 * (rows + cols)
    gbs = bytes_export / (export_ms * 1e-3) / 1e9
    return {"workload": "2D 160 x 160 sorted U[0,1] meshes, masses U[0,1], eps=0.01, 1000 iterations "
                        "(section 4.3); plan 25600 x 25600 FP64",
            "export": {"kernel": "k_plan_export<true>", "avg_launch_ms": export_ms,
                       "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": gbs / HBM_PEAK_GBS,
                                    "traffic": measured_traffic(TRAFFIC_PLAN, PLAN_SOURCES, rows),
                                    "algorithmic_bytes": bytes_export},
                       "plan_sum": total},
            "difference": {"kernel": "k_plan_diff<true> + k_plan_diff_final", "avg_ms": diff_ms,
                           "entries_per_s": rows * cols / (diff_ms * 1e-3),
                           "fro_fp32_vs_fp64_scans": float(out.item())}}


def _serving_pool(size, precision):
    """Materialised requests of the serving mix (70 % 1D graded n log-uniform
    in [1e3, 1e6], 30 % 2D tanh side log-uniform in [64, 512], eps 1e-2 or
    1e-3, tol 1e-6); arrivals reuse them round-robin."""
    import torch
    from paper_2605_26659_amd import finom_batch, problem_1d, problem_2d, workloads as wl
    reqs = wl.serving_requests(rate=2000.0, window=10.0, max_requests=size)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    descs, pts = [], []
    for r in reqs:
        p = wl.build_request_problem(r.problem)
        if r.problem[0] == "1d":
            descs.append(problem_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, p.tol, p.itr_max))
        else:
            descs.append(problem_2d(dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2),
                                    dev(p.u.ravel(order="F")), dev(p.v.ravel(order="F")),
                                    p.eps, p.tol, p.itr_max))
        pts.append(p.points)
    torch.cuda.synchronize()
    st, res = finom_batch(descs, precision=precision)
    work = np.array([pt * r["iters"] for pt, r in zip(pts, res)])
    return descs, np.array(pts), work


def _serve(descs, work, rate, window, precision, budget, seed, drain_s=60.0):
    from paper_2605_26659_amd import FinomServer
    rng = np.random.default_rng(seed)
    t, arr = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        arr.append(t)
    done, k = [], 0
    with FinomServer(budget, precision=precision) as srv:
        t0 = time.perf_counter()
        while len(done) < len(arr):
            now = time.perf_counter() - t0
            while k < len(arr) and arr[k] <= now:
                srv.submit(descs[k % len(descs)], sync=False)
                k += 1
            done += srv.poll(512, wait_ms=0)
            if now > window + drain_s:
                break
            nxt = arr[k] - now if k < len(arr) else 0.002
            time.sleep(max(0.0, min(nxt, 0.002)))
        t_end = time.perf_counter() - t0
        stats = srv.stats()
    lat = np.array([c["latency_ms"] for c in done]) if done else np.array([np.nan])
    served_work = float(sum(work[(c["ticket"] - 1) % len(descs)] for c in done))
    offered_work = float(sum(work[i % len(descs)] for i in range(len(arr))))
    return {"rate_per_s": rate, "window_s": window, "requests": len(arr), "completed": len(done),
            "p50_latency_ms": float(np.percentile(lat, 50)),
            "p99_latency_ms": float(np.percentile(lat, 99)),
            "offered_grid_pt_iters_per_s": offered_work / window,
            "served_grid_pt_iters_per_s": served_work / t_end,
            "elapsed_s": t_end, "gpu_busy_ms": stats["busy_ms"], "rounds": stats["rounds"]}


def bench_serving(precision, full):
    budget = 64 << 30
    descs, pts, work = _serving_pool(48, precision)
    # sustainable rates relative to the measured single-batch capacity
    cap_rate = 1.5e10 / float(work.mean())
    out = {"pool": len(descs), "mean_points": float(pts.mean()),
           "mean_work_grid_pt_iters": float(work.mean()), "budget_bytes": budget,
           "scan_mantissa": "fp32" if precision == 1 else "fp64",
           "note": "requests drawn round-robin from a pool of materialised requests of the "
                   "serving mix; latency = submit -> result published", "runs": []}
    fracs = (0.25, 0.5, 0.8) if full else (0.5,)
    for i, fr in enumerate(fracs):
        out["runs"].append(_serve(descs, work, fr * cap_rate, 3.0 if full else 2.0, precision,
                                  budget, 100 + i))
    # the configuration's nominal rate (Poisson, 2000 requests/s): a short
    # window by default, offered and served load side by side
    out["runs"].append(_serve(descs, work, 2000.0, 1.0 if full else 0.5, precision, budget, 200,
                              drain_s=120.0 if full else 30.0))
    return out


def _cpu_model():
    """The host CPU as lscpu names it (model, sockets, cores, threads), else
    /proc/cpuinfo's model name."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU(s)", "Vendor ID"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "Model name" not in info:
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        info["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return info or {"Model name": "unknown"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: --gpus {args.gpus} is not supported "
              "(independent problems shard trivially; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_26659_amd import dense_matvec, sinkhorn_w1_1d, workloads as wl

    if args.copy_calibration:
        # a plain device copy of known size: the HBM byte counters of this
        # kernel calibrate FETCH_SIZE / WRITE_SIZE of the sweeps
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "copies": 10}), flush=True)
        return

    # the tile table of every record (the single-record modes below included,
    # so that their profiles run the shapes the full run times)
    if not args.no_autotune:
        from paper_2605_26659_amd import finom_autotune
        for p in (1, 0):
            finom_autotune(p, args.tune_cache or None)

    if args.plan_only:
        print(json.dumps(bench_plan(args.steps)), flush=True)
        return
    if args.tanh_2d_only:
        print(json.dumps(bench_tanh_2d(1 if args.precision == "fp32" else 0)), flush=True)
        return
    if args.stream_2p24_only:
        print(json.dumps(bench_stream_2p24(1 if args.precision == "fp32" else 0)), flush=True)
        return
    if args.random_3d_only:
        print(json.dumps(bench_random_3d(1 if args.precision == "fp32" else 0)), flush=True)
        return

    prob = wl.config_graded_1d(args.n, args.eps, tol=args.tol)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    x, y, u, v = dev(prob.x), dev(prob.y), dev(prob.u), dev(prob.v)
    f = torch.empty_like(x)
    g = torch.empty_like(y)
    prec = 1 if args.precision == "fp32" else 0
    pts = 0.5 * (len(prob.x) + len(prob.y))

    def solve(p=prec):
        res, _, _ = sinkhorn_w1_1d(x, y, u, v, prob.eps, prob.tol, prob.itr_max, precision=p,
                                   f_out=f, g_out=g)
        return res

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    lat, its, loops, sweeps = [], [], [], []
    last = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        last = solve()
        lat.append(time.perf_counter() - t0)
        its.append(last["iters"])
        loops.append(last["loop_ms"])
        sweeps.append(last["sweeps"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    value = pts * sum(its) / total

    n, m = len(prob.x), len(prob.y)
    bytes_iter = (BYTES_KT[0] + BYTES_K[0]) * n + (BYTES_KT[1] + BYTES_K[1]) * m
    per_sweep_bytes = bytes_iter / 2.0
    sweep_ms = sum(loops) / max(1, sum(sweeps))
    if last["fast"] == 2:
        # dominant kernel: the resident solver, one launch per solve, timed by
        # HIP events around the launch on its stream
        launch_ms = sum(loops) / len(loops)
        ops = OPS_PER_PT_ITER * pts * sum(its) / len(its)
        achieved = ops / (launch_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
                    "frac": achieved / ALU_PEAK_TOPS,
                    "traffic": measured_traffic(TRAFFIC_RESIDENT, RESIDENT_SOURCES, args.n),
                    "kernel": "k_resident_1d<512, 8, 4, false>: the whole loop in one cooperative launch",
                    "avg_launch_ms": launch_ms, "avg_sweep_us": sweep_ms * 1e3,
                    "ops_per_grid_pt_iter": OPS_PER_PT_ITER,
                    "unit_note": "lane operations (each add, multiply, fma, ldexp, reciprocal counts once) "
                                 "against 256 CUs x 64 lanes x 2.4 GHz",
                    "streaming_equivalent_GBs": per_sweep_bytes / (sweep_ms * 1e-3) / 1e9}
        rv = RESIDENT_VALU
        if args.n == rv["n"] and sources_digest(RESIDENT_SOURCES) == rv["sources_sha256"]:
            roofline["valu_counters"] = {
                "issued_lane_ops_per_grid_pt_iter": rv["valu_insts"] * 64 / (rv["n"] * rv["iters"]),
                "valu_issue_frac": rv["valu_insts"] / (rv["launch_us"] * 1e-6 * VALU_ISSUE_PEAK),
                "note": "rocprofv3 SQ_INSTS_VALU per launch of the same workload: VALU wave instructions "
                        "issued against one per SIMD per 4 clocks (profiles/k_resident_1d_graded_1d_n2p20.md)"}
    else:
        # dominant kernels: the half-iteration sweeps; average launch duration
        # from the loop's HIP events divided by the sweeps executed
        achieved = per_sweep_bytes / (sweep_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(TRAFFIC_STREAM, STREAM_SOURCES, args.n),
                    "kernel": "the loop's sweeps, both half-iteration variants (K^T phi with the "
                              "fused marginal check, K psi), averaged over the loop's launches",
                    "avg_sweep_us": sweep_ms * 1e3,
                    "algorithmic_bytes_per_sweep": per_sweep_bytes}

    extra = {}
    if not args.no_fp64_compare:
        r64 = solve(0 if prec == 1 else 1)
        t0 = time.perf_counter()
        r64 = solve(0 if prec == 1 else 1)
        dt = time.perf_counter() - t0
        key = "fp64_scans" if prec == 1 else "fp32_scans"
        extra[key] = {"value": pts * r64["iters"] / dt, "unit": "grid-pt*iters/s", "solve_ms": dt * 1e3,
                      "iters": r64["iters"], "w1": r64["w1"], "marginal_err": r64["marginal_err"],
                      "state": state_repr(r64), "resident": r64["fast"] == 2,
                      "w1_rel_diff_vs_headline": abs(r64["w1"] - last["w1"]) / r64["w1"]}
        if key == "fp64_scans":
            # the FP64 loop runs the streaming general sweeps (k_sweep with
            # FP64 mantissas): the HBM roofline of the same 88 B per grid point
            # per iteration, from the loop's HIP events over its sweeps
            sw_s = r64["loop_ms"] * 1e-3 / max(1, r64["sweeps"])
            gbs64 = per_sweep_bytes / sw_s / 1e9
            extra[key]["roofline"] = {
                "bound": "hbm", "achieved": gbs64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs64 / HBM_PEAK_GBS,
                "traffic": measured_traffic(TRAFFIC_FP64, STREAM_SOURCES, args.n),
                "kernel": "k_sweep<double, 256, 4, IN_LOG2, EPI_UPDATE_CHECK / EPI_UPDATE, NEXT_AGG>",
                "avg_sweep_us": sw_s * 1e6, "algorithmic_bytes_per_sweep": per_sweep_bytes}
        if args.n == 1 << 20 and args.tol == 1e-6:
            extra[key]["vs_oracle"] = vs_oracle(r64, graded_golden(args.eps))
    if not args.no_dense:
        gin = torch.as_tensor(prob.eps * np.log(prob.v), dtype=torch.float64, device="cuda")
        out = torch.empty_like(x)
        dense_matvec(x, y, prob.eps, gin, out, domain=1, precision=prec, skip_checks=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 2
        e0.record()
        for _ in range(reps):
            dense_matvec(x, y, prob.eps, gin, out, domain=1, precision=prec, skip_checks=True)
        e1.record()
        torch.cuda.synchronize()
        per_product_s = e0.elapsed_time(e1) / reps * 1e-3
        dense_rate = pts / (2.0 * per_product_s)
        extra["dense_sinkhorn_gpu"] = {
            "value": dense_rate, "unit": "grid-pt*iters/s",
            "per_iteration_s": 2 * per_product_s,
            "time_to_tol_s": 2 * per_product_s * its[-1],
            "note": "dense on-the-fly-exp products; iterates equal FINOM's, so time to "
                    "tolerance = per-iteration time x FINOM's iteration count"}
        extra["speedup_vs_dense"] = value / dense_rate

    if not args.no_other:
        extra.update(bench_other_configs(prec))
        extra["plan_2d_160"] = bench_plan()
    if not args.no_batch:
        extra["batch_4096"] = bench_batch(prec)
    if args.serving or not args.no_serving:
        extra["serving"] = bench_serving(prec, args.serving)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, args.cpu_seconds)

    from paper_2605_26659_amd import finom_tile_config
    extra["tile_shapes"] = {p: [finom_tile_config(1 if p == "fp32" else 0, 512 << c) for c in range(13)]
                            for p in ("fp32", "fp64")}
    extra["tile_shapes_note"] = ("tile-shape index per merged-line length class 2^9..2^21 "
                                 "(0: 256x4, 1: 256x8, 2: 512x8, 3: 128x4, 4: 512x4)")
    # the paper's own timing (section 4.1, Table 1: C++ on a 14-core Xeon Gold
    # 5117 at 2.0 GHz, eps = 0.01, 1000 iterations), as context only
    extra["paper_cpu_context"] = {"workload": "1D Chebyshev nodes N=8000, 1000 iterations",
                                  "finom_s": 1.41e-1, "dense_s": 9.05e2,
                                  "finom_grid_pt_iters_per_s": 8000 * 1000 / 1.41e-1,
                                  "hardware": "Xeon Gold 5117 14-core 2.0 GHz (CPU)"}

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": "FINOM grid-pt*iters/s vs dense Sinkhorn at 1e-6 tol; p50/p99 solve latency",
        "value": value, "unit": "grid-pt*iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": f"1D W1 graded meshes n=m={args.n} (x=t^2, y=Chebyshev), "
                               f"3-GMM masses, eps={args.eps:g}, tol={args.tol:g}",
                   "n": args.n, "m": args.n, "eps": args.eps, "tol": args.tol,
                   "scan_mantissa": args.precision, "state": state_repr(last),
                   "stop_test": ("FP32-sum estimate, each stop confirmed by an FP64 check of the returned pair"
                                 if prec == 1 else "FP64")},
        "iters_per_solve": its[-1], "w1": last["w1"], "marginal_err": last["marginal_err"],
        "resumes": last["resumes"],
        "vs_oracle": (vs_oracle(last, graded_golden(args.eps))
                      if args.n == 1 << 20 and args.tol == 1e-6 else None),
        "p50_latency_ms": float(np.percentile(lat_ms, 50)),
        "p99_latency_ms": float(np.percentile(lat_ms, 99)),
        "roofline": roofline, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
