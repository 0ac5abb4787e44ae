"""Writes the converged reference results of the throughput workloads
(TEST INFRASTRUCTURE: calls only the oracle and the seeded input generators).

    python -m oracle.make_goldens [small_1d] [graded_1e-2] [graded_1e-3] [tanh_2d] [--threads T]

For each workload the oracle runs its Sinkhorn loop to the tolerance, exactly
as Algorithm 1 / Algorithm 2 state it (loop-head L1 check of the pre-update
psi, stop at err <= tol or at the cap), and stores in tests/golden/:
  - the completed iteration count and the checked marginal error;
  - W1 = <C, Gamma> of the returned pair by the plain definition: the dense
    double sum over every (i, j) in 1D, and on the tensor mesh the dense
    per-axis kernels of eq. 2d-kron with C = |dx| + |dy|;
  - the u-side marginal error of the returned pair, recomputed by the oracle;
  - the potentials f = eps ln phi and g = eps ln psi at fixed indices.

Workloads (inputs from paper_2605_26659_amd.workloads, seeded):
  small_1d: n = m = 512 sorted U(0,1), masses U(0.1,1), eps 0.01, tol 1e-9,
      cap 2000 (dense products, the plain definition).
  graded_1e-2, graded_1e-3: n = m = 2^20, x = t^2, y = ascending Chebyshev
      nodes, 3-component Gaussian-mixture masses, tol 1e-6, cap 20000.
  tanh_2d: 1024 x 1024 tanh-stretched tensor mesh (beta 2.5) for source and
      target, 4-component anisotropic Gaussian-mixture masses, eps 5e-3,
      tol 1e-6, cap 20000.

The 1D dense W1 sums 2^40 terms (about half an hour on 8 cores per file).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

from oracle import clib, dense  # noqa: E402
from paper_2605_26659_amd import workloads as wl  # noqa: E402

GOLDEN = ROOT / "tests" / "golden"


def sample_indices(n: int, k: int = 1024) -> np.ndarray:
    """k evenly spaced indices plus the first and last eight."""
    idx = np.unique(np.concatenate([np.rint(np.linspace(0, n - 1, k)).astype(np.int64),
                                    np.arange(min(8, n)), np.arange(max(n - 8, 0), n)]))
    return idx


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def golden_graded_1d(eps: float, threads: int) -> dict:
    p = wl.config_graded_1d(eps=eps)
    n, m = len(p.x), len(p.y)
    log(f"graded 1D n={n} eps={eps}: Algorithm 1 to tol {p.tol}")
    t0 = time.time()
    f, g, iters, err = clib.sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, p.tol, p.itr_max)
    t_alg = time.time() - t0
    log(f"  iters={iters} err={err:.6e} ({t_alg:.0f} s)")
    # u side of the returned pair: |phi (K psi) - u|, K psi by the recurrences
    t = clib.finom_logmatvec(p.x, p.y, g, p.eps)
    u_err = float(np.sum(np.abs(np.exp((f + t) / p.eps) - p.u)))
    log(f"  u-side error {u_err:.3e}; dense W1 over {n}x{m} terms on {threads} threads")
    t0 = time.time()
    w1 = clib.dense_cost_1d(p.x, p.y, f, g, p.eps, threads=threads)
    t_w1 = time.time() - t0
    log(f"  W1={w1!r} ({t_w1:.0f} s)")
    idx = sample_indices(n)
    return {
        "workload": f"graded 1D, n = m = 2^20, x = t^2, y = Chebyshev (ascending), "
                    f"3-GMM masses, eps = {eps:g}, tol = {p.tol:g}, cap {p.itr_max}",
        "source": "oracle: Algorithm 1 in C (log-form eq. p-DP / q-DP recurrences, FP64), "
                  "W1 by the dense double sum of |x_i - y_j| Gamma_ij",
        "n": n, "m": m, "eps": p.eps, "tol": p.tol, "itr_max": p.itr_max,
        "iters": iters, "err": err, "u_err": u_err, "w1": w1,
        "idx": idx.tolist(), "f": f[idx].tolist(), "g": g[idx].tolist(),
        "oracle_seconds": {"algorithm1": round(t_alg, 1), "w1": round(t_w1, 1)},
    }


def golden_tanh_2d(threads: int) -> dict:
    p = wl.config_tanh_2d()
    n1, m1 = p.u.shape
    log(f"tanh 2D {n1}x{m1} eps={p.eps}: Algorithm 2 to tol {p.tol}")
    t0 = time.time()
    F, G, iters, err = clib.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, p.tol,
                                        p.itr_max, threads=threads)
    t_alg = time.time() - t0
    log(f"  iters={iters} err={err:.6e} ({t_alg:.0f} s)")
    T = clib.finom_logmatvec_2d(p.x1, p.y1, p.x2, p.y2, G, p.eps, threads=threads)
    u_err = float(np.sum(np.abs(np.exp((F + T) / p.eps) - p.u)))
    t0 = time.time()
    w1 = dense.transport_cost_2d(p.x1, p.y1, p.x2, p.y2, F, G, p.eps)
    t_w1 = time.time() - t0
    log(f"  u-side error {u_err:.3e}; W1={w1!r} ({t_w1:.0f} s)")
    Ff, Gf = F.ravel(order="F"), G.ravel(order="F")
    idx = sample_indices(Ff.size)
    return {
        "workload": f"tanh 2D, {n1} x {m1} tensor mesh (beta 2.5), same mesh for both measures, "
                    f"4-GMM anisotropic masses, eps = {p.eps:g}, tol = {p.tol:g}, cap {p.itr_max}",
        "source": "oracle: Algorithm 2 in C (axis-by-axis log-form recurrences, FP64), "
                  "W1 by dense per-axis kernels (eq. 2d-kron, C = |dx| + |dy|)",
        "n1": n1, "m1": m1, "n2": p.v.shape[0], "m2": p.v.shape[1], "eps": p.eps,
        "tol": p.tol, "itr_max": p.itr_max, "iters": iters, "err": err, "u_err": u_err,
        "w1": w1, "idx": idx.tolist(), "f": Ff[idx].tolist(), "g": Gf[idx].tolist(),
        "layout": "column-major grids, element (k, i) at k + i * n1",
        "oracle_seconds": {"algorithm2": round(t_alg, 1), "w1": round(t_w1, 1)},
    }


def golden_small_1d(threads: int) -> dict:
    p = wl.config_small_1d()
    n, m = len(p.x), len(p.y)
    log(f"small 1D n={n}: dense Sinkhorn to tol {p.tol} or {p.itr_max} iterations")
    f, g, iters, err = clib.dense_sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, p.tol, p.itr_max,
                                              threads=threads)
    t = clib.dense_logmatvec(p.x, p.y, g, p.eps, threads=threads)
    u_err = float(np.sum(np.abs(np.exp((f + t) / p.eps) - p.u)))
    w1 = clib.dense_cost_1d(p.x, p.y, f, g, p.eps, threads=threads)
    log(f"  iters={iters} err={err:.6e} W1={w1!r}")
    idx = sample_indices(n, 128)
    return {
        "workload": f"small 1D, n = m = {n} sorted U(0,1), masses U(0.1,1), eps = {p.eps:g}, "
                    f"tol = {p.tol:g}, cap {p.itr_max}",
        "source": "oracle: dense log-domain Sinkhorn with Algorithm 1's loop (C), "
                  "W1 by the dense double sum",
        "n": n, "m": m, "eps": p.eps, "tol": p.tol, "itr_max": p.itr_max,
        "iters": iters, "err": err, "u_err": u_err, "w1": w1,
        "idx": idx.tolist(), "f": f[idx].tolist(), "g": g[idx].tolist(),
    }


WORKLOADS = {
    "small_1d": ("small_1d_n512.json", golden_small_1d),
    "graded_1e-2": ("graded_1d_2p20_eps1e-2.json", lambda th: golden_graded_1d(1e-2, th)),
    "graded_1e-3": ("graded_1d_2p20_eps1e-3.json", lambda th: golden_graded_1d(1e-3, th)),
    "tanh_2d": ("tanh_2d_1024_eps5e-3.json", golden_tanh_2d),
}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(WORKLOADS))
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1))
    a = ap.parse_args()
    clib.build(force=False)
    GOLDEN.mkdir(parents=True, exist_ok=True)
    for name in a.names:
        fname, fn = WORKLOADS[name]
        rec = fn(a.threads)
        (GOLDEN / fname).write_text(json.dumps(rec, indent=1) + "\n")
        log(f"wrote {GOLDEN / fname}")


if __name__ == "__main__":
    main()
