"""Seeded synthetic inputs for entropic W1 problems on non-uniform meshes.

This module only draws meshes, masses and regularisation strengths. It holds
none of the transport arithmetic, so that the FP64 CPU oracle and the HIP path
can both consume the same arrays without sharing any computation.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws in the
order meshes, then masses, then epsilon. Seeds follow ``26659 + 1000*config +
problem_index``.

Workload shapes follow the paper's experiments (section 4: Chebyshev nodes,
sorted uniform nodes, 2D sorted uniform tensor meshes, masses uniform on [0,1]
then normalised) and the graded/stretched variants used for the throughput
configurations (square-law mesh, Chebyshev-clustered mesh, tanh boundary-layer
mesh, Gaussian-mixture masses with a 1e-6 floor).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 26659


def seed_for(config: int, index: int = 0) -> int:
    return SEED_BASE + 1000 * config + index


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# meshes (all returned ascending, float64)
# --------------------------------------------------------------------------

def mesh_uniform_random(rng: np.random.Generator, n: int) -> np.ndarray:
    """Sorted Uniform(0,1) nodes (section 4.2, section 4.3)."""
    return np.sort(rng.uniform(0.0, 1.0, size=n))


def mesh_chebyshev(n: int) -> np.ndarray:
    """Chebyshev nodes 1/2 + 1/2 cos((2k-1) pi / 2N), k = 1..N (section 4.1).

    The formula decreases with k; the nodes are returned in ascending order.
    """
    k = np.arange(1, n + 1, dtype=np.float64)
    z = 0.5 + 0.5 * np.cos((2.0 * k - 1.0) * np.pi / (2.0 * n))
    return np.ascontiguousarray(z[::-1])


def mesh_square_law(n: int) -> np.ndarray:
    """Graded mesh x_i = t_i^2 with t_i = (i - 1/2)/n, clustered at 0."""
    t = (np.arange(1, n + 1, dtype=np.float64) - 0.5) / n
    return t * t


def mesh_tanh(n: int, beta: float = 2.5) -> np.ndarray:
    """Two-sided boundary-layer mesh z = (1 + tanh(beta(2s-1))/tanh(beta))/2."""
    if n == 1:
        return np.array([0.5])
    s = np.arange(n, dtype=np.float64) / (n - 1)
    return 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / np.tanh(beta))


# --------------------------------------------------------------------------
# masses (all strictly positive, normalised to sum 1)
# --------------------------------------------------------------------------

def normalise(w: np.ndarray) -> np.ndarray:
    return w / w.sum()


def masses_uniform(rng: np.random.Generator, n: int, lo: float = 0.0,
                   hi: float = 1.0) -> np.ndarray:
    w = rng.uniform(lo, hi, size=n)
    # Uniform(0,1) can in principle return exactly 0; keep masses positive.
    w = np.maximum(w, 1e-300)
    return normalise(w)


def masses_gmm_1d(rng: np.random.Generator, nodes: np.ndarray, k: int = 3,
                  floor: float = 1e-6) -> np.ndarray:
    """k-component Gaussian mixture density sampled at the nodes, plus a floor."""
    w = rng.dirichlet(np.ones(k))
    mu = rng.uniform(0.2, 0.8, size=k)
    sd = rng.uniform(0.02, 0.1, size=k)
    dens = np.zeros_like(nodes)
    for a, m, s in zip(w, mu, sd):
        dens += a * np.exp(-0.5 * ((nodes - m) / s) ** 2) / (s * np.sqrt(2 * np.pi))
    return normalise(dens + floor)


def masses_gmm_2d(rng: np.random.Generator, xs: np.ndarray, ys: np.ndarray,
                  k: int = 4, floor: float = 1e-6) -> np.ndarray:
    """Anisotropic rotated 2D Gaussian mixture on the tensor mesh xs x ys.

    Returned as an (len(xs), len(ys)) array; element [k, i] sits at
    (xs[k], ys[i]). Column-major vectorisation of this array is the paper's
    grid ordering (section 3.1).
    """
    w = rng.dirichlet(np.ones(k))
    mu = rng.uniform(0.2, 0.8, size=(k, 2))
    sd = rng.uniform(0.02, 0.1, size=(k, 2))
    th = rng.uniform(0.0, np.pi, size=k)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    dens = np.zeros_like(X)
    for a, m, s, t in zip(w, mu, sd, th):
        c, sn = np.cos(t), np.sin(t)
        dx, dy = X - m[0], Y - m[1]
        u = c * dx + sn * dy
        v = -sn * dx + c * dy
        dens += a * np.exp(-0.5 * ((u / s[0]) ** 2 + (v / s[1]) ** 2)) / (2 * np.pi * s[0] * s[1])
    return normalise(dens + floor)


# --------------------------------------------------------------------------
# problem records
# --------------------------------------------------------------------------

@dataclass
class Problem1D:
    x: np.ndarray
    y: np.ndarray
    u: np.ndarray
    v: np.ndarray
    eps: float
    tol: float
    itr_max: int
    name: str = ""

    @property
    def points(self) -> float:
        return 0.5 * (len(self.x) + len(self.y))


@dataclass
class Problem2D:
    x1: np.ndarray   # source mesh, first axis (N1)
    y1: np.ndarray   # source mesh, second axis (M1)
    x2: np.ndarray   # target mesh, first axis (N2)
    y2: np.ndarray   # target mesh, second axis (M2)
    u: np.ndarray    # (N1, M1)
    v: np.ndarray    # (N2, M2)
    eps: float
    tol: float
    itr_max: int
    name: str = ""

    @property
    def points(self) -> float:
        return 0.5 * (self.u.size + self.v.size)


# --------------------------------------------------------------------------
# the paper's experiments (section 4)
# --------------------------------------------------------------------------

def paper_chebyshev_1d(n: int, seed: int = seed_for(11), eps: float = 0.01,
                       iters: int = 1000) -> Problem1D:
    """Section 4.1: both measures on the N Chebyshev nodes, masses U[0,1]."""
    rng = rng_for(seed)
    x = mesh_chebyshev(n)
    y = x.copy()
    u = masses_uniform(rng, n)
    v = masses_uniform(rng, n)
    return Problem1D(x, y, u, v, eps, 0.0, iters, f"paper-chebyshev-{n}")


def paper_random_1d(n: int, seed: int = seed_for(12), eps: float = 0.01,
                    iters: int = 1000) -> Problem1D:
    """Section 4.2: independent sorted U[0,1] nodes, masses U[0,1]."""
    rng = rng_for(seed)
    x = mesh_uniform_random(rng, n)
    y = mesh_uniform_random(rng, n)
    u = masses_uniform(rng, n)
    v = masses_uniform(rng, n)
    return Problem1D(x, y, u, v, eps, 0.0, iters, f"paper-random-{n}")


def paper_random_2d(n: int, seed: int = seed_for(13), eps: float = 0.01,
                    iters: int = 1000) -> Problem2D:
    """Section 4.3: four independent sorted U[0,1] node vectors, N x N."""
    rng = rng_for(seed)
    x1 = mesh_uniform_random(rng, n)
    x2 = mesh_uniform_random(rng, n)
    y1 = mesh_uniform_random(rng, n)
    y2 = mesh_uniform_random(rng, n)
    u = masses_uniform(rng, n * n).reshape(n, n)
    v = masses_uniform(rng, n * n).reshape(n, n)
    return Problem2D(x1, y1, x2, y2, u, v, eps, 0.0, iters, f"paper-random2d-{n}")


def paper_random_nd(sizes_src, sizes_tgt, seed: int = seed_for(14), eps: float = 0.01,
                    iters: int = 1000):
    """Section 4.3's recipe in d dimensions (the remark closing section 3):
    independent sorted U[0,1] node vectors per axis, masses U[0,1] normalised,
    as column-major grids. Returns (source axes, target axes, u, v, eps, iters)."""
    rng = rng_for(seed)
    xs = [mesh_uniform_random(rng, k) for k in sizes_src]
    xt = [mesh_uniform_random(rng, k) for k in sizes_tgt]
    u = masses_uniform(rng, int(np.prod(sizes_src))).reshape(tuple(sizes_src), order="F")
    v = masses_uniform(rng, int(np.prod(sizes_tgt))).reshape(tuple(sizes_tgt), order="F")
    return xs, xt, u, v, eps, iters


# --------------------------------------------------------------------------
# throughput / correctness configurations
# --------------------------------------------------------------------------

def config_small_1d(seed: int = seed_for(1), n: int = 512) -> Problem1D:
    """n = m = 512 sorted uniform nodes, masses U(0.1,1), eps 0.01.

    Stop at marginal L1 error < 1e-9 or 2000 iterations.
    """
    rng = rng_for(seed)
    x = mesh_uniform_random(rng, n)
    y = mesh_uniform_random(rng, n)
    u = masses_uniform(rng, n, 0.1, 1.0)
    v = masses_uniform(rng, n, 0.1, 1.0)
    return Problem1D(x, y, u, v, 0.01, 1e-9, 2000, f"small1d-{n}")


def config_graded_1d(n: int = 1 << 20, eps: float = 1e-3,
                     seed: int = seed_for(2), tol: float = 1e-6,
                     itr_max: int = 20000) -> Problem1D:
    """Graded 1D meshes: x = t^2, y = ascending Chebyshev; 3-GMM masses."""
    rng = rng_for(seed)
    x = mesh_square_law(n)
    y = mesh_chebyshev(n)
    u = masses_gmm_1d(rng, x, 3)
    v = masses_gmm_1d(rng, y, 3)
    return Problem1D(x, y, u, v, eps, tol, itr_max, f"graded1d-{n}-eps{eps:g}")


def config_tanh_2d(side: int = 1024, eps: float = 5e-3, seed: int = seed_for(3),
                   tol: float = 1e-6, itr_max: int = 20000,
                   beta: float = 2.5) -> Problem2D:
    """side x side tanh-stretched tensor mesh, same mesh for source and target,
    4-component anisotropic Gaussian-mixture masses."""
    rng = rng_for(seed)
    z = mesh_tanh(side, beta)
    u = masses_gmm_2d(rng, z, z, 4)
    v = masses_gmm_2d(rng, z, z, 4)
    return Problem2D(z.copy(), z.copy(), z.copy(), z.copy(), u, v, eps, tol,
                     itr_max, f"tanh2d-{side}")


def batch_sizes(count: int = 4096, lo: int = 256, hi: int = 65536,
                seed: int = seed_for(4)) -> np.ndarray:
    rng = rng_for(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def config_batch_problem(index: int, n: int, tol: float = 1e-6,
                         itr_max: int = 20000, config: int = 4) -> Problem1D:
    """One member of the uneven batch: sorted U(0,1) meshes, 3-GMM masses,
    eps log-uniform in [1e-3, 1e-1]."""
    rng = rng_for(seed_for(config, index + 1))
    x = mesh_uniform_random(rng, n)
    y = mesh_uniform_random(rng, n)
    u = masses_gmm_1d(rng, x, 3)
    v = masses_gmm_1d(rng, y, 3)
    eps = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
    return Problem1D(x, y, u, v, eps, tol, itr_max, f"batch-{index}-{n}")


def config_batch(count: int = 4096, lo: int = 256, hi: int = 65536,
                 tol: float = 1e-6, itr_max: int = 20000) -> List[Problem1D]:
    sizes = batch_sizes(count, lo, hi)
    return [config_batch_problem(i, int(n), tol, itr_max) for i, n in enumerate(sizes)]


@dataclass
class Request:
    arrival: float           # seconds since the start of the window
    problem: object          # Problem1D or Problem2D
    index: int = 0


def serving_requests(rate: float = 2000.0, window: float = 10.0,
                     frac_1d: float = 0.7, n1d=(1000, 1_000_000),
                     side2d=(64, 512), eps_choices=(1e-2, 1e-3),
                     tol: float = 1e-6, itr_max: int = 20000,
                     seed: int = seed_for(5),
                     max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals of mixed 1D (graded meshes) and 2D (tanh meshes) solves.

    The arrival process and per-request parameters come from one generator;
    each request's arrays come from its own seed so a request can be rebuilt
    alone.
    """
    rng = rng_for(seed)
    out: List[Request] = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        if max_requests is not None and i >= max_requests:
            break
        is1d = rng.uniform() < frac_1d
        eps = float(eps_choices[int(rng.integers(len(eps_choices)))])
        if is1d:
            n = int(np.rint(np.exp(rng.uniform(np.log(n1d[0]), np.log(n1d[1])))))
            out.append(Request(t, ("1d", n, eps, tol, itr_max, seed_for(5, i + 1)), i))
        else:
            s = int(np.rint(np.exp(rng.uniform(np.log(side2d[0]), np.log(side2d[1])))))
            out.append(Request(t, ("2d", s, eps, tol, itr_max, seed_for(5, i + 1)), i))
        i += 1
    return out


def build_request_problem(spec) -> object:
    """Materialise a serving request's arrays from its (kind, size, eps, tol,
    itr_max, seed) tuple."""
    kind, size, eps, tol, itr_max, seed = spec
    if kind == "1d":
        return config_graded_1d(size, eps, seed, tol, itr_max)
    return config_tanh_2d(size, eps, seed, tol, itr_max)
