"""Dense plans and plan differences (HIP) against the FP64 oracle.

* finom_plan_1d / finom_plan_2d element by element against the oracle's
  plan (section 2.1; eq. 2d-block-entry on tensor meshes): single points,
  ragged column chunks, padded leading dimensions, entries that underflow;
* finom_plan_diff_1d / _2d against the oracle's ||Gamma_a - Gamma_b||_F on
  potentials that differ well above rounding, zero for equal potentials,
  the same bits on repeated calls;
* the plan-difference column of section 4's tables: FINOM on the GPU
  (FP64 scans, 1000 iterations, eps = 0.01) against the standard Sinkhorn
  iteration of the oracle with dense products, at the paper's sizes that the
  oracle runs in seconds.
"""
import numpy as np
import pytest

from oracle import clib, dense
from paper_2605_26659_amd import workloads as wl

from gpuhelp import dev, host

pytestmark = pytest.mark.gpu

# Plan entries: both sides form the same argument ((f + g) - C) / eps in FP64
# with the same operation order, so they differ only by the two FP64
# exponentials, each within a few ulp. Entries below the normal range lose
# relative accuracy, hence the absolute floor.
RTOL_ENTRY = 1e-14
ATOL_ENTRY = 1e-300


def _pot(rng, k, scale):
    return rng.uniform(-scale, scale, k)


@pytest.mark.parametrize("n,m,pad", [(1, 1, 0), (1, 5, 3), (7, 1, 0), (37, 4099, 0), (300, 2048, 5),
                                     (129, 2049, 1)])
def test_plan_1d_entries(n, m, pad):
    from paper_2605_26659_amd import finom_plan_1d
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1000 + n + m)
    x, y = np.sort(rng.uniform(0, 1, n)), np.sort(rng.uniform(0, 1, m))
    f, g = _pot(rng, n, 0.05), _pot(rng, m, 0.05)
    eps = 0.02
    ld = m + pad
    gamma = torch.full((n, ld), -7.0, dtype=torch.float64, device="cuda")
    finom_plan_1d(dev(x), dev(y), dev(f), dev(g), eps, gamma, ld=ld)
    out = host(gamma)
    ref = dense.plan_1d(x, y, f, g, eps)
    np.testing.assert_allclose(out[:, :m], ref, rtol=RTOL_ENTRY, atol=ATOL_ENTRY)
    assert np.all(out[:, m:] == -7.0)


def test_plan_1d_underflow_and_unsorted():
    """Small eps: entries far from the diagonal underflow to subnormals and
    zero; meshes in any order (entries are independent)."""
    from paper_2605_26659_amd import finom_plan_1d
    rng = np.random.default_rng(1001)
    x, y = rng.uniform(0, 1, 257), rng.uniform(0, 1, 300)
    f, g = _pot(rng, 257, 1e-3), _pot(rng, 300, 1e-3)
    eps = 1.3e-3
    out = host(finom_plan_1d(dev(x), dev(y), dev(f), dev(g), eps))
    ref = dense.plan_1d(x, y, f, g, eps)
    assert np.any(ref == 0.0) and np.any((ref > 0) & (ref < 2.2250738585072014e-308))
    np.testing.assert_allclose(out, ref, rtol=RTOL_ENTRY, atol=ATOL_ENTRY)


@pytest.mark.parametrize("n1,m1,n2,m2,pad", [(1, 1, 1, 1, 0), (3, 4, 5, 2, 0), (10, 10, 10, 10, 2),
                                             (17, 9, 13, 21, 0), (40, 52, 45, 50, 3), (6, 5, 300, 1, 0),
                                             (2, 3, 1, 300, 0)])
def test_plan_2d_entries(n1, m1, n2, m2, pad):
    from paper_2605_26659_amd import finom_plan_2d
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2000 + n1 * m1 + n2 * m2)
    x1, y1 = np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1))
    x2, y2 = np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2))
    F, G = _pot(rng, n1 * m1, 0.05), _pot(rng, n2 * m2, 0.05)
    eps = 0.03
    cols = n2 * m2
    ld = cols + pad
    gamma = torch.full((n1 * m1, ld), -7.0, dtype=torch.float64, device="cuda")
    finom_plan_2d(dev(x1), dev(y1), dev(x2), dev(y2), dev(F), dev(G), eps, gamma, ld=ld)
    out = host(gamma)
    ref = dense.plan_2d(x1, y1, x2, y2, F, G, eps)
    np.testing.assert_allclose(out[:, :cols], ref, rtol=RTOL_ENTRY, atol=ATOL_ENTRY)
    assert np.all(out[:, cols:] == -7.0)


@pytest.mark.parametrize("n,m", [(1, 1), (5, 3000), (700, 650), (2500, 2100)])
def test_plan_diff_1d(n, m):
    from paper_2605_26659_amd import finom_plan_diff_1d
    rng = np.random.default_rng(3000 + n + m)
    x, y = np.sort(rng.uniform(0, 1, n)), np.sort(rng.uniform(0, 1, m))
    eps = 0.01
    fa, ga = _pot(rng, n, 0.02), _pot(rng, m, 0.02)
    fb, gb = fa + 1e-4 * rng.standard_normal(n), ga + 1e-4 * rng.standard_normal(m)
    d, x_, y_ = dev, dev(x), dev(y)
    got = float(host(finom_plan_diff_1d(x_, y_, d(fa), d(ga), d(fb), d(gb), eps))[0])
    ref = dense.plan_difference(dense.plan_1d(x, y, fa, ga, eps), dense.plan_1d(x, y, fb, gb, eps))
    # the entry differences are ~1e-2 relative, far above the exponentials'
    # rounding; the sums of squares differ by summation order only
    assert abs(got - ref) <= 1e-11 * ref
    again = float(host(finom_plan_diff_1d(x_, y_, d(fa), d(ga), d(fb), d(gb), eps))[0])
    assert again == got
    zero = float(host(finom_plan_diff_1d(x_, y_, d(fa), d(ga), d(fa), d(ga), eps))[0])
    assert zero == 0.0


@pytest.mark.parametrize("n1,m1,n2,m2", [(1, 1, 1, 1), (7, 6, 9, 4), (30, 31, 29, 33), (45, 40, 41, 44)])
def test_plan_diff_2d(n1, m1, n2, m2):
    from paper_2605_26659_amd import finom_plan_diff_2d
    rng = np.random.default_rng(4000 + n1 * m1 + n2 * m2)
    x1, y1 = np.sort(rng.uniform(0, 1, n1)), np.sort(rng.uniform(0, 1, m1))
    x2, y2 = np.sort(rng.uniform(0, 1, n2)), np.sort(rng.uniform(0, 1, m2))
    eps = 0.02
    Fa, Ga = _pot(rng, n1 * m1, 0.02), _pot(rng, n2 * m2, 0.02)
    Fb, Gb = Fa + 1e-4 * rng.standard_normal(n1 * m1), Ga + 1e-4 * rng.standard_normal(n2 * m2)
    mesh = [dev(a) for a in (x1, y1, x2, y2)]
    got = float(host(finom_plan_diff_2d(*mesh, dev(Fa), dev(Ga), dev(Fb), dev(Gb), eps))[0])
    ref = dense.plan_difference(dense.plan_2d(x1, y1, x2, y2, Fa, Ga, eps),
                                dense.plan_2d(x1, y1, x2, y2, Fb, Gb, eps))
    assert abs(got - ref) <= 1e-11 * ref
    zero = float(host(finom_plan_diff_2d(*mesh, dev(Fa), dev(Ga), dev(Fa), dev(Ga), eps))[0])
    assert zero == 0.0


def test_plan_argument_errors():
    from paper_2605_26659_amd import FINOM_E_ARG, FinomError, finom_plan_1d, load
    torch = pytest.importorskip("torch")
    x, y = dev(np.linspace(0, 1, 4)), dev(np.linspace(0, 1, 3))
    f, g = dev(np.zeros(4)), dev(np.zeros(3))
    gamma = torch.full((4, 3), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(FinomError) as e:
        finom_plan_1d(x, y, f, g, 0.0, gamma)
    assert e.value.status == FINOM_E_ARG
    with pytest.raises(FinomError):
        finom_plan_1d(x, y, f, g, float("nan"), gamma)
    L = load()
    s = torch.cuda.current_stream().cuda_stream
    assert L.finom_plan_1d(x.data_ptr(), 4, y.data_ptr(), 3, f.data_ptr(), g.data_ptr(), 0.1,
                           gamma.data_ptr(), 2, s) == FINOM_E_ARG          # ld < m
    assert L.finom_plan_1d(x.data_ptr(), 0, y.data_ptr(), 3, f.data_ptr(), g.data_ptr(), 0.1,
                           gamma.data_ptr(), 3, s) == FINOM_E_ARG          # empty mesh
    assert L.finom_plan_1d(None, 4, y.data_ptr(), 3, f.data_ptr(), g.data_ptr(), 0.1,
                           gamma.data_ptr(), 3, s) == FINOM_E_ARG
    torch.cuda.synchronize()
    assert np.all(host(gamma) == 5.0)


# ----------------------------------------------------------------------------
# Section 4's plan-difference column
# ----------------------------------------------------------------------------

def _finom_1d(p, precision=0):
    from paper_2605_26659_amd import sinkhorn_w1_1d
    res, f, g = sinkhorn_w1_1d(dev(p.x), dev(p.y), dev(p.u), dev(p.v), p.eps, 0.0, p.itr_max,
                               precision=precision)
    assert res["iters"] == p.itr_max
    return f, g


# Tables 1 and 2 print ||Delta Gamma||_F between 5e-18 and 5e-17 for these
# runs. Here one side is FINOM on the GPU and the other the oracle's dense
# iteration, and the two runs round differently (sums in another order, other
# exponential implementations), so the bound allows an order of magnitude.
PAPER_FP64_BOUND = 1e-15


@pytest.mark.parametrize("kind,n", [("chebyshev", 500), ("chebyshev", 2000), ("random", 500),
                                    ("random", 2000)])
def test_paper_1d_plan_difference(kind, n):
    from paper_2605_26659_amd import finom_plan_diff_1d
    p = (wl.paper_chebyshev_1d if kind == "chebyshev" else wl.paper_random_1d)(n)
    f, g = _finom_1d(p)
    fd, gd, itd, _ = clib.dense_sinkhorn_1d(p.x, p.y, p.u, p.v, p.eps, 0.0, p.itr_max)
    assert itd == p.itr_max
    got = float(host(finom_plan_diff_1d(dev(p.x), dev(p.y), f, g, dev(fd), dev(gd), p.eps))[0])
    ref = dense.plan_difference(dense.plan_1d(p.x, p.y, host(f), host(g), p.eps),
                                dense.plan_1d(p.x, p.y, fd, gd, p.eps))
    print(f"\n[plan difference] {kind} N={n}: GPU {got:.3e}, oracle {ref:.3e}", flush=True)
    assert 0.0 < got <= PAPER_FP64_BOUND and ref <= PAPER_FP64_BOUND
    # the same potentials on both sides: the two evaluations of the norm
    # differ only by the exponentials' rounding, small next to the entries'
    # differences
    assert abs(got - ref) <= 0.05 * ref


@pytest.mark.parametrize("side", [10, 20, 40])
def test_paper_2d_plan_difference(side):
    from paper_2605_26659_amd import finom_plan_diff_2d, sinkhorn_w1_2d
    p = wl.paper_random_2d(side)
    res, F, G = sinkhorn_w1_2d(dev(p.x1), dev(p.y1), dev(p.x2), dev(p.y2), dev(p.u.ravel(order="F")),
                               dev(p.v.ravel(order="F")), p.eps, 0.0, p.itr_max)
    assert res["iters"] == p.itr_max
    # the standard iteration with the full (NM) x (NM) kernel where it is
    # small; at 40 x 40 with dense K_x and K_y applied axis by axis
    r = dense.sinkhorn_2d(p.x1, p.y1, p.x2, p.y2, p.u, p.v, p.eps, 0.0, p.itr_max, full=side <= 20)
    Fd, Gd = r.f.ravel(order="F"), r.g.ravel(order="F")
    mesh = [dev(a) for a in (p.x1, p.y1, p.x2, p.y2)]
    got = float(host(finom_plan_diff_2d(*mesh, F, G, dev(Fd), dev(Gd), p.eps))[0])
    ref = dense.plan_difference(dense.plan_2d(p.x1, p.y1, p.x2, p.y2, host(F), host(G), p.eps),
                                dense.plan_2d(p.x1, p.y1, p.x2, p.y2, Fd, Gd, p.eps))
    print(f"\n[plan difference] 2D {side}x{side}: GPU {got:.3e}, oracle {ref:.3e}", flush=True)
    assert 0.0 < got <= PAPER_FP64_BOUND and ref <= PAPER_FP64_BOUND
    assert abs(got - ref) <= 0.05 * ref


def test_plan_2d_full_paper_size_sampled():
    """The largest plan of section 4.3 (160 x 160 grids: 25600 x 25600 FP64
    entries, 5.2 GB), exported whole on the device; sampled entries against
    the oracle's definition, row sums against the marginal u."""
    from paper_2605_26659_amd import finom_plan_2d, sinkhorn_w1_2d
    torch = pytest.importorskip("torch")
    p = wl.paper_random_2d(160, iters=50)
    mesh = [dev(a) for a in (p.x1, p.y1, p.x2, p.y2)]
    res, F, G = sinkhorn_w1_2d(*mesh, dev(p.u.ravel(order="F")), dev(p.v.ravel(order="F")), p.eps, 0.0, 50)
    gamma = finom_plan_2d(*mesh, F, G, p.eps)
    assert tuple(gamma.shape) == (25600, 25600)
    rng = np.random.default_rng(160)
    r = rng.integers(0, 25600, 20000)
    c = rng.integers(0, 25600, 20000)
    got = host(gamma[torch.as_tensor(r, device="cuda"), torch.as_tensor(c, device="cuda")])
    want = dense.plan_entries([p.x1, p.y1], [p.x2, p.y2], host(F), host(G), p.eps, r, c)
    np.testing.assert_allclose(got, want, rtol=RTOL_ENTRY, atol=ATOL_ENTRY)
    # the last update is phi = u / K psi: every row sums to its mass
    rows = host(gamma.sum(dim=1))
    del gamma
    np.testing.assert_allclose(rows, p.u.ravel(order="F"), rtol=1e-10, atol=0)


def test_plan_1d_full_paper_size_sampled():
    """Section 4.1's largest run (Chebyshev nodes, N = 8000, 1000 iterations,
    eps = 0.01): the 8000 x 8000 plan exported whole, sampled entries against
    the oracle computed one by one, row sums against u."""
    from paper_2605_26659_amd import finom_plan_1d
    torch = pytest.importorskip("torch")
    p = wl.paper_chebyshev_1d(8000)
    f, g = _finom_1d(p)
    gamma = finom_plan_1d(dev(p.x), dev(p.y), f, g, p.eps)
    rng = np.random.default_rng(8000)
    r = rng.integers(0, 8000, 20000)
    c = rng.integers(0, 8000, 20000)
    # half of the samples near the diagonal, where the mass is
    c[:10000] = np.clip(r[:10000] + rng.integers(-40, 41, 10000), 0, 7999)
    got = host(gamma[torch.as_tensor(r, device="cuda"), torch.as_tensor(c, device="cuda")])
    want = dense.plan_entries([p.x], [p.y], host(f), host(g), p.eps, r, c)
    np.testing.assert_allclose(got, want, rtol=RTOL_ENTRY, atol=ATOL_ENTRY)
    rows = host(gamma.sum(dim=1))
    del gamma
    np.testing.assert_allclose(rows, p.u, rtol=1e-10, atol=0)
