"""The entry point that allocates nothing (finom_matvec_noalloc) against the
one it mirrors (finom_matvec), through the C ABI: two calls in a row, the
second on a smaller input, must give the same bits as finom_matvec, and both
agree with the oracle's dense product (section 2.1's K psi)."""
import numpy as np
import pytest

from gpuhelp import TOL_F32, TOL_F64, dev, host, rand_meshes, torch_cuda

pytestmark = pytest.mark.gpu


def _case(seed, n, m, eps):
    x, y = rand_meshes(seed, n, m, ties=True)
    rng = np.random.default_rng(seed + 1)
    g = rng.normal(scale=0.3 * eps * 50, size=m)
    return x, y, g, eps


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_matvec_on_two_calls(precision):
    torch = torch_cuda()
    from oracle import clib
    from paper_2605_26659_amd import finom_matvec, finom_matvec_noalloc
    tol = TOL_F64 if precision == 0 else TOL_F32
    # several tiles with a ragged tail, then a smaller problem (fewer tiles)
    for seed, n, m, eps in ((11, 70001, 65537, 1e-2), (12, 3001, 2500, 1e-3)):
        print(f"noalloc case seed={seed} n={n} m={m} eps={eps} precision={precision}", flush=True)
        x, y, g, eps = _case(seed, n, m, eps)
        dx, dy, dg = dev(x), dev(y), dev(g)
        out_na = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        finom_matvec_noalloc(dx, dy, eps, dg, out_na, precision=precision, domain=1)
        ref = finom_matvec(dx, dy, eps, dg, precision=precision, domain=1, skip_checks=True)
        torch.cuda.synchronize()
        a, b = host(out_na), host(ref)
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
        want = clib.finom_logmatvec(x, y, g, eps)
        assert float(np.max(np.abs(a - want)) / eps) <= tol


def test_noalloc_linear_domain_and_limit():
    torch = torch_cuda()
    from paper_2605_26659_amd import FINOM_E_ARG, FinomError, finom_matvec, finom_matvec_noalloc
    x, y, _, eps = _case(13, 5000, 4097, 0.05)
    psi = np.random.default_rng(14).uniform(0.1, 1.0, 4097)
    dx, dy, dp = dev(x), dev(y), dev(psi)
    out = torch.empty(5000, dtype=torch.float64, device="cuda")
    finom_matvec_noalloc(dx, dy, eps, dp, out, domain=0)
    ref = finom_matvec(dx, dy, eps, dp, domain=0, skip_checks=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), host(ref))
    # beyond the fixed array: refused on the host before anything is enqueued
    big = torch.zeros(1 << 21, dtype=torch.float64, device="cuda")
    big2 = torch.zeros((1 << 21) + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(FinomError) as e:
        finom_matvec_noalloc(big2, big, eps, big, big2)
    assert e.value.status == FINOM_E_ARG
