"""Helpers for the GPU parity tests: device tensors and shared cases."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rand_meshes(seed, n, m, ties=False, dup=False):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, n))
    y = np.sort(rng.uniform(0, 1, m))
    if ties:
        k = max(1, min(n, m) // 3)
        y[rng.choice(m, k, replace=False)] = x[rng.choice(n, k, replace=False)]
        y = np.sort(y)
    if dup:
        x[: n // 3] = np.round(x[: n // 3], 2)   # repeated coordinates
        x = np.sort(x)
    return x, y


# tolerances on |out_gpu - out_oracle| / eps (log domain), i.e. on the relative
# error of each entry of K psi
TOL_F64 = 1e-12
TOL_F32 = 2e-6


def check_slack(g, t, eps, v):
    """How far two FP64 evaluations of the marginal error sum_j |exp((g_j +
    t_j)/eps) - v_j| of one pair can differ. The log values (g + t) / eps of
    magnitude up to a = (max|g| + max|t|) / eps are formed through a log-form
    recurrence of up to len(v) sequential steps on one side (the oracle's)
    and from rounded potentials on the other, so each carries a rounding that
    grows like sqrt(len) units of 2^-53 of a; each term |psi_j (K^T phi)_j -
    v_j| moves by that much relative to v_j. Four times that, on the total
    mass. The same bound serves the u side, whose exact value is 0."""
    a = (np.max(np.abs(g)) + np.max(np.abs(t))) / eps
    return 4.0 * np.sqrt(len(v)) * 2.0 ** -53 * a * float(np.sum(v))
