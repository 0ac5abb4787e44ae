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
