"""The C ABI library loads and exports every function the header declares
(no GPU call is made)."""
import ctypes

import pytest

from paper_2605_26659_amd import _binding


def test_header_declares_the_boundary():
    names = _binding.declared_functions()
    for must in ("finom_matvec", "dense_matvec", "sinkhorn_w1_1d", "finom_strerror",
                 "finom_release", "finom_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not _binding.LIB_PATH.exists():
        pytest.fail("libfinom.so is not built (run python -m paper_2605_26659_amd.build)")
    lib = ctypes.CDLL(str(_binding.LIB_PATH))
    missing = [n for n in _binding.declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = _binding.load()
    assert lib.finom_strerror(0) == b"ok"
    assert b"sorted" in lib.finom_strerror(-2) or b"decreasing" in lib.finom_strerror(-2)
    assert lib.finom_version().startswith(b"finom-gfx950")


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _binding.load(tmp_path / "nope.so")


def test_header_declares_the_plan_and_nd_entry_points():
    names = _binding.declared_functions()
    for must in ("finom_plan_1d", "finom_plan_2d", "finom_plan_diff_1d", "finom_plan_diff_2d",
                 "sinkhorn_w1_nd"):
        assert must in names


def test_binding_rejects_host_tensors_without_gpu():
    """Argument marshalling refuses host (CPU) tensors, other dtypes and
    mismatched axis lists before anything reaches the library."""
    torch = pytest.importorskip("torch")
    from paper_2605_26659_amd import finom_plan_1d, finom_plan_diff_1d, sinkhorn_w1_nd
    x = torch.zeros(4, dtype=torch.float64)
    g = torch.empty((4, 4), dtype=torch.float64)
    with pytest.raises(TypeError):
        finom_plan_1d(x, x, x, x, 0.1, g)
    with pytest.raises(TypeError):
        finom_plan_diff_1d(x, x, x, x, x, x, 0.1, torch.empty(1, dtype=torch.float64))
    with pytest.raises(ValueError):
        sinkhorn_w1_nd([x, x], [x], x, x, 0.1, 0.0, 1)
