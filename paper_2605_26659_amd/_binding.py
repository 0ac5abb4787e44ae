"""ctypes binding to libfinom.so (argument marshalling only).

Every numerical step runs in the HIP library. Tensors are torch CUDA
(HIP) float64 tensors; the stream is torch's current stream unless one is
given. If the library is not built, importing the entry points raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import re
import weakref
from pathlib import Path

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libfinom.so"
HEADER = _PKG.parent / "include" / "finom.h"

FINOM_OK = 0
FINOM_NOT_CONVERGED = 1
FINOM_E_ARG = -1
FINOM_E_UNSORTED = -2
FINOM_E_MASS = -3
FINOM_E_NOMEM = -4
FINOM_E_HIP = -5
FINOM_E_ADMIT = -6
FINOM_E_NUMERIC = -7


class FinomError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = ""
        if status in (FINOM_E_HIP, FINOM_E_NOMEM):
            try:
                detail = load().finom_last_error().decode()
            except Exception:
                detail = ""
        super().__init__(f"{where}: {strerror(status)} (status {status})" + (f": {detail}" if detail else ""))


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("domain", C.c_int32),
                ("skip_checks", C.c_int32), ("graph_iters", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("w1", C.c_double), ("marginal_err", C.c_double), ("iters", C.c_int64),
                ("converged", C.c_int32), ("status", C.c_int32), ("loop_ms", C.c_double),
                ("sweeps", C.c_int64), ("fast", C.c_int32), ("resumes", C.c_int32)]

    def as_dict(self):
        return {"w1": self.w1, "marginal_err": self.marginal_err, "iters": int(self.iters),
                "converged": bool(self.converged), "status": int(self.status),
                "loop_ms": float(self.loop_ms), "sweeps": int(self.sweeps), "fast": int(self.fast),
                "resumes": int(self.resumes)}


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("reserved", C.c_int32),
                ("n1", C.c_int64), ("m1", C.c_int64), ("n2", C.c_int64), ("m2", C.c_int64),
                ("x1", C.c_void_p), ("y1", C.c_void_p), ("x2", C.c_void_p), ("y2", C.c_void_p),
                ("u", C.c_void_p), ("v", C.c_void_p),
                ("eps", C.c_double), ("tol", C.c_double), ("itr_max", C.c_int64),
                ("f_out", C.c_void_p), ("g_out", C.c_void_p)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("res", Result), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("live", C.c_int64), ("queued", C.c_int64),
                ("rounds", C.c_int64), ("grid_pt_iters", C.c_double), ("busy_ms", C.c_double),
                ("hbm_used", C.c_uint64), ("hbm_budget", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = C.c_void_p
_i64 = C.c_int64
_d = C.c_double


def declared_functions():
    """Names of the functions include/finom.h declares."""
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("FINOM")))


def load(path: os.PathLike | None = None):
    """Load the library (no GPU call is made)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2605_26659_amd.build` "
                           "(there is no CPU fallback)")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so the process holds one runtime (two runtimes in one process do not
    # both see the device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(str(p))
    L.finom_matvec.argtypes = [_vp, _i64, _vp, _i64, _d, _vp, _vp, C.POINTER(Opts), _vp]
    L.dense_matvec.argtypes = L.finom_matvec.argtypes
    L.finom_matvec_noalloc.argtypes = L.finom_matvec.argtypes
    L.dense_matvec_2d.argtypes = [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _d, _vp, _vp, C.c_int32, _vp]
    L.sinkhorn_w1_1d.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _d, _d, _i64, C.POINTER(Opts),
                                 _vp, _vp, C.POINTER(Result), _vp]
    L.finom_strerror.restype = C.c_char_p
    L.finom_strerror.argtypes = [C.c_int]
    L.finom_version.restype = C.c_char_p
    L.finom_last_error.restype = C.c_char_p
    L.finom_release.restype = None
    if hasattr(L, "sinkhorn_w1_2d"):
        L.sinkhorn_w1_2d.argtypes = [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _d, _d,
                                     _i64, C.POINTER(Opts), _vp, _vp, C.POINTER(Result), _vp]
    L.sinkhorn_w1_nd.argtypes = [C.c_int32, C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_i64),
                                 C.POINTER(_vp), _vp, _vp, _d, _d, _i64, C.POINTER(Opts), _vp, _vp,
                                 C.POINTER(Result), _vp]
    L.finom_plan_1d.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _d, _vp, _i64, _vp]
    L.finom_plan_2d.argtypes = [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _d, _vp,
                                _i64, _vp]
    L.finom_plan_diff_1d.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _d, _vp, _vp]
    L.finom_plan_diff_2d.argtypes = [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp,
                                     _vp, _d, _vp, _vp]
    L.finom_batch.argtypes = [C.POINTER(Problem), _i64, C.POINTER(Opts), C.POINTER(Result), _vp]
    L.finom_footprint.argtypes = [C.POINTER(Problem), C.POINTER(Opts)]
    L.finom_footprint.restype = _i64
    L.finom_server_create.argtypes = [C.c_uint64, C.POINTER(Opts), C.POINTER(_vp)]
    L.finom_server_submit.argtypes = [_vp, C.POINTER(Problem), C.POINTER(_i64)]
    L.finom_server_poll.argtypes = [_vp, C.POINTER(Completion), _i64, C.POINTER(_i64), C.c_int32]
    L.finom_server_stats_get.argtypes = [_vp, C.POINTER(ServerStats)]
    L.finom_server_destroy.argtypes = [_vp]
    L.finom_server_destroy.restype = None
    L.finom_autotune.argtypes = [C.c_int32, C.c_char_p, _vp]
    L.finom_tile_config.argtypes = [C.c_int32, _i64]
    if path is None:
        _lib = L
        atexit.register(_release_at_exit)
    return L


_servers = weakref.WeakSet()


def _release_at_exit():
    """Before the interpreter and the HIP runtime shut down: stop live
    servers, wait for the device, and free the library's cached device and
    pinned workspace (finom_release), so nothing of the library is left for
    the runtime's own teardown."""
    if _lib is None:
        return
    for srv in list(_servers):
        try:
            srv.close()
        except Exception:
            pass
    try:
        torch = _torch()
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
        _lib.finom_release()
    except Exception:
        pass


def strerror(status: int) -> str:
    try:
        return load().finom_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


# ----------------------------------------------------------------------------
# torch plumbing
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream))


def _dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _opts(precision=0, domain=0, skip_checks=False, graph_iters=0):
    return Opts(int(precision), int(domain), int(bool(skip_checks)), int(graph_iters))


def _check(st, where, allow_warn=True):
    if st < 0 or (st > 0 and not allow_warn):
        raise FinomError(st, where)
    return st


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ----------------------------------------------------------------------------

def finom_matvec(x_rows, y_cols, eps, inp, out=None, *, precision=0, domain=0,
                 skip_checks=False, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(x_rows.numel(), dtype=torch.float64, device=x_rows.device)
    st = load().finom_matvec(_dev(x_rows, "x_rows"), x_rows.numel(), _dev(y_cols, "y_cols"),
                             y_cols.numel(), float(eps), _dev(inp, "in"), _dev(out, "out"),
                             C.byref(_opts(precision, domain, skip_checks)), _stream_ptr(stream))
    _check(st, "finom_matvec")
    return out


def finom_matvec_noalloc(x_rows, y_cols, eps, inp, out, *, precision=0, domain=0, stream=None):
    """finom_matvec through the entry point that allocates nothing; `out` is
    required (n float64 values on the device). No device-side input checks."""
    st = load().finom_matvec_noalloc(_dev(x_rows, "x_rows"), x_rows.numel(), _dev(y_cols, "y_cols"),
                                     y_cols.numel(), float(eps), _dev(inp, "in"), _dev(out, "out"),
                                     C.byref(_opts(precision, domain, True)), _stream_ptr(stream))
    _check(st, "finom_matvec_noalloc")
    return out


def dense_matvec(x_rows, y_cols, eps, inp, out=None, *, precision=0, domain=0,
                 skip_checks=False, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(x_rows.numel(), dtype=torch.float64, device=x_rows.device)
    st = load().dense_matvec(_dev(x_rows, "x_rows"), x_rows.numel(), _dev(y_cols, "y_cols"),
                             y_cols.numel(), float(eps), _dev(inp, "in"), _dev(out, "out"),
                             C.byref(_opts(precision, domain, skip_checks)), _stream_ptr(stream))
    _check(st, "dense_matvec")
    return out


def dense_matvec_2d(x1, y1, x2, y2, eps, inp, out=None, *, full=False, stream=None):
    """eps ln (K e^{in/eps}) on tensor meshes, densely: the per-axis matrix
    products on the matrix cores (full=False) or the full (n1 m1) x (n2 m2)
    product (full=True). in: n2*m2, out: n1*m1, flat column-major."""
    torch = _torch()
    n1, m1, n2, m2 = x1.numel(), y1.numel(), x2.numel(), y2.numel()
    if inp.numel() != n2 * m2:
        raise ValueError("in holds n2 * m2 values")
    if out is None:
        out = torch.empty(n1 * m1, dtype=torch.float64, device=x1.device)
    st = load().dense_matvec_2d(_dev(x1, "x1"), n1, _dev(y1, "y1"), m1, _dev(x2, "x2"), n2, _dev(y2, "y2"), m2,
                                float(eps), _dev(inp, "in"), _dev(out, "out"), int(bool(full)),
                                _stream_ptr(stream))
    _check(st, "dense_matvec_2d")
    return out


def sinkhorn_w1_1d(x, y, u, v, eps, tol, itr_max, *, precision=0, skip_checks=False,
                   graph_iters=0, f_out=None, g_out=None, want_potentials=True, stream=None):
    """Returns (result dict, f, g); f, g are eps ln phi / eps ln psi (device)."""
    torch = _torch()
    if want_potentials:
        if f_out is None:
            f_out = torch.empty(x.numel(), dtype=torch.float64, device=x.device)
        if g_out is None:
            g_out = torch.empty(y.numel(), dtype=torch.float64, device=y.device)
    res = Result()
    st = load().sinkhorn_w1_1d(_dev(x, "x"), x.numel(), _dev(y, "y"), y.numel(), _dev(u, "u"),
                               _dev(v, "v"), float(eps), float(tol), int(itr_max),
                               C.byref(_opts(precision, 0, skip_checks, graph_iters)),
                               _dev(f_out, "f_out") if f_out is not None else None,
                               _dev(g_out, "g_out") if g_out is not None else None,
                               C.byref(res), _stream_ptr(stream))
    _check(st, "sinkhorn_w1_1d")
    return res.as_dict(), f_out, g_out


def sinkhorn_w1_2d(x1, y1, x2, y2, u, v, eps, tol, itr_max, *, precision=0, skip_checks=False,
                   graph_iters=0, f_out=None, g_out=None, want_potentials=True, stream=None):
    """u is (len(x1), len(y1)) and v is (len(x2), len(y2)), both stored
    column-major (the paper's grid order): pass ``t.T.contiguous().T``-style
    tensors or flat column-major vectors. Returns (result, F, G) as flat
    column-major vectors."""
    torch = _torch()
    n1, m1, n2, m2 = x1.numel(), y1.numel(), x2.numel(), y2.numel()
    if want_potentials:
        if f_out is None:
            f_out = torch.empty(n1 * m1, dtype=torch.float64, device=x1.device)
        if g_out is None:
            g_out = torch.empty(n2 * m2, dtype=torch.float64, device=x1.device)
    res = Result()
    st = load().sinkhorn_w1_2d(_dev(x1, "x1"), n1, _dev(y1, "y1"), m1, _dev(x2, "x2"), n2,
                               _dev(y2, "y2"), m2, _dev(u, "u"), _dev(v, "v"), float(eps),
                               float(tol), int(itr_max),
                               C.byref(_opts(precision, 0, skip_checks, graph_iters)),
                               _dev(f_out, "f_out") if f_out is not None else None,
                               _dev(g_out, "g_out") if g_out is not None else None,
                               C.byref(res), _stream_ptr(stream))
    _check(st, "sinkhorn_w1_2d")
    return res.as_dict(), f_out, g_out


def sinkhorn_w1_nd(x_src, x_tgt, u, v, eps, tol, itr_max, *, precision=0, skip_checks=False,
                   graph_iters=0, f_out=None, g_out=None, want_potentials=True, stream=None):
    """d-dimensional tensor meshes: x_src, x_tgt are sequences of d axis
    coordinate tensors; u, v flat column-major grids (axis 0 fastest).
    Returns (result, F, G) as flat column-major vectors."""
    torch = _torch()
    d = len(x_src)
    if len(x_tgt) != d:
        raise ValueError("x_src and x_tgt need the same number of axes")
    ns = (_i64 * d)(*[t.numel() for t in x_src])
    nt = (_i64 * d)(*[t.numel() for t in x_tgt])
    ps = (_vp * d)(*[_dev(t, f"x_src[{i}]").value for i, t in enumerate(x_src)])
    pt = (_vp * d)(*[_dev(t, f"x_tgt[{i}]").value for i, t in enumerate(x_tgt)])
    na = math.prod(t.numel() for t in x_src)
    nb = math.prod(t.numel() for t in x_tgt)
    if want_potentials:
        if f_out is None:
            f_out = torch.empty(na, dtype=torch.float64, device=u.device)
        if g_out is None:
            g_out = torch.empty(nb, dtype=torch.float64, device=u.device)
    res = Result()
    st = load().sinkhorn_w1_nd(d, ns, ps, nt, pt, _dev(u, "u"), _dev(v, "v"), float(eps), float(tol),
                               int(itr_max), C.byref(_opts(precision, 0, skip_checks, graph_iters)),
                               _dev(f_out, "f_out") if f_out is not None else None,
                               _dev(g_out, "g_out") if g_out is not None else None,
                               C.byref(res), _stream_ptr(stream))
    _check(st, "sinkhorn_w1_nd")
    return res.as_dict(), f_out, g_out


def finom_plan_1d(x, y, f, g, eps, gamma=None, *, ld=None, stream=None):
    """Dense plan (n, ld) with gamma[i, j] = exp((f_i + g_j - |x_i - y_j|)/eps)
    for j < m (device tensor; columns j >= m are left as they were)."""
    torch = _torch()
    n, m = x.numel(), y.numel()
    ld = m if ld is None else int(ld)
    if gamma is None:
        gamma = torch.empty((n, ld), dtype=torch.float64, device=x.device)
    if gamma.numel() < n * ld:
        raise ValueError("gamma holds fewer than n * ld doubles")
    st = load().finom_plan_1d(_dev(x, "x"), n, _dev(y, "y"), m, _dev(f, "f"), _dev(g, "g"),
                              float(eps), _dev(gamma, "gamma"), ld, _stream_ptr(stream))
    _check(st, "finom_plan_1d")
    return gamma


def finom_plan_2d(x1, y1, x2, y2, f, g, eps, gamma=None, *, ld=None, stream=None):
    """Dense plan of tensor meshes, (n1 m1, ld), rows and columns in
    column-major grid order; f, g flat column-major (as sinkhorn_w1_2d returns)."""
    torch = _torch()
    n1, m1, n2, m2 = x1.numel(), y1.numel(), x2.numel(), y2.numel()
    ld = n2 * m2 if ld is None else int(ld)
    if gamma is None:
        gamma = torch.empty((n1 * m1, ld), dtype=torch.float64, device=x1.device)
    if gamma.numel() < n1 * m1 * ld:
        raise ValueError("gamma holds fewer than n1 * m1 * ld doubles")
    st = load().finom_plan_2d(_dev(x1, "x1"), n1, _dev(y1, "y1"), m1, _dev(x2, "x2"), n2,
                              _dev(y2, "y2"), m2, _dev(f, "f"), _dev(g, "g"), float(eps),
                              _dev(gamma, "gamma"), ld, _stream_ptr(stream))
    _check(st, "finom_plan_2d")
    return gamma


def finom_plan_diff_1d(x, y, fa, ga, fb, gb, eps, out=None, *, stream=None):
    """||Gamma_a - Gamma_b||_F as a one-element device tensor."""
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    st = load().finom_plan_diff_1d(_dev(x, "x"), x.numel(), _dev(y, "y"), y.numel(),
                                   _dev(fa, "fa"), _dev(ga, "ga"), _dev(fb, "fb"), _dev(gb, "gb"),
                                   float(eps), _dev(out, "out"), _stream_ptr(stream))
    _check(st, "finom_plan_diff_1d")
    return out


def finom_plan_diff_2d(x1, y1, x2, y2, fa, ga, fb, gb, eps, out=None, *, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x1.device)
    st = load().finom_plan_diff_2d(_dev(x1, "x1"), x1.numel(), _dev(y1, "y1"), y1.numel(),
                                   _dev(x2, "x2"), x2.numel(), _dev(y2, "y2"), y2.numel(),
                                   _dev(fa, "fa"), _dev(ga, "ga"), _dev(fb, "fb"), _dev(gb, "gb"),
                                   float(eps), _dev(out, "out"), _stream_ptr(stream))
    _check(st, "finom_plan_diff_2d")
    return out


def finom_release():
    load().finom_release()


def finom_version() -> str:
    return load().finom_version().decode()


# ----------------------------------------------------------------------------
# batches and serving
# ----------------------------------------------------------------------------

def problem_1d(x, y, u, v, eps, tol, itr_max, f_out=None, g_out=None):
    """Descriptor of a 1D problem (device tensors) for finom_batch / FinomServer."""
    return {"dim": 1, "x1": x, "x2": y, "u": u, "v": v, "eps": eps, "tol": tol,
            "itr_max": itr_max, "f_out": f_out, "g_out": g_out}


def problem_2d(x1, y1, x2, y2, u, v, eps, tol, itr_max, f_out=None, g_out=None):
    """Descriptor of a 2D problem; u, v and the outputs are flat column-major."""
    return {"dim": 2, "x1": x1, "y1": y1, "x2": x2, "y2": y2, "u": u, "v": v, "eps": eps,
            "tol": tol, "itr_max": itr_max, "f_out": f_out, "g_out": g_out}


def _problem_struct(d):
    P = Problem()
    P.dim = int(d["dim"])
    P.reserved = 0
    P.n1 = d["x1"].numel()
    P.n2 = d["x2"].numel()
    P.x1 = _dev(d["x1"], "x1")
    P.x2 = _dev(d["x2"], "x2")
    if P.dim == 2:
        P.m1 = d["y1"].numel()
        P.m2 = d["y2"].numel()
        P.y1 = _dev(d["y1"], "y1")
        P.y2 = _dev(d["y2"], "y2")
    else:
        P.m1 = P.m2 = 1
    P.u = _dev(d["u"], "u")
    P.v = _dev(d["v"], "v")
    P.eps = float(d["eps"])
    P.tol = float(d["tol"])
    P.itr_max = int(d["itr_max"])
    P.f_out = _dev(d["f_out"], "f_out") if d.get("f_out") is not None else None
    P.g_out = _dev(d["g_out"], "g_out") if d.get("g_out") is not None else None
    return P


def with_outputs(d):
    """Adds freshly allocated f_out / g_out tensors to a descriptor."""
    torch = _torch()
    out = dict(d)
    dev = d["x1"].device
    if d["dim"] == 1:
        na, nb = d["x1"].numel(), d["x2"].numel()
    else:
        na = d["x1"].numel() * d["y1"].numel()
        nb = d["x2"].numel() * d["y2"].numel()
    out["f_out"] = torch.empty(na, dtype=torch.float64, device=dev)
    out["g_out"] = torch.empty(nb, dtype=torch.float64, device=dev)
    return out


def finom_footprint(d, *, precision=0) -> int:
    return int(load().finom_footprint(C.byref(_problem_struct(d)), C.byref(_opts(precision))))


def finom_batch(problems, *, precision=0, skip_checks=False, graph_iters=0, stream=None):
    """Solves a list of descriptors together. Returns (status, [result dict]);
    each result carries its own status. Raises only for runtime failures."""
    n = len(problems)
    arr = (Problem * max(n, 1))()
    for i, d in enumerate(problems):
        arr[i] = _problem_struct(d)
    res = (Result * max(n, 1))()
    st = load().finom_batch(arr, n, C.byref(_opts(precision, 0, skip_checks, graph_iters)), res,
                            _stream_ptr(stream))
    if st in (FINOM_E_HIP, FINOM_E_NOMEM):
        raise FinomError(st, "finom_batch")
    return st, [res[i].as_dict() for i in range(n)]


def finom_autotune(precision=0, cache_path=None, stream=None):
    st = load().finom_autotune(int(precision), cache_path.encode() if cache_path else None,
                               _stream_ptr(stream))
    _check(st, "finom_autotune")


def finom_tile_config(precision, merged) -> int:
    return int(load().finom_tile_config(int(precision), int(merged)))


class FinomServer:
    """Continuous-batching solver (one host thread and stream of its own).
    Descriptors' tensors are kept referenced until their completion is polled."""

    def __init__(self, hbm_budget_bytes, *, precision=0, graph_iters=0, skip_checks=False):
        self._lib = load()
        h = C.c_void_p()
        st = self._lib.finom_server_create(int(hbm_budget_bytes),
                                           C.byref(_opts(precision, 0, skip_checks, graph_iters)),
                                           C.byref(h))
        _check(st, "finom_server_create")
        self._h = h
        self._keep = {}
        _servers.add(self)

    def submit(self, d, sync=True) -> int:
        """Queues a problem; returns its ticket. With sync, torch's current
        stream is synchronised first so the inputs are complete."""
        if sync:
            _torch().cuda.current_stream().synchronize()
        P = _problem_struct(d)
        t = C.c_int64(0)
        st = self._lib.finom_server_submit(self._h, C.byref(P), C.byref(t))
        _check(st, "finom_server_submit")
        self._keep[int(t.value)] = d
        return int(t.value)

    def poll(self, max_items=256, wait_ms=0):
        buf = (Completion * max(1, max_items))()
        n = C.c_int64(0)
        st = self._lib.finom_server_poll(self._h, buf, int(max_items), C.byref(n), int(wait_ms))
        _check(st, "finom_server_poll")
        out = []
        for i in range(n.value):
            c = buf[i]
            r = c.res.as_dict()
            r.update(ticket=int(c.ticket), latency_ms=float(c.latency_ms),
                     queue_ms=float(c.queue_ms), problem=self._keep.pop(int(c.ticket), None))
            out.append(r)
        return out

    def stats(self):
        s = ServerStats()
        self._lib.finom_server_stats_get(self._h, C.byref(s))
        return s.as_dict()

    def close(self):
        if self._h:
            self._lib.finom_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
