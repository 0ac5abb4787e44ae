"""ctypes front end to oracle.c (test infrastructure; see the package docstring).

``build()`` compiles oracle.c with gcc (no GPU code, IEEE semantics: no
fast-math). Functions raise if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_l = C.c_long
_d = C.c_double


def build(force: bool = True) -> Path:
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            raise RuntimeError("oracle/liboracle.so is not built; run oracle.clib.build()")
        L = C.CDLL(str(_LIB))
        L.orc_dividing_index.argtypes = [_dp, _l, _dp, _l, _lp]
        L.orc_vector_rep.argtypes = [_dp, _l, _dp, _l, _d, _lp, _dp, _lp, _dp, _dp, _lp, _dp]
        L.orc_rep_matvec.argtypes = [_l, _l, _lp, _dp, _lp, _dp, _dp, _lp, _dp, _dp, _dp,
                                     C.POINTER(_l), C.POINTER(_l)]
        L.orc_finom_logmatvec.argtypes = [_dp, _l, _dp, _l, _dp, _d, _dp]
        L.orc_sinkhorn_1d.argtypes = [_dp, _l, _dp, _l, _dp, _dp, _d, _d, _l, _dp, _dp,
                                      C.POINTER(_d), C.c_void_p]
        L.orc_sinkhorn_1d.restype = _l
        L.orc_sinkhorn_2d.argtypes = [_dp, _l, _dp, _l, _dp, _l, _dp, _l, _dp, _dp, _d, _d,
                                      _l, _dp, _dp, C.POINTER(_d), C.c_void_p, C.c_int]
        L.orc_sinkhorn_2d.restype = _l
        L.orc_finom_logmatvec_2d.argtypes = [_dp, _l, _dp, _l, _dp, _l, _dp, _l, _dp, _d,
                                             _dp, C.c_int]
        L.orc_dense_logmatvec.argtypes = [_dp, _l, _dp, _l, _dp, _d, _dp, C.c_void_p, _l,
                                          C.c_int]
        L.orc_dense_cost_1d.argtypes = [_dp, _l, _dp, _l, _dp, _dp, _d, C.c_int]
        L.orc_dense_cost_1d.restype = _d
        L.orc_dense_sinkhorn_1d.argtypes = [_dp, _l, _dp, _l, _dp, _dp, _d, _d, _l, _dp, _dp,
                                            C.POINTER(_d), C.c_int]
        L.orc_dense_sinkhorn_1d.restype = _l
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _threads(t):
    return int(t) if t else min(16, os.cpu_count() or 1)


def dividing_index(x, y):
    x, y = _f64(x), _f64(y)
    z = np.zeros(len(x), np.int64)
    lib().orc_dividing_index(x, len(x), y, len(y), z)
    return z


def vector_rep(x, y, eps):
    """(zeta, r, eta list, r', eta' list) per Theorems 2.1 and 2.2 (0-based)."""
    x, y = _f64(x), _f64(y)
    n, m = len(x), len(y)
    zeta = np.zeros(n, np.int64)
    r = np.zeros(max(n - 1, 1)); rp = np.zeros(max(n - 1, 1))
    eta = np.zeros(max(m, 1)); etap = np.zeros(max(m, 1))
    eo = np.zeros(n + 1, np.int64); epo = np.zeros(n + 1, np.int64)
    lib().orc_vector_rep(x, n, y, m, float(eps), zeta, r, eo, eta, rp, epo, etap)
    etas = [eta[eo[i]:eo[i + 1]].copy() for i in range(n)]
    etaps = [etap[epo[i]:epo[i + 1]].copy() for i in range(n)]
    return zeta, r[: n - 1], etas, rp[: n - 1], etaps, (r, eo, eta, rp, epo, etap)


def rep_matvec(x, y, psi, eps):
    """K psi via eq. (p-DP)/(q-DP) from the stored representation, with the
    counts of multiplications and additions."""
    x, y, psi = _f64(x), _f64(y), _f64(psi)
    n, m = len(x), len(y)
    zeta, _, _, _, _, (r, eo, eta, rp, epo, etap) = vector_rep(x, y, eps)
    out = np.zeros(n)
    nm, na = _l(0), _l(0)
    lib().orc_rep_matvec(n, m, zeta, r, eo, eta, rp, epo, etap, psi, out,
                         C.byref(nm), C.byref(na))
    return out, int(nm.value), int(na.value), zeta


def finom_logmatvec(xr, yc, g, eps):
    xr, yc, g = _f64(xr), _f64(yc), _f64(g)
    out = np.zeros(len(xr))
    lib().orc_finom_logmatvec(xr, len(xr), yc, len(yc), g, float(eps), out)
    return out


def finom_logmatvec_2d(xr, yr, xc, yc, G, eps, threads=None):
    """eps ln(K e^{G/eps}) on a column-major grid; G is (len(xc), len(yc))."""
    xr, yr, xc, yc = map(_f64, (xr, yr, xc, yc))
    Gf = np.asfortranarray(G, dtype=np.float64).ravel(order="F")
    T = np.zeros(len(xr) * len(yr))
    lib().orc_finom_logmatvec_2d(xr, len(xr), yr, len(yr), xc, len(xc), yc, len(yc),
                                 Gf, float(eps), T, _threads(threads))
    return T.reshape((len(xr), len(yr)), order="F")


def sinkhorn_1d(x, y, u, v, eps, tol, itr_max, trace=False):
    """Algorithm 1 on the CPU. Returns (f, g, iters, err[, err_trace])."""
    x, y, u, v = map(_f64, (x, y, u, v))
    f = np.zeros(len(x)); g = np.zeros(len(y))
    err = _d(0.0)
    tr = np.zeros(int(itr_max) + 1) if trace else None
    it = lib().orc_sinkhorn_1d(x, len(x), y, len(y), u, v, float(eps), float(tol),
                               int(itr_max), f, g, C.byref(err),
                               tr.ctypes.data if trace else None)
    if trace:
        return f, g, int(it), float(err.value), tr[: it + 1]
    return f, g, int(it), float(err.value)


def sinkhorn_2d(x1, y1, x2, y2, u, v, eps, tol, itr_max, threads=None, trace=False):
    """Algorithm 2 on the CPU. u is (N1, M1), v is (N2, M2) arrays."""
    x1, y1, x2, y2 = map(_f64, (x1, y1, x2, y2))
    uf = np.asarray(u, np.float64).ravel(order="F").copy()
    vf = np.asarray(v, np.float64).ravel(order="F").copy()
    F = np.zeros(uf.size); G = np.zeros(vf.size)
    err = _d(0.0)
    tr = np.zeros(int(itr_max) + 1) if trace else None
    it = lib().orc_sinkhorn_2d(x1, len(x1), y1, len(y1), x2, len(x2), y2, len(y2), uf, vf,
                               float(eps), float(tol), int(itr_max), F, G, C.byref(err),
                               tr.ctypes.data if trace else None, _threads(threads))
    F = F.reshape((len(x1), len(y1)), order="F")
    G = G.reshape((len(x2), len(y2)), order="F")
    if trace:
        return F, G, int(it), float(err.value), tr[: it + 1]
    return F, G, int(it), float(err.value)


def dense_logmatvec(xr, yc, g, eps, rows=None, threads=None):
    xr, yc, g = _f64(xr), _f64(yc), _f64(g)
    if rows is None:
        out = np.zeros(len(xr))
        lib().orc_dense_logmatvec(xr, len(xr), yc, len(yc), g, float(eps), out, None, 0,
                                  _threads(threads))
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        out = np.zeros(len(rows))
        lib().orc_dense_logmatvec(xr, len(xr), yc, len(yc), g, float(eps), out,
                                  rows.ctypes.data, len(rows), _threads(threads))
    return out


def dense_cost_1d(x, y, f, g, eps, threads=None):
    x, y, f, g = map(_f64, (x, y, f, g))
    return float(lib().orc_dense_cost_1d(x, len(x), y, len(y), f, g, float(eps),
                                         _threads(threads)))


def dense_sinkhorn_1d(x, y, u, v, eps, tol, itr_max, threads=None):
    x, y, u, v = map(_f64, (x, y, u, v))
    f = np.zeros(len(x)); g = np.zeros(len(y))
    err = _d(0.0)
    it = lib().orc_dense_sinkhorn_1d(x, len(x), y, len(y), u, v, float(eps), float(tol),
                                     int(itr_max), f, g, C.byref(err), _threads(threads))
    return f, g, int(it), float(err.value)
