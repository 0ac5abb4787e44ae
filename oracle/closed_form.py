"""Closed forms and brute force that pin the oracle (test infrastructure).

* 1D W1 with cost |x - y| equals the integral of |F_mu - F_nu| (distribution
  functions), a classical identity for the problem of eq. (w1Definition).
* The same value is reached by the monotone (north-west corner) coupling.
* Brute-force LP of eq. (w1Definition) with scipy's HiGHS on tiny inputs.
* Entropic gap: the entropic plan's cost exceeds W1 by at most
  eps * min(H(u), H(v)) (H = Shannon entropy); this follows from comparing the
  objective of eq. (regularized problem) at its minimiser and at the
  unregularised optimum, with the entropy of any coupling between H(u)+H(v)
  and max(H(u), H(v)).
"""
from __future__ import annotations

import numpy as np


def w1_closed_form(x, u, y, v) -> float:
    """integral over the line of |F_mu(t) - F_nu(t)| dt for sorted x, y."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    u = np.asarray(u, np.float64); v = np.asarray(v, np.float64)
    z = np.concatenate([x, y])
    w = np.concatenate([u, -v])
    order = np.argsort(z, kind="mergesort")
    z, w = z[order], w[order]
    cdf_diff = np.cumsum(w)          # F_mu - F_nu just right of z_k
    gaps = np.diff(z)
    return float(np.sum(np.abs(cdf_diff[:-1]) * gaps))


def monotone_coupling(u, v):
    """North-west corner rule: the monotone coupling of two sorted measures."""
    u = np.array(u, np.float64); v = np.array(v, np.float64)
    n, m = len(u), len(v)
    P = np.zeros((n, m))
    i = j = 0
    while i < n and j < m:
        t = min(u[i], v[j])
        P[i, j] = t
        u[i] -= t; v[j] -= t
        if u[i] <= v[j]:
            i += 1
        else:
            j += 1
    return P


def w1_lp(x, u, y, v) -> float:
    """Brute-force LP of eq. (w1Definition); tiny inputs only."""
    from scipy.optimize import linprog
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    n, m = len(x), len(y)
    c = np.abs(x[:, None] - y[None, :]).ravel()
    A = []
    for i in range(n):
        row = np.zeros((n, m)); row[i, :] = 1; A.append(row.ravel())
    for j in range(m):
        col = np.zeros((n, m)); col[:, j] = 1; A.append(col.ravel())
    b = np.concatenate([u, v])
    res = linprog(c, A_eq=np.array(A), b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def w1_lp_points(px, py, u, qx, qy, v) -> float:
    """LP with L1 cost between 2D point clouds (tiny inputs only)."""
    from scipy.optimize import linprog
    n, m = len(px), len(qx)
    c = (np.abs(px[:, None] - qx[None, :]) + np.abs(py[:, None] - qy[None, :])).ravel()
    A = []
    for i in range(n):
        row = np.zeros((n, m)); row[i, :] = 1; A.append(row.ravel())
    for j in range(m):
        col = np.zeros((n, m)); col[:, j] = 1; A.append(col.ravel())
    res = linprog(c, A_eq=np.array(A), b_eq=np.concatenate([u, v]),
                  bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def entropy(p) -> float:
    p = np.asarray(p, np.float64).ravel()
    return float(-np.sum(p * np.log(p)))


def entropic_w1_bounds(x, u, y, v, eps, err=0.0):
    """Interval that <C, Gamma_eps> must lie in, with slack diam*err for
    marginals that are off by err in L1."""
    w = w1_closed_form(x, u, y, v)
    diam = max(x[-1], y[-1]) - min(x[0], y[0])
    gap = eps * min(entropy(u), entropy(v))
    return w - diam * err, w + gap + diam * err
