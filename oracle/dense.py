"""Dense FP64 definitions (test infrastructure; see the package docstring).

Everything here is the plain O(N*M) definition, written for reading, not speed:

* kernel matrix K = exp(-C/eps), C_ij = |x_i - y_j|            (section 2.1)
* Sinkhorn scaling iteration psi = v / K^T phi, phi = u / K psi  (eq. iteration)
* loop head check ||diag(psi) K^T phi - v||_1 > tol, cap itr_max (Algorithm 1)
* plan Gamma = diag(phi) K diag(psi) and cost <C, Gamma>         (section 2.1)
* ||Gamma_a - Gamma_b||_F, the plans' difference                  (section 4)
* 2D: K = K_y (x) K_x on column-major grids; products evaluated
  axis by axis as vec(K_x Psi K_y^T) and vec(K_x^T Phi K_y)      (eqs. 2d-kron,
  2d-kpsi, 2d-ktphi; Algorithm 2)

The iteration is carried in the log domain (potentials f = eps ln phi,
g = eps ln psi), which is the log-domain stabilisation of the remark in
section 2.3 applied at every step: exactly the same iterates as the linear
scaling form, without overflow.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_BLOCK = 1 << 22  # matrix entries per block, keeps memory bounded


def kernel_matrix(x: np.ndarray, y: np.ndarray, eps: float) -> np.ndarray:
    """K_ij = exp(-|x_i - y_j| / eps) (section 2.1)."""
    return np.exp(-np.abs(x[:, None] - y[None, :]) / eps)


def cost_matrix(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.abs(x[:, None] - y[None, :])


def _lse_rows(a: np.ndarray) -> np.ndarray:
    """log(sum(exp(a), axis=1)) with a max shift; rows of all -inf give -inf."""
    mx = np.max(a, axis=1)
    safe = np.where(np.isfinite(mx), mx, 0.0)
    s = np.sum(np.exp(a - safe[:, None]), axis=1)
    with np.errstate(divide="ignore"):
        return safe + np.log(s)


def logmatvec(xr: np.ndarray, yc: np.ndarray, g: np.ndarray, eps: float) -> np.ndarray:
    """out_i = eps * ln( sum_j exp((g_j - |xr_i - yc_j|)/eps) ).

    With g = eps ln psi this is eps ln (K psi)_i for the kernel of rows xr and
    columns yc. K^T phi is the same call with the roles of the meshes swapped.
    """
    xr = np.asarray(xr, np.float64)
    yc = np.asarray(yc, np.float64)
    g = np.asarray(g, np.float64)
    out = np.empty(len(xr))
    step = max(1, _BLOCK // max(1, len(yc)))
    for a in range(0, len(xr), step):
        b = min(len(xr), a + step)
        arg = (g[None, :] - np.abs(xr[a:b, None] - yc[None, :])) / eps
        out[a:b] = eps * _lse_rows(arg)
    return out


def log_moment_matvec(xr, yc, g, eps):
    """eps * ln( sum_j |xr_i - yc_j| exp((g_j - |xr_i - yc_j|)/eps) ).

    The cost-weighted product (C o K) psi in log form; used for <C, Gamma>.
    Rows whose every column coincides with them give -inf.
    """
    xr = np.asarray(xr, np.float64)
    yc = np.asarray(yc, np.float64)
    g = np.asarray(g, np.float64)
    out = np.empty(len(xr))
    step = max(1, _BLOCK // max(1, len(yc)))
    for a in range(0, len(xr), step):
        b = min(len(xr), a + step)
        c = np.abs(xr[a:b, None] - yc[None, :])
        with np.errstate(divide="ignore"):
            arg = (g[None, :] - c) / eps + np.log(c)
        out[a:b] = eps * _lse_rows(arg)
    return out


def matvec(xr, yc, psi, eps):
    """Linear-domain K psi (small sizes only; may underflow for small eps)."""
    return kernel_matrix(np.asarray(xr), np.asarray(yc), eps) @ np.asarray(psi)


def marginal_error(g: np.ndarray, t: np.ndarray, v: np.ndarray, eps: float) -> float:
    """||diag(psi) K^T phi - v||_1 with g = eps ln psi and t = eps ln K^T phi."""
    return float(np.sum(np.abs(np.exp((g + t) / eps) - v)))


@dataclass
class SinkhornResult:
    f: np.ndarray
    g: np.ndarray
    iters: int
    err: float
    w1: float
    converged: bool


def transport_cost_1d(x, y, f, g, eps) -> float:
    """<C, Gamma> with Gamma_ij = exp((f_i + g_j - |x_i - y_j|)/eps)."""
    tot = 0.0
    step = max(1, _BLOCK // max(1, len(y)))
    for a in range(0, len(x), step):
        b = min(len(x), a + step)
        c = np.abs(x[a:b, None] - y[None, :])
        tot += float(np.sum(c * np.exp((f[a:b, None] + g[None, :] - c) / eps)))
    return tot


def plan_1d(x, y, f, g, eps) -> np.ndarray:
    """Gamma = diag(phi) K diag(psi) as an n x m matrix (section 2.1):
    Gamma_ij = exp((f_i + g_j - |x_i - y_j|)/eps)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    f = np.asarray(f, np.float64); g = np.asarray(g, np.float64)
    c = cost_matrix(x, y)
    return np.exp((f[:, None] + g[None, :] - c) / eps)


def plan_2d(x1, y1, x2, y2, F, G, eps) -> np.ndarray:
    """Gamma of tensor meshes as an (N1 M1) x (N2 M2) matrix, rows and columns
    in column-major grid order: row k + i N1 is source point (x1_k, y1_i),
    column l + j N2 target point (x2_l, y2_j), and the cost is
    |x1_k - x2_l| + |y1_i - y2_j| (eq. 2d-block-entry). F, G: grids or flat
    column-major vectors."""
    XR, YR = np.meshgrid(np.asarray(x1, np.float64), np.asarray(y1, np.float64), indexing="ij")
    XC, YC = np.meshgrid(np.asarray(x2, np.float64), np.asarray(y2, np.float64), indexing="ij")
    c = (np.abs(XR.ravel(order="F")[:, None] - XC.ravel(order="F")[None, :])
         + np.abs(YR.ravel(order="F")[:, None] - YC.ravel(order="F")[None, :]))
    f = np.asarray(F, np.float64).ravel(order="F")
    g = np.asarray(G, np.float64).ravel(order="F")
    return np.exp((f[:, None] + g[None, :] - c) / eps)


def plan_entries(xs, xt, F, G, eps, rows, cols) -> np.ndarray:
    """Selected entries Gamma[rows[t], cols[t]] of the plan on tensor meshes
    with any number of axes (1D: one axis each), one by one from the
    definition. rows / cols index the column-major grids (axis 0 fastest);
    the cost is sum_a |xs[a]_k - xt[a]_l|."""
    f = np.asarray(F, np.float64).ravel(order="F")
    g = np.asarray(G, np.float64).ravel(order="F")
    out = np.empty(len(rows))
    for t, (r, c) in enumerate(zip(rows, cols)):
        cost = 0.0
        rr, cc = int(r), int(c)
        for a in range(len(xs)):
            k, rr = rr % len(xs[a]), rr // len(xs[a])
            l, cc = cc % len(xt[a]), cc // len(xt[a])
            cost += abs(float(xs[a][k]) - float(xt[a][l]))
        out[t] = np.exp(((f[int(r)] + g[int(c)]) - cost) / eps)
    return out


def plan_difference(gamma_a, gamma_b) -> float:
    """||Gamma_a - Gamma_b||_F, the plan-difference column of section 4's tables."""
    d = np.asarray(gamma_a, np.float64) - np.asarray(gamma_b, np.float64)
    return float(np.sqrt(np.sum(d * d)))


def sinkhorn_1d(x, y, u, v, eps, tol, itr_max) -> SinkhornResult:
    """Algorithm 1 semantics with dense products, in log form.

    Initialisation phi = 1/n, psi = 1/m. Loop while l < itr_max and the
    marginal error of the current (phi, psi) exceeds tol; each pass updates
    psi from K^T phi, then phi from K psi. The returned pair is the one whose
    error was checked last.
    """
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    u = np.asarray(u, np.float64); v = np.asarray(v, np.float64)
    n, m = len(x), len(y)
    f = np.full(n, eps * np.log(1.0 / n))
    g = np.full(m, eps * np.log(1.0 / m))
    lu, lv = eps * np.log(u), eps * np.log(v)
    it = 0
    while True:
        t = logmatvec(y, x, f, eps)                 # eps ln K^T phi
        err = marginal_error(g, t, v, eps)
        if not (it < itr_max and err > tol):
            break
        g = lv - t                                  # psi = v / K^T phi
        s = logmatvec(x, y, g, eps)                 # eps ln K psi
        f = lu - s                                  # phi = u / K psi
        it += 1
    w1 = transport_cost_1d(x, y, f, g, eps)
    return SinkhornResult(f, g, it, err, w1, err <= tol)


# --------------------------------------------------------------------------
# 2D (column-major grids, element [k, i] <-> index k + i*N)
# --------------------------------------------------------------------------

def logmatvec_2d(xr, yr, xc, yc, G, eps):
    """eps ln (K e^{G/eps}) for K = K_y (x) K_x, axis by axis.

    G is (len(xc), len(yc)); K_x has rows xr / columns xc, K_y rows yr /
    columns yc. The result is (len(xr), len(yr)) = eps ln(K_x E K_y^T).
    """
    G = np.asarray(G, np.float64)
    S = np.empty((len(xr), G.shape[1]))
    for j in range(G.shape[1]):                      # columns: K_x along axis 0
        S[:, j] = logmatvec(xr, xc, G[:, j], eps)
    T = np.empty((len(xr), len(yr)))
    for k in range(len(xr)):                         # rows: K_y along axis 1
        T[k, :] = logmatvec(yr, yc, S[k, :], eps)
    return T


def logmatvec_2d_full(xr, yr, xc, yc, G, eps):
    """The same product through the full (NM)x(NM) kernel (tiny sizes only).

    Entry ((k,i),(l,j)) = exp(-(|xr_k - xc_l| + |yr_i - yc_j|)/eps) (eq. 2d-block-entry).
    """
    XR, YR = np.meshgrid(xr, yr, indexing="ij")
    XC, YC = np.meshgrid(xc, yc, indexing="ij")
    pr_x, pr_y = XR.ravel(order="F"), YR.ravel(order="F")
    pc_x, pc_y = XC.ravel(order="F"), YC.ravel(order="F")
    c = np.abs(pr_x[:, None] - pc_x[None, :]) + np.abs(pr_y[:, None] - pc_y[None, :])
    arg = (np.asarray(G).ravel(order="F")[None, :] - c) / eps
    return (eps * _lse_rows(arg)).reshape((len(xr), len(yr)), order="F")


def transport_cost_2d(x1, y1, x2, y2, F, G, eps) -> float:
    """<C, Gamma> with C = |dx| + |dy|, evaluated axis by axis.

    <C_x, Gamma> = sum_{k,i} phi_ki (M_x Psi K_y^T)_ki and
    <C_y, Gamma> = sum_{k,i} phi_ki (K_x Psi M_y^T)_ki, M = C o K.
    """
    F = np.asarray(F); G = np.asarray(G)
    # x-moment along axis 0, plain along axis 1
    S = np.empty((len(x1), G.shape[1]))
    for j in range(G.shape[1]):
        S[:, j] = log_moment_matvec(x1, x2, G[:, j], eps)
    Tx = np.empty((len(x1), len(y1)))
    for k in range(len(x1)):
        Tx[k, :] = logmatvec(y1, y2, S[k, :], eps)
    # plain along axis 0, y-moment along axis 1
    for j in range(G.shape[1]):
        S[:, j] = logmatvec(x1, x2, G[:, j], eps)
    Ty = np.empty((len(x1), len(y1)))
    for k in range(len(x1)):
        Ty[k, :] = log_moment_matvec(y1, y2, S[k, :], eps)
    return float(np.sum(np.exp((F + Tx) / eps)) + np.sum(np.exp((F + Ty) / eps)))


def transport_cost_2d_full(x1, y1, x2, y2, F, G, eps) -> float:
    XR, YR = np.meshgrid(x1, y1, indexing="ij")
    XC, YC = np.meshgrid(x2, y2, indexing="ij")
    pr_x, pr_y = XR.ravel(order="F"), YR.ravel(order="F")
    pc_x, pc_y = XC.ravel(order="F"), YC.ravel(order="F")
    c = np.abs(pr_x[:, None] - pc_x[None, :]) + np.abs(pr_y[:, None] - pc_y[None, :])
    gam = np.exp((np.asarray(F).ravel(order="F")[:, None]
                  + np.asarray(G).ravel(order="F")[None, :] - c) / eps)
    return float(np.sum(c * gam))


def sinkhorn_2d(x1, y1, x2, y2, u, v, eps, tol, itr_max, full=False) -> SinkhornResult:
    """Algorithm 2 semantics (log form). u is (N1, M1), v is (N2, M2).

    Initialisation Phi = 1/(N1 M1), Psi = 1/(N2 M2). Each pass:
    T = K_x^T Phi K_y (Psi = v / T), then T = K_x Psi K_y^T (Phi = u / T).
    """
    u = np.asarray(u, np.float64); v = np.asarray(v, np.float64)
    mv = logmatvec_2d_full if full else logmatvec_2d
    F = np.full(u.shape, eps * np.log(1.0 / u.size))
    G = np.full(v.shape, eps * np.log(1.0 / v.size))
    lu, lv = eps * np.log(u), eps * np.log(v)
    it = 0
    while True:
        T = mv(x2, y2, x1, y1, F, eps)               # eps ln K^T phi, (N2, M2)
        err = float(np.sum(np.abs(np.exp((G + T) / eps) - v)))
        if not (it < itr_max and err > tol):
            break
        G = lv - T
        S = mv(x1, y1, x2, y2, G, eps)               # eps ln K psi, (N1, M1)
        F = lu - S
        it += 1
    cost = (transport_cost_2d_full if full else transport_cost_2d)(x1, y1, x2, y2, F, G, eps)
    return SinkhornResult(F, G, it, err, cost, err <= tol)


# --------------------------------------------------------------------------
# d dimensions (the remark closing section 3): K = K_{d-1} (x) ... (x) K_0 on
# column-major grids (axis 0 fastest), each product applied axis by axis
# --------------------------------------------------------------------------

def logmatvec_nd(xr, xc, G, eps):
    """eps ln (K e^{G/eps}) with K_a of rows xr[a] and columns xc[a].

    G has shape (len(xc[0]), ..., len(xc[d-1])); the result has shape
    (len(xr[0]), ..., len(xr[d-1])). Axis a is replaced by the 1D product
    along it, one fibre at a time, for a = 0, 1, ..., d-1.
    """
    T = np.asarray(G, np.float64)
    for a in range(len(xr)):
        A = np.moveaxis(T, a, -1)
        out = np.empty(A.shape[:-1] + (len(xr[a]),))
        for idx in np.ndindex(*A.shape[:-1]):
            out[idx] = logmatvec(xr[a], xc[a], A[idx], eps)
        T = np.moveaxis(out, -1, a)
    return T


def _grid_points(axes):
    """Coordinates of every grid point, in column-major order: (N, d)."""
    mesh = np.meshgrid(*[np.asarray(a, np.float64) for a in axes], indexing="ij")
    return np.stack([m.ravel(order="F") for m in mesh], axis=1)


def cost_matrix_nd(xs, xt):
    """C_rc = sum_a |p_r,a - q_c,a| between all source and target grid points."""
    P, Q = _grid_points(xs), _grid_points(xt)
    return np.sum(np.abs(P[:, None, :] - Q[None, :, :]), axis=2)


def logmatvec_nd_full(xr, xc, G, eps):
    """The same product through the full kernel (tiny sizes only)."""
    c = cost_matrix_nd(xr, xc)
    arg = (np.asarray(G, np.float64).ravel(order="F")[None, :] - c) / eps
    return (eps * _lse_rows(arg)).reshape(tuple(len(a) for a in xr), order="F")


def transport_cost_nd(xs, xt, F, G, eps) -> float:
    """<C, Gamma> with C = sum_c |x_c - y_c|: for each axis c, the product
    with the moment kernel C_c o K_c along c and K_a along the other axes,
    summed against phi."""
    F = np.asarray(F, np.float64)
    tot = 0.0
    for c in range(len(xs)):
        T = np.asarray(G, np.float64)
        for a in range(len(xs)):
            A = np.moveaxis(T, a, -1)
            out = np.empty(A.shape[:-1] + (len(xs[a]),))
            mv = log_moment_matvec if a == c else logmatvec
            for idx in np.ndindex(*A.shape[:-1]):
                out[idx] = mv(xs[a], xt[a], A[idx], eps)
            T = np.moveaxis(out, -1, a)
        tot += float(np.sum(np.exp((F + T) / eps)))
    return tot


def transport_cost_nd_full(xs, xt, F, G, eps) -> float:
    c = cost_matrix_nd(xs, xt)
    f = np.asarray(F, np.float64).ravel(order="F")
    g = np.asarray(G, np.float64).ravel(order="F")
    return float(np.sum(c * np.exp((f[:, None] + g[None, :] - c) / eps)))


def sinkhorn_nd(xs, xt, u, v, eps, tol, itr_max, full=False) -> SinkhornResult:
    """The loop of Algorithms 1 and 2 on d-dimensional tensor meshes (log
    form). u has shape (len(xs[0]), ...), v shape (len(xt[0]), ...).
    Initialisation Phi = 1/|u|, Psi = 1/|v|; each pass updates Psi from
    K^T Phi, then Phi from K Psi; the loop head checks the v marginal."""
    u = np.asarray(u, np.float64); v = np.asarray(v, np.float64)
    mv = logmatvec_nd_full if full else logmatvec_nd
    F = np.full(u.shape, eps * np.log(1.0 / u.size))
    G = np.full(v.shape, eps * np.log(1.0 / v.size))
    lu, lv = eps * np.log(u), eps * np.log(v)
    it = 0
    while True:
        T = mv(xt, xs, F, eps)                       # eps ln K^T phi, target grid
        err = float(np.sum(np.abs(np.exp((G + T) / eps) - v)))
        if not (it < itr_max and err > tol):
            break
        G = lv - T
        S = mv(xs, xt, G, eps)                       # eps ln K psi, source grid
        F = lu - S
        it += 1
    cost = (transport_cost_nd_full if full else transport_cost_nd)(xs, xt, F, G, eps)
    return SinkhornResult(F, G, it, err, cost, err <= tol)
