/*
 * finom.h - C ABI of the MI355X (gfx950) FINOM library.
 *
 * Entropic Wasserstein-1 with L1 cost on non-uniform 1D meshes and 2D
 * tensor-product meshes, solved by Sinkhorn iterations whose kernel-vector
 * products K psi and K^T phi use the dividing-index split of
 * K = exp(-C/eps) into two quasi-collinear blocks and their O(N)
 * recurrences (section 2, eq. decompose to p+q, eq. p-DP, eq. q-DP;
 * section 3, eq. 2d-kron, Algorithms 1 and 2).
 *
 * Conventions for every entry point
 *  - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *    owned by the caller, float64, contiguous. The library never frees them.
 *  - Meshes must be non-decreasing (ties allowed); the library does not sort,
 *    because sorting would permute the caller's masses.
 *  - Every coordinate must satisfy |c| / (eps ln 2) < 2^25: the products are
 *    formed from 2^(+-c/(eps ln 2)) with a 32-bit binary exponent. Checked on
 *    the end points of each mesh (FINOM_E_ARG) unless skip_checks is set.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is enqueued on that stream. Entry points that return host results
 *    (finom_result, device-side validation) synchronise that stream.
 *  - Internal workspace is cached per stream and released by finom_release().
 *    Calls on the same stream from different host threads must be serialised
 *    by the caller; distinct streams are independent.
 *  - Return value: FINOM_OK (0), a positive warning (results written) or a
 *    negative error (nothing written). No exception crosses the ABI.
 *  - Potentials are returned in natural-log units: f = eps ln phi and
 *    g = eps ln psi, so Gamma_ij = exp((f_i + g_j - C_ij)/eps).
 */
#ifndef FINOM_H
#define FINOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FINOM_OK = 0,
    FINOM_NOT_CONVERGED = 1,   /* iteration cap reached before err <= tol; results valid */
    FINOM_E_ARG = -1,          /* bad argument (null pointer, size < 1, eps <= 0, ...)   */
    FINOM_E_UNSORTED = -2,     /* a mesh is decreasing somewhere or holds a NaN         */
    FINOM_E_MASS = -3,         /* a mass is <= 0 / non-finite, or sum(u) != sum(v)      */
    FINOM_E_NOMEM = -4,        /* device or pinned allocation failed                    */
    FINOM_E_HIP = -5,          /* a HIP runtime call failed                              */
    FINOM_E_ADMIT = -6,        /* serving: request larger than the HBM budget           */
    FINOM_E_NUMERIC = -7       /* non-finite marginal error during the iteration        */
} finom_status;

/* Options. A NULL pointer means all defaults (zero-initialised struct). */
typedef struct {
    int32_t precision;  /* 0 = FP64 scans; 1 = FP32-mantissa scans. State, convergence
                           check and cost are FP64 in both modes.                        */
    int32_t domain;     /* matvec entry points only: 0 = linear (out = K in, in >= 0);
                           1 = log (in = eps ln psi, out = eps ln K psi).               */
    int32_t skip_checks;/* 1 = trust the inputs: no device-side sortedness / mass checks
                           (and no stream synchronisation for them).                    */
    int32_t graph_iters;/* solver: iterations per captured HIP graph launch; 0 = default.*/
} finom_opts;

typedef struct {
    double w1;            /* <C, Gamma> of the returned pair, FP64                       */
    double marginal_err;  /* ||diag(psi) K^T phi - v||_1 of the returned pair (loop-head
                             check of Algorithm 1), FP64                                 */
    int64_t iters;        /* completed iterations l                                      */
    int32_t converged;    /* marginal_err <= tol                                         */
    int32_t status;       /* the value the call returned                                 */
    double loop_ms;       /* GPU time of the iteration loop (HIP events on `stream`),
                             excluding setup and the final cost reduction             */
    int64_t sweeps;       /* half-iteration products executed in the loop: 2 l + 1     */
} finom_result;

/*
 * K * in for the 1D kernel K_ij = exp(-|x_rows_i - y_cols_j| / eps)
 * (section 2.1) through the dividing-index split and the two recurrences
 * (eq. decompose to p+q, eq. p-DP, eq. q-DP).
 *   x_rows: n row coordinates; y_cols: m column coordinates (both ascending).
 *   in: m values (domain 0: psi >= 0; domain 1: eps ln psi, -inf allowed).
 *   out: n values (domain 0: K psi; domain 1: eps ln K psi).
 * K^T * u is the same call with (y_cols, m) as rows and (x_rows, n) as
 * columns. Errors: FINOM_E_ARG, FINOM_E_UNSORTED, FINOM_E_NOMEM, FINOM_E_HIP.
 */
int finom_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m,
                 double eps, const double* in, double* out, const finom_opts* opts,
                 void* stream);

/*
 * The same product evaluated densely, O(n*m) kernel entries generated on the
 * fly ("standard Sinkhorn" product of section 4). Baseline; identical
 * signature and semantics to finom_matvec.
 */
int dense_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m,
                 double eps, const double* in, double* out, const finom_opts* opts,
                 void* stream);

/*
 * Algorithm 1 (1D FINOM Sinkhorn) on meshes x (n) and y (m), masses u (n) and
 * v (m), all > 0 with sum(u) == sum(v) within 1e-12 relative.
 * Initialisation phi = 1/n, psi = 1/m. Loop while l < itr_max and
 * ||diag(psi) K^T phi - v||_1 > tol: psi = v / K^T phi, phi = u / K psi.
 * f_out (n) / g_out (m): device outputs eps ln phi / eps ln psi of the
 * returned pair (the one whose error was checked last); either may be NULL.
 * res (HOST pointer, required) receives w1 = <C, Gamma>, the error, l.
 * Returns FINOM_OK, FINOM_NOT_CONVERGED, or an error
 * (FINOM_E_ARG / _UNSORTED / _MASS / _NOMEM / _HIP / _NUMERIC).
 */
int sinkhorn_w1_1d(const double* x, int64_t n, const double* y, int64_t m,
                   const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream);

/*
 * Algorithm 2 (2D FINOM Sinkhorn) on tensor-product meshes: source grid
 * x1 (n1) x y1 (m1), target grid x2 (n2) x y2 (m2), cost |dx| + |dy|, so
 * K = K_y (x) K_x (eq. 2d-kron). u (n1*m1) and v (n2*m2) are column-major:
 * element (k, i) at k + i*n1 (the paper's grid order, section 3.1). Each
 * product is evaluated axis by axis, K^T phi = vec(K_x^T Phi K_y) and
 * K psi = vec(K_x Psi K_y^T) (eq. 2d-ktphi, eq. 2d-kpsi), with the potentials
 * absorbed as in the appendix (columns with the right absorption, rows with
 * the left one). Initialisation Phi = 1/(n1 m1), Psi = 1/(n2 m2); the loop,
 * the check and the outputs (f_out: n1*m1, g_out: n2*m2, column-major) are as
 * in sinkhorn_w1_1d. w1 = <|dx| + |dy|, Gamma> in FP64.
 */
int sinkhorn_w1_2d(const double* x1, int64_t n1, const double* y1, int64_t m1,
                   const double* x2, int64_t n2, const double* y2, int64_t m2,
                   const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream);

/* Human-readable text for a status code (static storage). */
const char* finom_strerror(int status);

/* Frees all cached device/pinned workspace (all streams). Not concurrent-safe
 * with running calls. */
void finom_release(void);

/* Library version string, e.g. "finom-gfx950 0.1". */
const char* finom_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FINOM_H */
