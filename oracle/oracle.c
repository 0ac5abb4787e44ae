/*
 * FP64 CPU oracle in plain C (TEST INFRASTRUCTURE: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this).
 *
 * Arrays are 0-based here; the paper is 1-based. Meshes are ascending.
 *
 * Parts:
 *   1. Dividing index (Definition in section 2.2): zeta[i] = #{j : y_j <= x_i}.
 *   2. Vector representation of K_L and K_U (Theorems 2.1 and 2.2), built
 *      from the matrix entries themselves with the footnote conventions
 *      (r_i := 1 when the denominator entry is 0), and the linear-domain
 *      product of eq. (decompose to p+q) with eq. (p-DP) / eq. (q-DP),
 *      instrumented with multiplication and addition counters (section 2.3).
 *   3. The same recurrences in log form: the stabilisation remark of
 *      section 2.3 with absorption at every step. p and q are carried as
 *      logarithms; r_i becomes a subtraction of (x_{i+1} - x_i)/eps and the
 *      block-edge dot products become log-sum-exp over the segment.
 *   4. Algorithm 1 (1D) and Algorithm 2 with the appendix's decoupled sweeps
 *      (2D), in log form, built on part 3.
 *   5. Dense definitions: eps*ln(K e^{g/eps}) and <C, Gamma> by direct sums.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ 1 -- */

void orc_dividing_index(const double* x, long n, const double* y, long m, long* zeta)
{
    long j = 0;
    for (long i = 0; i < n; ++i) {
        while (j < m && y[j] <= x[i]) ++j;
        zeta[i] = j;
    }
}

/* ------------------------------------------------------------------ 2 -- */

/* Entries of K_L (check k) and K_U (hat k), 0-based row i, column j. */
static double kl_entry(const double* x, const double* y, const long* zeta,
                       long i, long j, double eps)
{
    return (j < zeta[i]) ? exp(-(x[i] - y[j]) / eps) : 0.0;
}

static double ku_entry(const double* x, const double* y, const long* zeta,
                       long i, long j, double eps)
{
    return (j >= zeta[i]) ? exp(-(y[j] - x[i]) / eps) : 0.0;
}

/*
 * Builds r (n-1), eta (zeta[n-1] entries, offsets eta_off[n+1]),
 * rp (n-1), etap (m - zeta[0] entries, offsets etap_off[n+1]).
 * eta_i holds row i, columns zeta(i-1)..zeta(i)-1 (zeta(-1) := 0);
 * etap_i holds row i, columns zeta(i)..zeta(i+1)-1 (zeta(n) := m).
 */
void orc_vector_rep(const double* x, long n, const double* y, long m, double eps,
                    long* zeta, double* r, long* eta_off, double* eta,
                    double* rp, long* etap_off, double* etap)
{
    orc_dividing_index(x, n, y, m, zeta);
    for (long i = 0; i + 1 < n; ++i) {
        double den = kl_entry(x, y, zeta, i, 0, eps);
        r[i] = (den == 0.0) ? 1.0 : kl_entry(x, y, zeta, i + 1, 0, eps) / den;
        double denp = ku_entry(x, y, zeta, i + 1, m - 1, eps);
        rp[i] = (denp == 0.0) ? 1.0 : ku_entry(x, y, zeta, i, m - 1, eps) / denp;
    }
    long k = 0;
    eta_off[0] = 0;
    for (long i = 0; i < n; ++i) {
        long lo = (i == 0) ? 0 : zeta[i - 1];
        for (long j = lo; j < zeta[i]; ++j) eta[k++] = kl_entry(x, y, zeta, i, j, eps);
        eta_off[i + 1] = k;
    }
    k = 0;
    etap_off[0] = 0;
    for (long i = 0; i < n; ++i) {
        long hi = (i + 1 < n) ? zeta[i + 1] : m;
        for (long j = zeta[i]; j < hi; ++j) etap[k++] = ku_entry(x, y, zeta, i, j, eps);
        etap_off[i + 1] = k;
    }
}

/*
 * K psi = p + q from the stored representation, counting operations.
 * A running value that is still the empty sum is assigned, not added to, and
 * is not multiplied by r; in the generic case (zeta(1) >= 1, zeta(N) < M) the
 * counts are exactly those of section 2.3.
 */
void orc_rep_matvec(long n, long m, const long* zeta, const double* r,
                    const long* eta_off, const double* eta, const double* rp,
                    const long* etap_off, const double* etap, const double* psi,
                    double* out, long* n_mul, long* n_add)
{
    long mul = 0, add = 0;
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    /* forward, eq. (p-DP) */
    int have = 0;
    double acc = 0.0;
    for (long i = 0; i < n; ++i) {
        if (have && i > 0) { acc = r[i - 1] * acc; ++mul; }
        long lo = (i == 0) ? 0 : zeta[i - 1];
        for (long j = lo; j < zeta[i]; ++j) {
            double t = eta[eta_off[i] + (j - lo)] * psi[j]; ++mul;
            if (have) { acc += t; ++add; } else { acc = t; have = 1; }
        }
        p[i] = have ? acc : 0.0;
    }
    /* backward, eq. (q-DP) */
    have = 0;
    acc = 0.0;
    for (long i = n - 1; i >= 0; --i) {
        if (have && i < n - 1) { acc = rp[i] * acc; ++mul; }
        long hi = (i + 1 < n) ? zeta[i + 1] : m;
        for (long j = zeta[i]; j < hi; ++j) {
            double t = etap[etap_off[i] + (j - zeta[i])] * psi[j]; ++mul;
            if (have) { acc += t; ++add; } else { acc = t; have = 1; }
        }
        q[i] = have ? acc : 0.0;
    }
    for (long i = 0; i < n; ++i) { out[i] = p[i] + q[i]; ++add; }
    free(p); free(q);
    *n_mul = mul; *n_add = add;
}

/* ------------------------------------------------------------------ 3 -- */

static double lse2(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    return (a > b) ? a + log1p(exp(b - a)) : b + log1p(exp(a - b));
}

/*
 * out_i = eps * ln( sum_j exp((g_j - |xr_i - yc_j|)/eps) ), through the two
 * recurrences in log form. g is read with stride gstride, out written with
 * stride ostride (a line of a 2D array). plogs/qlogs: scratch of length R.
 */
static void finom_logmatvec_line(const double* xr, long R, const double* yc, long C,
                                 const double* g, long gstride, double eps,
                                 double* out, long ostride, double* P, double* Q,
                                 long* zeta)
{
    orc_dividing_index(xr, R, yc, C, zeta);
    /* p: rows in increasing order; row i's new block edge = columns
       zeta(i-1)..zeta(i)-1, each weighted by exp(-(x_i - y_j)/eps). */
    double acc = -INFINITY;
    for (long i = 0; i < R; ++i) {
        if (i > 0) acc -= (xr[i] - xr[i - 1]) / eps;          /* r_{i-1} */
        long lo = (i == 0) ? 0 : zeta[i - 1];
        for (long j = lo; j < zeta[i]; ++j)
            acc = lse2(acc, (g[j * gstride] - (xr[i] - yc[j])) / eps);
        P[i] = acc;
    }
    /* q: rows in decreasing order; row i's block edge = columns
       zeta(i)..zeta(i+1)-1, weighted by exp(-(y_j - x_i)/eps). */
    acc = -INFINITY;
    for (long i = R - 1; i >= 0; --i) {
        if (i < R - 1) acc -= (xr[i + 1] - xr[i]) / eps;      /* r'_i */
        long hi = (i + 1 < R) ? zeta[i + 1] : C;
        for (long j = zeta[i]; j < hi; ++j)
            acc = lse2(acc, (g[j * gstride] - (yc[j] - xr[i])) / eps);
        Q[i] = acc;
    }
    for (long i = 0; i < R; ++i) out[i * ostride] = eps * lse2(P[i], Q[i]);
}

void orc_finom_logmatvec(const double* xr, long R, const double* yc, long C,
                         const double* g, double eps, double* out)
{
    double* P = (double*)malloc(sizeof(double) * R);
    double* Q = (double*)malloc(sizeof(double) * R);
    long* z = (long*)malloc(sizeof(long) * R);
    finom_logmatvec_line(xr, R, yc, C, g, 1, eps, out, 1, P, Q, z);
    free(P); free(Q); free(z);
}

/* ------------------------------------------------------------------ 4 -- */

static double marginal_err(const double* gg, const double* t, const double* v,
                           long m, double eps)
{
    double s = 0.0;
    for (long j = 0; j < m; ++j) s += fabs(exp((gg[j] + t[j]) / eps) - v[j]);
    return s;
}

/*
 * Algorithm 1. f = eps ln phi (n), g = eps ln psi (m) are outputs; returns the
 * number of completed iterations and writes the last checked marginal error.
 * err_trace (nullable, length itr_max + 1) receives the error of every check.
 */
long orc_sinkhorn_1d(const double* x, long n, const double* y, long m,
                     const double* u, const double* v, double eps, double tol,
                     long itr_max, double* f, double* g, double* err_out,
                     double* err_trace)
{
    long big = (n > m) ? n : m;
    double* t = (double*)malloc(sizeof(double) * big);
    double* P = (double*)malloc(sizeof(double) * big);
    double* Q = (double*)malloc(sizeof(double) * big);
    long* z = (long*)malloc(sizeof(long) * big);
    for (long i = 0; i < n; ++i) f[i] = eps * log(1.0 / (double)n);
    for (long j = 0; j < m; ++j) g[j] = eps * log(1.0 / (double)m);
    long it = 0;
    double err;
    for (;;) {
        finom_logmatvec_line(y, m, x, n, f, 1, eps, t, 1, P, Q, z);   /* K^T phi */
        err = marginal_err(g, t, v, m, eps);
        if (err_trace) err_trace[it] = err;
        if (!(it < itr_max && err > tol)) break;
        for (long j = 0; j < m; ++j) g[j] = eps * log(v[j]) - t[j];
        finom_logmatvec_line(x, n, y, m, g, 1, eps, t, 1, P, Q, z);   /* K psi */
        for (long i = 0; i < n; ++i) f[i] = eps * log(u[i]) - t[i];
        ++it;
    }
    *err_out = err;
    free(t); free(P); free(Q); free(z);
    return it;
}

/*
 * eps ln of K e^{G/eps} on a column-major grid, K = K_y (x) K_x: first every
 * column along the first axis (rows xr, columns xc), then every row along the
 * second axis (rows yr, columns yc). G is nxc x nyc; S is nxr x nyc scratch;
 * T (output) is nxr x nyr.
 */
static void logmatvec_2d(const double* xr, long nxr, const double* yr, long nyr,
                         const double* xc, long nxc, const double* yc, long nyc,
                         const double* G, double eps, double* S, double* T,
                         int threads)
{
    long big = nxr + nyr + nxc + nyc;
#pragma omp parallel num_threads(threads)
    {
        double* P = (double*)malloc(sizeof(double) * big);
        double* Q = (double*)malloc(sizeof(double) * big);
        long* z = (long*)malloc(sizeof(long) * big);
#pragma omp for schedule(static)
        for (long j = 0; j < nyc; ++j)
            finom_logmatvec_line(xr, nxr, xc, nxc, G + j * nxc, 1, eps,
                                 S + j * nxr, 1, P, Q, z);
#pragma omp for schedule(static)
        for (long k = 0; k < nxr; ++k)
            finom_logmatvec_line(yr, nyr, yc, nyc, S + k, nxr, eps,
                                 T + k, nxr, P, Q, z);
        free(P); free(Q); free(z);
    }
}

/* Algorithm 2 with the decoupled stabilised sweeps of the appendix. */
long orc_sinkhorn_2d(const double* x1, long n1, const double* y1, long m1,
                     const double* x2, long n2, const double* y2, long m2,
                     const double* u, const double* v, double eps, double tol,
                     long itr_max, double* F, double* G, double* err_out,
                     double* err_trace, int threads)
{
    long a = n1 * m1, b = n2 * m2;
    long big = (a > b) ? a : b;
    long sbig = (n1 * m2 > n2 * m1) ? n1 * m2 : n2 * m1;
    double* S = (double*)malloc(sizeof(double) * sbig);
    double* T = (double*)malloc(sizeof(double) * big);
    for (long k = 0; k < a; ++k) F[k] = eps * log(1.0 / (double)a);
    for (long k = 0; k < b; ++k) G[k] = eps * log(1.0 / (double)b);
    long it = 0;
    double err;
    for (;;) {
        logmatvec_2d(x2, n2, y2, m2, x1, n1, y1, m1, F, eps, S, T, threads);
        err = marginal_err(G, T, v, b, eps);
        if (err_trace) err_trace[it] = err;
        if (!(it < itr_max && err > tol)) break;
        for (long k = 0; k < b; ++k) G[k] = eps * log(v[k]) - T[k];
        logmatvec_2d(x1, n1, y1, m1, x2, n2, y2, m2, G, eps, S, T, threads);
        for (long k = 0; k < a; ++k) F[k] = eps * log(u[k]) - T[k];
        ++it;
    }
    *err_out = err;
    free(S); free(T);
    return it;
}

void orc_finom_logmatvec_2d(const double* xr, long nxr, const double* yr, long nyr,
                            const double* xc, long nxc, const double* yc, long nyc,
                            const double* G, double eps, double* T, int threads)
{
    double* S = (double*)malloc(sizeof(double) * nxr * nyc);
    logmatvec_2d(xr, nxr, yr, nyr, xc, nxc, yc, nyc, G, eps, S, T, threads);
    free(S);
}

/* ------------------------------------------------------------------ 5 -- */

/* Dense definition for the listed rows (rows == NULL: all R rows). */
void orc_dense_logmatvec(const double* xr, long R, const double* yc, long C,
                         const double* g, double eps, double* out,
                         const long* rows, long nrows, int threads)
{
    long cnt = rows ? nrows : R;
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
    for (long k = 0; k < cnt; ++k) {
        long i = rows ? rows[k] : k;
        double mx = -INFINITY;
        for (long j = 0; j < C; ++j) {
            double a = (g[j] - fabs(xr[i] - yc[j])) / eps;
            if (a > mx) mx = a;
        }
        double s = 0.0;
        for (long j = 0; j < C; ++j) s += exp((g[j] - fabs(xr[i] - yc[j])) / eps - mx);
        out[k] = eps * (mx + log(s));
    }
}

/* <C, Gamma> = sum_ij |x_i - y_j| exp((f_i + g_j - |x_i - y_j|)/eps). */
double orc_dense_cost_1d(const double* x, long n, const double* y, long m,
                         const double* f, const double* g, double eps, int threads)
{
    double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(dynamic, 16) num_threads(threads)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (long j = 0; j < m; ++j) {
            double c = fabs(x[i] - y[j]);
            s += c * exp((f[i] + g[j] - c) / eps);
        }
        tot += s;
    }
    return tot;
}

/* Dense Algorithm 1 loop (the definition, for sizes NumPy is slow at). */
long orc_dense_sinkhorn_1d(const double* x, long n, const double* y, long m,
                           const double* u, const double* v, double eps, double tol,
                           long itr_max, double* f, double* g, double* err_out,
                           int threads)
{
    long big = (n > m) ? n : m;
    double* t = (double*)malloc(sizeof(double) * big);
    for (long i = 0; i < n; ++i) f[i] = eps * log(1.0 / (double)n);
    for (long j = 0; j < m; ++j) g[j] = eps * log(1.0 / (double)m);
    long it = 0;
    double err;
    for (;;) {
        orc_dense_logmatvec(y, m, x, n, f, eps, t, NULL, 0, threads);
        err = marginal_err(g, t, v, m, eps);
        if (!(it < itr_max && err > tol)) break;
        for (long j = 0; j < m; ++j) g[j] = eps * log(v[j]) - t[j];
        orc_dense_logmatvec(x, n, y, m, g, eps, t, NULL, 0, threads);
        for (long i = 0; i < n; ++i) f[i] = eps * log(u[i]) - t[i];
        ++it;
    }
    *err_out = err;
    free(t);
    return it;
}
