// Dense baselines of the 2D product (section 4's standard Sinkhorn on tensor
// meshes): eps ln (K e^{G/eps}) with K = K_y (x) K_x (eq. 2d-kron).
//
// Per axis (full = 0): K e^{G/eps} = K_x E K_y^T for the column-major grid E,
// two dense matrix products with every kernel entry exp(-|a - b|/eps)
// generated as its tile is loaded, never stored. They run on the matrix cores
// in FP64 (v_mfma_f64_16x16x4f64). Each product works on shifted linear
// values: the columns of E are divided by their largest entry (c_j) before
// the first product and the rows of the intermediate by theirs (d_k) before
// the second, so every operand lies in (0, 1] and the products stay inside
// FP64 where eps is not too small for the mesh (the smallest kernel entry,
// exp(-diam/eps), must not underflow); the logs add the shifts back.
//
// Full (full = 1): every output sums over every input grid point with its
// own exponential exp((G_lj - |x_k - x2_l| - |y_i - y2_j|)/eps), as the
// standard iteration with the (NM) x (NM) kernel does; a running maximum per
// output keeps the sum in range. This is a matrix-vector product (one input
// vector), so it runs on the vector units, bound by the exponentials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "../../include/finom.h"
#include "finom_host.hpp"

namespace finom {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = A B: A is M x K, B is K x N, both generated or read column-major.
struct GemmArgs {
    const double* A;    // !GA: A[r + c lda]
    long long lda;
    const double* ar;   // GA: A[r][c] = exp(-|ar[r] - ac[c]| inv_eps)
    const double* ac;
    const double* B;    // !GB: B[k + n ldb]
    long long ldb;
    const double* bk;   // GB: B[k][n] = exp(-|bk[k] - bn[n]| inv_eps)
    const double* bn;
    long long M, N, K;
    double inv_eps, eps;
    const double* shift;   // per column (SHIFT_COL) or per row of C
    double* out;           // out[r + c ldo] = shift + eps ln C[r][c]
    long long ldo;
};

constexpr int kGemmBlock = 256;   // four waves, 2 x 2, each one 16 x 16 block of C
constexpr int kGemmTile = 32;     // C tile per block (at 1024 x 1024, four blocks per CU)
constexpr int kGemmK = 32;        // K per LDS stage (eight MFMA steps)

template <bool GA, bool GB, bool SHIFT_COL>
__global__ __launch_bounds__(kGemmBlock) void k_dense2d_gemm(GemmArgs g)
{
    __shared__ double As[kGemmK][kGemmTile + 1];
    __shared__ double Bs[kGemmK][kGemmTile + 1];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const long long m0 = (long long)blockIdx.x * kGemmTile, n0 = (long long)blockIdx.y * kGemmTile;
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};

    for (long long k0 = 0; k0 < g.K; k0 += kGemmK) {
        // A tile: 32 rows x 32 k; element e = t + 256 q: row e % 32, k e / 32
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + kGemmBlock * q;
            const int r = e & 31, k = e >> 5;
            const long long gr = m0 + r, gk = k0 + k;
            double v = 0.0;
            if (gr < g.M && gk < g.K) {
                if (GA) v = exp(-fabs(g.ar[gr] - g.ac[gk]) * g.inv_eps);
                else v = g.A[gr + gk * g.lda];
            }
            As[k][r] = v;
        }
        // B tile: 32 k x 32 columns; element e: k e % 32, column e / 32
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + kGemmBlock * q;
            const int k = e & 31, c = e >> 5;
            const long long gk = k0 + k, gc = n0 + c;
            double v = 0.0;
            if (gk < g.K && gc < g.N) {
                if (GB) v = exp(-fabs(g.bk[gk] - g.bn[gc]) * g.inv_eps);
                else v = g.B[gk + gc * g.ldb];
            }
            Bs[k][c] = v;
        }
        __syncthreads();
        // MFMA 16x16x4: lane l takes A[l % 16][l / 16] and B[l / 16][l % 16]
#pragma unroll
        for (int kk = 0; kk < kGemmK; kk += 4) {
            const int kr = kk + (lane >> 4);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[kr][wr + (lane & 15)], Bs[kr][wc + (lane & 15)], acc, 0, 0,
                                                       0);
        }
        __syncthreads();
    }
    // lane l, register v holds C[(l / 16) + 4 v][l % 16] of the wave's 16 x 16 block
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long r = m0 + wr + (lane >> 4) + 4 * v;
        const long long c = n0 + wc + (lane & 15);
        if (r < g.M && c < g.N) g.out[r + c * g.ldo] = (SHIFT_COL ? g.shift[c] : g.shift[r]) + g.eps * log(acc[v]);
    }
}

// Column j of the rows x cols column-major grid G: c_j = max, E = exp((G - c_j)/eps).
__global__ __launch_bounds__(kBlock) void k_dense2d_col_shift(const double* __restrict__ G, long long rows,
                                                             long long cols, double inv_eps, double* __restrict__ E,
                                                             double* __restrict__ c)
{
    __shared__ double s_red[kBlock / kWave];
    const long long j = blockIdx.x;
    double mx = -__builtin_inf();
    for (long long l = threadIdx.x; l < rows; l += kBlock) mx = fmax(mx, G[l + j * rows]);
    // block maximum: within each wave, then across the waves in LDS
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) mx = fmax(mx, __shfl_down(mx, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = mx;
    __syncthreads();
    double m = s_red[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, s_red[w]);
    if (threadIdx.x == 0) c[j] = m;
    for (long long l = threadIdx.x; l < rows; l += kBlock) E[l + j * rows] = exp((G[l + j * rows] - m) * inv_eps);
}

// Row maxima of the rows x cols column-major grid S: a block takes 64 rows,
// its four waves a quarter of the columns each (a wave reads 64 consecutive
// rows of one column at a time), combined in LDS.
__global__ __launch_bounds__(kBlock) void k_dense2d_row_max(const double* __restrict__ S, long long rows,
                                                           long long cols, double* __restrict__ d)
{
    __shared__ double s_m[kBlock];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const long long k = (long long)blockIdx.x * kWave + lane;
    double mx = -__builtin_inf();
    if (k < rows)
        for (long long j = w; j < cols; j += kBlock / kWave) mx = fmax(mx, S[k + j * rows]);
    s_m[threadIdx.x] = mx;
    __syncthreads();
    if (w == 0 && k < rows) {
        double m = s_m[lane];
#pragma unroll
        for (int q = 1; q < kBlock / kWave; ++q) m = fmax(m, s_m[lane + q * kWave]);
        d[k] = m;
    }
}

// E = exp((S - d_k)/eps) over the whole grid.
__global__ __launch_bounds__(kBlock) void k_dense2d_row_exp(const double* __restrict__ S, long long rows,
                                                           long long n, const double* __restrict__ d, double inv_eps,
                                                           double* __restrict__ E)
{
    const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (e < n) E[e] = exp((S[e] - d[e % rows]) * inv_eps);
}

// The full product: output (k, i) = eps ln sum_{l, j} exp((G[l + j n2] -
// |x1_k - x2_l| - |y1_i - y2_j|)/eps), one thread per output, inputs staged
// through LDS in chunks, the sum kept against a running maximum.
constexpr int kFullChunk = 1024;

__global__ __launch_bounds__(kBlock) void k_dense2d_full(const double* __restrict__ x1, long long n1,
                                                        const double* __restrict__ y1, long long m1,
                                                        const double* __restrict__ x2, long long n2,
                                                        const double* __restrict__ y2, long long m2,
                                                        const double* __restrict__ G, double inv_eps, double eps,
                                                        double* __restrict__ out)
{
    __shared__ double s_g[kFullChunk], s_x[kFullChunk], s_y[kFullChunk];
    const long long o = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nout = n1 * m1;
    const bool live = o < nout;
    const long long k = live ? o % n1 : 0, i = live ? o / n1 : 0;
    const double xk = x1[k], yi = y1[i];
    double mx = -__builtin_inf(), s = 0.0;
    const long long nin = n2 * m2;
    for (long long c0 = 0; c0 < nin; c0 += kFullChunk) {
        const int cnt = (int)min((long long)kFullChunk, nin - c0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kBlock) {
            const long long e = c0 + q;
            s_g[q] = G[e];
            s_x[q] = x2[e % n2];
            s_y[q] = y2[e / n2];
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double tq = (s_g[q] - fabs(xk - s_x[q]) - fabs(yi - s_y[q])) * inv_eps;
            if (tq > mx) {
                s = s * exp(mx - tq) + 1.0;
                mx = tq;
            } else {
                s += exp(tq - mx);
            }
        }
    }
    if (live) out[o] = eps * (mx + log(s));
}

}  // namespace finom

using namespace finom;

extern "C" int dense_matvec_2d(const double* x1, int64_t n1, const double* y1, int64_t m1, const double* x2,
                               int64_t n2, const double* y2, int64_t m2, double eps, const double* in, double* out,
                               int32_t full, void* stream)
{
    if (!x1 || !y1 || !x2 || !y2 || !in || !out || n1 < 1 || m1 < 1 || n2 < 1 || m2 < 1) return FINOM_E_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps) || (full != 0 && full != 1)) return FINOM_E_ARG;
    if (n1 > (1LL << 30) || m1 > (1LL << 30) || n2 > (1LL << 30) || m2 > (1LL << 30)) return FINOM_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const double inv_eps = 1.0 / eps;
    try {
        if (full) {
            const long long nout = (long long)n1 * m1;
            hipLaunchKernelGGL(k_dense2d_full, dim3(blocks_for(nout)), dim3(kBlock), 0, s, x1, (long long)n1, y1,
                               (long long)m1, x2, (long long)n2, y2, (long long)m2, in, inv_eps, eps, out);
            HIPCHK(hipGetLastError());
            return FINOM_OK;
        }
        Alloc al(stream);
        double* E = al.dev<double>((size_t)n2 * m2);   // shifted e^{G/eps}, n2 x m2
        double* c = al.dev<double>(m2);
        double* S = al.dev<double>((size_t)n1 * m2);   // eps ln (K_x E) + c, n1 x m2
        double* F = al.dev<double>((size_t)n1 * m2);   // shifted e^{S/eps}
        double* d = al.dev<double>(n1);
        al.uploaded();
        hipLaunchKernelGGL(k_dense2d_col_shift, dim3((unsigned)m2), dim3(kBlock), 0, s, in, (long long)n2,
                           (long long)m2, inv_eps, E, c);
        GemmArgs g1;
        memset(&g1, 0, sizeof(g1));
        g1.ar = x1; g1.ac = x2;                 // K_x: rows x1, columns x2
        g1.B = E; g1.ldb = n2;
        g1.M = n1; g1.N = m2; g1.K = n2;
        g1.inv_eps = inv_eps; g1.eps = eps;
        g1.shift = c; g1.out = S; g1.ldo = n1;
        hipLaunchKernelGGL((k_dense2d_gemm<true, false, true>),
                           dim3((unsigned)((n1 + kGemmTile - 1) / kGemmTile), (unsigned)((m2 + kGemmTile - 1) / kGemmTile)),
                           dim3(kGemmBlock), 0, s, g1);
        hipLaunchKernelGGL(k_dense2d_row_max, dim3((unsigned)((n1 + kWave - 1) / kWave)), dim3(kBlock), 0, s, S,
                           (long long)n1, (long long)m2, d);
        hipLaunchKernelGGL(k_dense2d_row_exp, dim3(blocks_for((long long)n1 * m2)), dim3(kBlock), 0, s, S,
                           (long long)n1, (long long)n1 * m2, d, inv_eps, F);
        GemmArgs g2;
        memset(&g2, 0, sizeof(g2));
        g2.A = F; g2.lda = n1;
        g2.bk = y2; g2.bn = y1;                 // K_y^T: B[j][i] = exp(-|y2_j - y1_i|/eps)
        g2.M = n1; g2.N = m1; g2.K = m2;
        g2.inv_eps = inv_eps; g2.eps = eps;
        g2.shift = d; g2.out = out; g2.ldo = n1;
        hipLaunchKernelGGL((k_dense2d_gemm<false, true, false>),
                           dim3((unsigned)((n1 + kGemmTile - 1) / kGemmTile), (unsigned)((m1 + kGemmTile - 1) / kGemmTile)),
                           dim3(kGemmBlock), 0, s, g2);
        HIPCHK(hipGetLastError());
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}
