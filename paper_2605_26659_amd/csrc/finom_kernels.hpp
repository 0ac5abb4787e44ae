// FINOM sweep kernels for gfx950.
//
// A "line" is one 1D product K psi between row mesh xr and column mesh yc
// (K^T phi is the same product with the meshes swapped). With the dividing
// index zeta(i) = #{j : y_j <= x_i} (section 2.2) the product splits into
//   p_i = sum_{j < zeta(i)} e^{-(x_i - y_j)/eps} psi_j     (lower block K_L)
//   q_i = sum_{j >= zeta(i)} e^{-(y_j - x_i)/eps} psi_j    (upper block K_U)
// (eq. decompose to p+q). The recurrences p_{i+1} = r_i p_i + eta_{i+1}.psi
// and q_i = r'_i q_{i+1} + eta'_i.psi (eq. p-DP, eq. q-DP) have ratios
// r_i = r'_i = e^{-(x_{i+1}-x_i)/eps}, whose running products telescope to
// e^{-(x_i - x_s)/eps}. Dividing the affine scan by that closed-form product
// leaves two plain sums over the columns,
//   p_i = 2^{-x_i kappa} * sum_{j < zeta(i)} 2^{g_j + y_j kappa}
//   q_i = 2^{+x_i kappa} * sum_{j >= zeta(i)} 2^{g_j - y_j kappa},
// with kappa = 1/(eps ln 2) and g = log2 psi. In extended-exponent arithmetic
// these sums neither overflow nor cancel, so the scan is an associative,
// commutative addition: a prefix sum and a suffix sum over the columns,
// queried by every row at zeta(i).
//
// Work is split into merge-path tiles of T = BLOCK*IPT consecutive elements of
// the merged (rows + columns) sequence, so every tile carries the same amount
// of work on graded meshes. A tile stages its column terms in LDS, scans them
// (per-thread sequential sums, wavefront shuffles, LDS across waves) and then
// answers its rows. Lines longer than one tile get their carries from the
// tile-aggregate kernel (k_tile_aggregate), whose last block per line scans
// the tile totals.
#pragma once
#include "finom_device.hpp"
#include "finom_types.hpp"

namespace finom {

template <typename M>
struct TileGeom {
    long long r0, r1, c0, c1;
};

__device__ __forceinline__ TileGeom<double> tile_geom(const LineDesc& L, int tile, int T)
{
    // Clamped so that a corrupt partition (unsorted input with checks off)
    // can only produce wrong values, never an out-of-range access.
    TileGeom<double> g;
    const long long m0 = (long long)tile * T;
    long long m1 = m0 + T;
    if (m1 > L.R + L.C) m1 = L.R + L.C;
    g.r0 = min(max((long long)L.trs[tile], 0LL), L.R);
    g.r1 = min(max((long long)L.trs[tile + 1], g.r0), L.R);
    g.c0 = min(max(m0 - g.r0, 0LL), L.C);
    g.c1 = min(max(m1 - g.r1, g.c0), L.C);
    if (g.r1 - g.r0 > T) g.r1 = g.r0 + T;
    if (g.c1 - g.c0 > T) g.c1 = g.c0 + T;
    return g;
}

template <int INM>
__device__ __forceinline__ double load_in(const double* p, double scale)
{
    const double v = *p;
    if (INM == IN_LOG2) return v;
    if (INM == IN_NAT) return v * scale;
    return (v > 0.0) ? log2(v) : -__builtin_inf();
}

// Column terms of the lower (L) and upper (U) block, and for the moment
// product the coordinate-weighted terms.
template <typename M, int INM, bool MOMENT>
__device__ __forceinline__ void column_terms(const LineDesc& L, long long j, Ext<M>* t)
{
    const double g = load_in<INM>(L.gin + j * L.gstride, L.in_scale);
    const double y = L.yc[j] - L.shift;
    t[0] = ext_exp2<M>(g + y * L.kappa);
    t[1] = ext_exp2<M>(g - y * L.kappa);
    if (MOMENT) {
        const Ext<M> yy = Ext<M>{frexp_mant((M)y), (y == 0.0) ? kZeroExp : frexp_exp((M)y)};
        t[2] = ext_mul(t[0], yy);
        t[3] = ext_mul(t[1], yy);
    }
}

// ---------------------------------------------------------------------------
// Tile aggregates + per-line carries (only for lines with more than one tile)
// ---------------------------------------------------------------------------
template <typename M, int BLOCK, int IPT, int INM, bool MOMENT>
__global__ __launch_bounds__(BLOCK) void k_tile_aggregate(const WorkItem* __restrict__ work,
                                                         const LineDesc* __restrict__ lines,
                                                         const ProbState* __restrict__ ps,
                                                         Ext<M>* __restrict__ agg,
                                                         Ext<M>* __restrict__ carry,
                                                         unsigned int* __restrict__ line_ctr)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NS = MOMENT ? 4 : 2;
    __shared__ Ext<M> s_tmp[2 * (BLOCK / kWave)];
    __shared__ int s_last;
    const WorkItem w = work[blockIdx.x];
    const LineDesc L = lines[w.line];
    if (ps[L.prob].done) return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const long long nc = tg.c1 - tg.c0;

    Ext<M> acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = ext_zero<M>();
    for (long long k = threadIdx.x; k < nc; k += BLOCK) {
        Ext<M> t[NS];
        column_terms<M, INM, MOMENT>(L, tg.c0 + k, t);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = ext_add(acc[s], t[s]);
    }
#pragma unroll
    for (int s = 0; s < NS; s += 2) {
        Ext<M> el, eu, tl, tu;
        block_scan_both<M, BLOCK>(acc[s], acc[s + 1], el, eu, tl, tu, s_tmp);
        __syncthreads();
        if (threadIdx.x == 0) {
            agg[(long long)(L.agg_base + w.tile) * NS + s] = tl;
            agg[(long long)(L.agg_base + w.tile) * NS + s + 1] = tu;
        }
    }
    // Last block of this line turns the tile totals into carries:
    // lower-block carry = sum over earlier tiles, upper = sum over later tiles.
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int prev = atomicAdd(line_ctr + w.line, 1u);
        s_last = (prev + 1 == (unsigned int)L.ntiles);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int G = L.ntiles;
#pragma unroll
    for (int s = 0; s < NS; s += 2) {
        Ext<M> run_l = ext_zero<M>(), run_u = ext_zero<M>();
        const int nchunks = (G + BLOCK - 1) / BLOCK;
        for (int c = 0; c < nchunks; ++c) {
            // forward chunk c for L, backward chunk (nchunks-1-c) for U
            const int tl_i = c * BLOCK + threadIdx.x;
            const int cu = nchunks - 1 - c;
            const int tu_i = cu * BLOCK + threadIdx.x;
            const Ext<M> vl = (tl_i < G) ? agg[(long long)(L.agg_base + tl_i) * NS + s] : ext_zero<M>();
            const Ext<M> vu = (tu_i < G) ? agg[(long long)(L.agg_base + tu_i) * NS + s + 1] : ext_zero<M>();
            Ext<M> el, eu, totl, totu;
            block_scan_both<M, BLOCK>(vl, vu, el, eu, totl, totu, s_tmp);
            __syncthreads();
            if (tl_i < G) carry[(long long)(L.agg_base + tl_i) * NS + s] = ext_add(run_l, el);
            if (tu_i < G) carry[(long long)(L.agg_base + tu_i) * NS + s + 1] = ext_add(eu, run_u);
            run_l = ext_add(run_l, totl);
            run_u = ext_add(run_u, totu);
        }
    }
    if (threadIdx.x == 0) line_ctr[w.line] = 0u;
}

// ---------------------------------------------------------------------------
// Per-problem reduction of block partials by the last block to finish.
// ---------------------------------------------------------------------------
template <int BLOCK, int EPI>
__device__ __forceinline__ void finish_problem(ProbState* __restrict__ P, double* __restrict__ partial,
                                               int part_off, int nparts, int slot,
                                               double block_value, double* s_red, int* s_last)
{
    if (threadIdx.x == 0) partial[slot] = block_value;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int prev = atomicAdd(&P->counter, 1u);
        *s_last = (prev + 1 == (unsigned int)nparts);
    }
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
    double v = 0.0;
    for (int k = threadIdx.x; k < nparts; k += BLOCK) v += partial[part_off + k];
    v = block_sum_f64<BLOCK>(v, s_red);
    if (threadIdx.x == 0) {
        if (EPI == EPI_UPDATE_CHECK) {
            P->err = v;
            if (!(v == v) || v == __builtin_inf()) P->status = 1;
            if (P->iters >= P->itr_max || !(v > P->tol)) {
                P->done = 1;
                P->converged = (v <= P->tol) ? 1 : 0;
            } else {
                P->iters += 1;
            }
        } else {
            P->w1 = v;
        }
        P->counter = 0u;
    }
}

// ---------------------------------------------------------------------------
// The tile sweep: column terms -> LDS scan -> rows query at zeta -> epilogue
// ---------------------------------------------------------------------------
template <typename M, int BLOCK, int IPT, int INM, int EPI, bool MOMENT>
__global__ __launch_bounds__(BLOCK) void k_sweep(const WorkItem* __restrict__ work,
                                                const LineDesc* __restrict__ lines,
                                                ProbState* __restrict__ ps,
                                                const Ext<M>* __restrict__ carry,
                                                double* __restrict__ partial)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NS = MOMENT ? 4 : 2;
    __shared__ Ext<M> s_sum[NS][T + 1];
    __shared__ Ext<M> s_tmp[2 * (BLOCK / kWave)];
    __shared__ double s_red[BLOCK / kWave];
    __shared__ int s_last;

    const WorkItem w = work[blockIdx.x];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const int nc = (int)(tg.c1 - tg.c0);
    const int nr = (int)(tg.r1 - tg.r0);

    // 1. column terms, striped (coalesced) loads, staged in LDS
    for (int k = threadIdx.x; k < nc; k += BLOCK) {
        Ext<M> t[NS];
        column_terms<M, INM, MOMENT>(L, tg.c0 + k, t);
#pragma unroll
        for (int s = 0; s < NS; ++s) s_sum[s][k] = t[s];
    }
    __syncthreads();

    // 2. blocked scan: thread owns columns [tid*IPT, tid*IPT + IPT)
#pragma unroll
    for (int s = 0; s < NS; s += 2) {
        Ext<M> vl[IPT], vu[IPT];
        Ext<M> sl = ext_zero<M>(), su = ext_zero<M>();
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int idx = threadIdx.x * IPT + q;
            vl[q] = (idx < nc) ? s_sum[s][idx] : ext_zero<M>();
            vu[q] = (idx < nc) ? s_sum[s + 1][idx] : ext_zero<M>();
            sl = ext_add(sl, vl[q]);
            su = ext_add(su, vu[q]);
        }
        Ext<M> el, eu, tl, tu;
        block_scan_both<M, BLOCK>(sl, su, el, eu, tl, tu, s_tmp);
        // exclusive prefix (lower block) and inclusive-from suffix (upper block)
        Ext<M> run = el;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int idx = threadIdx.x * IPT + q;
            if (idx < nc) s_sum[s][idx] = run;
            run = ext_add(run, vl[q]);
        }
        run = eu;
#pragma unroll
        for (int q = IPT - 1; q >= 0; --q) {
            const int idx = threadIdx.x * IPT + q;
            run = ext_add(run, vu[q]);
            if (idx < nc) s_sum[s + 1][idx] = run;
        }
        if (threadIdx.x == 0) {
            s_sum[s][nc] = tl;
            s_sum[s + 1][nc] = ext_zero<M>();
        }
        __syncthreads();
    }

    // 3. rows: each queries the column scan at its dividing index
    Ext<M> cr[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s)
        cr[s] = (L.ntiles > 1) ? carry[(long long)(L.agg_base + w.tile) * NS + s] : ext_zero<M>();

    double red = 0.0;
    for (int k = threadIdx.x; k < nr; k += BLOCK) {
        const long long i = tg.r0 + k;
        const double x = L.xr[i] - L.shift;
        int z = L.zeta[i] - (int)tg.c0;
        z = min(max(z, 0), nc);
        const Ext<M> down = ext_exp2<M>(-x * L.kappa);
        const Ext<M> up = ext_exp2<M>(x * L.kappa);
        double val;
        if (!MOMENT) {
            const Ext<M> pl = ext_mul(ext_add(cr[0], s_sum[0][z]), down);
            const Ext<M> qu = ext_mul(ext_add(s_sum[1][z], cr[1]), up);
            val = ext_log2(ext_add(pl, qu));
        } else {
            // lower: sum (x - y_j) w_j = x S - SY ; upper: sum (y_j - x) w_j = SY - x S
            const Ext<M> xx = Ext<M>{frexp_mant((M)x), (x == 0.0) ? kZeroExp : frexp_exp((M)x)};
            const Ext<M> nx = Ext<M>{-xx.m, xx.e};
            const Ext<M> Sl = ext_add(cr[0], s_sum[0][z]);
            const Ext<M> Su = ext_add(s_sum[1][z], cr[1]);
            const Ext<M> SYl = ext_add(cr[2], s_sum[2][z]);
            const Ext<M> SYu = ext_add(s_sum[3][z], cr[3]);
            Ext<M> dl = ext_add(ext_mul(Sl, xx), Ext<M>{-SYl.m, SYl.e});
            Ext<M> du = ext_add(SYu, ext_mul(Su, nx));
            if (dl.m < M(0)) dl = ext_zero<M>();
            if (du.m < M(0)) du = ext_zero<M>();
            val = ext_log2(ext_add(ext_mul(dl, down), ext_mul(du, up)));
        }
        const long long o = i * L.ostride;
        if (EPI == EPI_STORE_LOG2) {
            L.out[o] = val;
        } else if (EPI == EPI_STORE_NAT) {
            L.out[o] = val * L.out_scale;
        } else if (EPI == EPI_STORE_LIN) {
            L.out[o] = exp2(val);
        } else if (EPI == EPI_UPDATE) {
            L.out[o] = L.a0[o] - val;
        } else if (EPI == EPI_UPDATE_CHECK) {
            // marginal error of the pair checked at the loop head:
            // |psi_old (K^T phi) - v| = v |2^{g_old + t - log2 v} - 1|
            const double lv = L.a0[o];
            const double d = L.a2[o] + val - lv;
            red += L.a1[o] * fabs(expm1(d * 0.69314718055994530942));
            L.out[o] = lv - val;
        } else if (EPI == EPI_COST) {
            red += exp2(L.a0[o] + val);
        }
    }
    if (EPI == EPI_UPDATE_CHECK || EPI == EPI_COST) {
        const double b = block_sum_f64<BLOCK>(red, s_red);
        finish_problem<BLOCK, EPI>(P, partial, L.prob_part_off, L.prob_nparts,
                                   L.part_base + w.tile, b, s_red, &s_last);
    }
}

}  // namespace finom
