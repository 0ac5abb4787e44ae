// Fast sweeps for lines whose tiles fit the FP32 exponent range.
//
// Within one merge-path tile the column terms 2^{g_j +- y_j kappa} of the
// Sinkhorn products span a bounded range of binary exponents: after the
// potential update g_j = log2 v_j - log2 (K^T phi)_j, and the kernel entry
// 2^{-kappa |x - y|} changes by at most 2^{kappa |y - y'|} between two
// columns, so over a tile the exponents vary by at most
//   (max - min of log2 v over the tile) + 2 kappa (y_last - y_first).
// When that bound is small (kFastBound) every term of the tile is a normal
// FP32 number relative to the tile's largest exponent, and the tile's prefix
// and suffix sums can run in plain FP32 arithmetic against one block-wide
// reference exponent instead of per-element extended arithmetic. The bound is
// static (meshes, masses, eps), so lines are classified once at setup
// (k_tile_bounds) and the two kinds run as different kernels.
//
// Rows and columns read 2^{c kappa} as a precomputed extended number per mesh
// point (k_exp_coords), so a sweep forms one exponential per column
// (2^{g_j}) and per updated row (2^{new potential}) instead of three.
//
// Tile totals for the next sweep's carries use a block-wide reference too;
// terms more than 2^-126 below the tile's largest vanish, which changes a
// total by less than its own rounding.
#pragma once
#include "finom_kernels.hpp"

namespace finom {

constexpr double kFastBound = 90.0;    // log2 range of a tile's terms

// ------------------------------------------------------------ FP32 helpers

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(dpp_i<CTRL, RM>(0, __float_as_int(v)));
}

__device__ __forceinline__ float readlane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ float wave_incl_prefix_f(float v)
{
    v += dpp_f<0x111>(v);          // row_shr:1
    v += dpp_f<0x112>(v);          // row_shr:2
    v += dpp_f<0x114>(v);          // row_shr:4
    v += dpp_f<0x118>(v);          // row_shr:8
    v += dpp_f<0x142, 0xA>(v);     // row_bcast:15
    v += dpp_f<0x143, 0xC>(v);     // row_bcast:31
    return v;
}

__device__ __forceinline__ float wave_incl_suffix_f(float v)
{
    v += dpp_f<0x101>(v);          // row_shl:1
    v += dpp_f<0x102>(v);          // row_shl:2
    v += dpp_f<0x104>(v);          // row_shl:4
    v += dpp_f<0x108>(v);          // row_shl:8
    const float t1 = readlane_f(v, 16), t2 = readlane_f(v, 32), t3 = readlane_f(v, 48);
    const float s1 = t2 + t3;
    const float s0 = t1 + s1;
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    const float add = (row == 0) ? s0 : (row == 1) ? s1 : (row == 2) ? t3 : 0.f;
    return v + add;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    v = max(v, dpp_i<0x111, 0xF>(kZeroExp, v));
    v = max(v, dpp_i<0x112, 0xF>(kZeroExp, v));
    v = max(v, dpp_i<0x114, 0xF>(kZeroExp, v));
    v = max(v, dpp_i<0x118, 0xF>(kZeroExp, v));
    v = max(v, dpp_i<0x142, 0xA>(kZeroExp, v));
    v = max(v, dpp_i<0x143, 0xC>(kZeroExp, v));
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

// Block maxima of two integers; s_i holds 2 * (BLOCK / 64) entries.
template <int BLOCK>
__device__ __forceinline__ void block_max2_i(int& a, int& b, int* s_i)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int wa = wave_max_i(a), wb = wave_max_i(b);
    __syncthreads();
    if (lane == 0) {
        s_i[wid] = wa;
        s_i[NW + wid] = wb;
    }
    __syncthreads();
    int ra = s_i[0], rb = s_i[NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        ra = max(ra, s_i[w]);
        rb = max(rb, s_i[NW + w]);
    }
    a = ra;
    b = rb;
}

// Block sums of two floats (same order in every block); s_f holds 2 * NW.
template <int BLOCK>
__device__ __forceinline__ void block_sum2_f(float& a, float& b, float* s_f)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const float wa = readlane_f(wave_incl_prefix_f(a), kWave - 1);
    const float wb = readlane_f(wave_incl_prefix_f(b), kWave - 1);
    __syncthreads();
    if (lane == 0) {
        s_f[wid] = wa;
        s_f[NW + wid] = wb;
    }
    __syncthreads();
    float ra = s_f[0], rb = s_f[NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        ra += s_f[w];
        rb += s_f[NW + w];
    }
    a = ra;
    b = rb;
}

// Block totals of two families of extended values, N per thread, against
// the block-wide largest exponent of each family.
template <int BLOCK, int N>
__device__ __forceinline__ void block_total2_ref(const Ext<float>* va, const Ext<float>* vb, Ext<float>& ta,
                                                 Ext<float>& tb, int* s_i, float* s_f)
{
    int ra = kZeroExp, rb = kZeroExp;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        ra = max(ra, va[q].e);
        rb = max(rb, vb[q].e);
    }
    block_max2_i<BLOCK>(ra, rb, s_i);
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        sa += ldexp_m(va[q].m, va[q].e - ra);
        sb += ldexp_m(vb[q].m, vb[q].e - rb);
    }
    block_sum2_f<BLOCK>(sa, sb, s_f);
    ta = Ext<float>{sa, ra};
    tb = Ext<float>{sb, rb};
}

// 2^s as (mantissa in [1, 2), integer exponent), s finite
__device__ __forceinline__ Ext<float> split_exp2(double s)
{
    const double k = floor(s);
    return Ext<float>{__builtin_amdgcn_exp2f((float)(s - k)), (int)k};
}

// log2 of a positive extended value with the mantissa normalised to
// [1/2, 1) first, so the FP32 logarithm works on a small argument
__device__ __forceinline__ double ext_log2n(Ext<float> a)
{
    if (!(a.m > 0.f)) return -__builtin_inf();
    const float mm = __builtin_amdgcn_frexp_mantf(a.m);
    const int me = __builtin_amdgcn_frexp_expf(a.m);
    return (double)__builtin_amdgcn_logf(mm) + (double)(a.e + me);
}

// Terms of the next sweep's columns from a new potential p and the
// column's 2^{c kappa} = E: lower 2^{p + c kappa}, upper 2^{p - c kappa}.
__device__ __forceinline__ void next_terms(double p, Ext<float> E, float rcpE, Ext<float>& lo, Ext<float>& up)
{
    const Ext<float> ep = split_exp2(p);
    lo = Ext<float>{ep.m * E.m, ep.e + E.e};
    up = Ext<float>{ep.m * rcpE, ep.e - E.e};
}

// Per-thread total of extended values against the exponent of the first
// one added (all of a tile's terms lie within kFastBound binary orders of
// each other, so the FP32 sum neither overflows nor loses a relevant term).
struct RefAcc {
    float s;
    int r;
};

__device__ __forceinline__ void ref_add(RefAcc& a, Ext<float> v)
{
    if (a.r == kZeroExp) a.r = v.e;
    a.s += ldexp_m(v.m, v.e - a.r);
}

// ------------------------------------------------------------ fast sweep
// Lines with unit strides (1D problems) whose tiles passed k_tile_bounds.
template <int BLOCK, int IPT, int EPI, bool NEXT_AGG>
__global__ __launch_bounds__(BLOCK) void k_sweep_fast(const WorkItem* __restrict__ work,
                                                     const LineDesc* __restrict__ lines,
                                                     ProbState* __restrict__ ps,
                                                     const Ext<float>* __restrict__ agg,
                                                     double* __restrict__ partial,
                                                     const double* __restrict__ dec_partial, int parity,
                                                     Ext<float>* __restrict__ agg_next)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    constexpr bool CHECK = (EPI == EPI_UPDATE_CHECK);
    __shared__ float s_l[T + 1];
    __shared__ float s_u[T + 1];
    __shared__ float s_f[2 * NW];
    __shared__ int s_i[2 * NW];
    __shared__ double s_red[NW];

    const WorkItem w = work[blockIdx.x];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const int nc = (int)(tg.c1 - tg.c0);
    const int nr = (int)(tg.r1 - tg.r0);
    const int ncq = (nc + BLOCK - 1) / BLOCK;
    const int nrq = (nr + BLOCK - 1) / BLOCK;
    const bool decide = dec_partial && L.dec_part_off >= 0;
    const double* __restrict__ gin = L.gin + tg.c0;
    const Ext<float>* __restrict__ EC = (const Ext<float>*)L.ec + tg.c0;
    const Ext<float>* __restrict__ ER = (const Ext<float>*)L.er + tg.r0;
    const int* __restrict__ ZT = L.zeta + tg.r0;
    const double* __restrict__ A0 = L.a0 + tg.r0;

    // ---- A. every load of the tile first (tail lanes re-read an in-range element)
    double gq[IPT], a0q[IPT];
    Ext<float> ecq[IPT], erq[IPT];
    int zq[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= ncq) break;
        const int j = min((int)threadIdx.x + q * BLOCK, nc - 1);
        gq[q] = gin[j];
        ecq[q] = EC[j];
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= nrq) break;
        const int i = min((int)threadIdx.x + q * BLOCK, nr - 1);
        erq[q] = ER[i];
        zq[q] = ZT[i];
        a0q[q] = A0[i];
    }
    // reference exponents: the tile's first column terms
    double g0 = 0.0;
    Ext<float> E0 = ext_zero<float>();
    if (nc > 0) {
        g0 = gin[0];
        E0 = EC[0];
    }
    Ext<float> cl = ext_zero<float>(), cu = ext_zero<float>();
    if (L.ntiles > 1) {
        for (int t = threadIdx.x; t < L.ntiles; t += BLOCK) {
            const Ext<float>* a = agg + (long long)(L.agg_base + t) * 2;
            if (t < w.tile) cl = ext_add(cl, a[0]);
            else if (t > w.tile) cu = ext_add(cu, a[1]);
        }
    }
    double dv = 0.0;
    if (decide)
        for (int k = threadIdx.x; k < L.dec_nparts; k += BLOCK) dv += dec_partial[L.dec_part_off + k];

    // ---- B. stop decision of the loop head (uniform across the block)
    if (decide) {
        const double err = block_sum_f64<BLOCK>(dv, s_red);
        const long long l = P->cnt[parity];
        const bool stop = (l >= P->itr_max) || !(err > P->tol);
        if (L.writes_state && w.tile == 0 && threadIdx.x == 0) {
            P->err = err;
            if (!(err == err) || err == __builtin_inf()) P->status = 1;
            if (stop) {
                P->iters = l;
                P->converged = (err <= P->tol) ? 1 : 0;
                P->done = 1;
            } else {
                P->cnt[parity ^ 1] = l + 1;
            }
        }
        if (stop) return;
    }

    // ---- C. carries, references, column terms straight to LDS
    Ext<float> CL = ext_zero<float>(), CU = ext_zero<float>();
    if (L.ntiles > 1) block_total2_ref<BLOCK, 1>(&cl, &cu, CL, CU, s_i, s_f);
    int rl = CL.e, ru = CU.e;
    if (nc > 0) {
        const Ext<float> e0 = split_exp2(g0);
        rl = max(rl, e0.e + E0.e);
        ru = max(ru, e0.e - E0.e);
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= ncq) break;
        const int k = threadIdx.x + q * BLOCK;
        if (k < nc) {
            const Ext<float> eg = split_exp2(gq[q]);
            const Ext<float> E = ecq[q];
            s_l[k] = ldexp_m(eg.m * E.m, eg.e + E.e - rl);
            s_u[k] = ldexp_m(eg.m * __builtin_amdgcn_rcpf(E.m), eg.e - E.e - ru);
        }
    }
    const float cl_rel = ldexp_m(CL.m, CL.e - rl);
    const float cu_rel = ldexp_m(CU.m, CU.e - ru);
    __syncthreads();

    // ---- D. blocked scan: thread owns columns [tid*ncq, tid*ncq + ncq)
    {
        float vl[IPT], vu[IPT];
        float sl = 0.f, su = 0.f;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q >= ncq) break;
            const int idx = threadIdx.x * ncq + q;
            vl[q] = (idx < nc) ? s_l[idx] : 0.f;
            vu[q] = (idx < nc) ? s_u[idx] : 0.f;
            sl += vl[q];
            su += vu[q];
        }
        const int lane = threadIdx.x & (kWave - 1);
        const int wid = threadIdx.x / kWave;
        const float il = wave_incl_prefix_f(sl);
        const float iu = wave_incl_suffix_f(su);
        if (lane == kWave - 1) s_f[wid] = il;
        if (lane == 0) s_f[NW + wid] = iu;
        __syncthreads();
        float pre = 0.f, suf = 0.f;
        for (int v = 0; v < wid; ++v) pre += s_f[v];
        for (int v = wid + 1; v < NW; ++v) suf += s_f[NW + v];
        float run = pre + dpp_f<0x138>(il);    // wave_shr:1 -> exclusive prefix
        float runu = dpp_f<0x130>(iu) + suf;   // wave_shl:1 -> exclusive suffix
        const float tot = pre + readlane_f(il, kWave - 1);
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q >= ncq) break;
            const int idx = threadIdx.x * ncq + q;
            if (idx < nc) s_l[idx] = run;
            run += vl[q];
        }
#pragma unroll
        for (int q = IPT - 1; q >= 0; --q) {
            if (q >= ncq) continue;
            const int idx = threadIdx.x * ncq + q;
            runu += vu[q];
            if (idx < nc) s_u[idx] = runu;
        }
        if (threadIdx.x == BLOCK - 1) s_l[nc] = tot;
        if (threadIdx.x == 0) s_u[nc] = 0.f;
        __syncthreads();
    }

    // ---- E. rows: p = (C_L + S_L[z]) 2^{rl - x kappa}, q = (S_U[z] + C_U) 2^{ru + x kappa}
    double red = 0.0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
    double* __restrict__ OUT = L.out + tg.r0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= nrq) break;
        const int k = threadIdx.x + q * BLOCK;
        const bool live = k < nr;
        int z = zq[q] - (int)tg.c0;
        z = min(max(z, 0), nc);
        const Ext<float> E = erq[q];
        const float rE = __builtin_amdgcn_rcpf(E.m);
        const float pm = cl_rel + s_l[z];
        const float qm = s_u[z] + cu_rel;
        const double val = ext_log2n(ext_add(Ext<float>{pm * rE, rl - E.e}, Ext<float>{qm * E.m, ru + E.e}));
        const double pnew = a0q[q] - val;
        if (CHECK && live) {
            // |psi_old (K^T phi) - v| = v |2^{g_old + t - log2 v} - 1|, exponent in FP64
            const long long o = tg.r0 + k;
            const double d = (L.a2[o] - a0q[q]) + val;
            red += (double)((float)L.a1[o] * fabsf(expm1f((float)(d * 0.69314718055994530942))));
        }
        if (live) {
            OUT[k] = pnew;
            if (NEXT_AGG) {
                Ext<float> lo, up;
                next_terms(pnew, E, rE, lo, up);
                ref_add(n1, lo);
                ref_add(n2, up);
            }
        }
    }
    if (CHECK) {
        const double b = block_sum_f64<BLOCK>(red, s_red);
        if (threadIdx.x == 0) partial[L.part_base + w.tile] = b;
    }
    if (NEXT_AGG && L.ntiles > 1) {
        Ext<float> a1 = Ext<float>{n1.s, n1.r}, a2 = Ext<float>{n2.s, n2.r}, t1, t2;
        block_total2_ref<BLOCK, 1>(&a1, &a2, t1, t2, s_i, s_f);
        if (threadIdx.x == 0) {
            agg_next[(long long)(L.agg_base + w.tile) * 2 + 0] = t1;
            agg_next[(long long)(L.agg_base + w.tile) * 2 + 1] = t2;
        }
    }
}

// Tile totals of a fast line's column terms (the carries of its first sweep),
// computed exactly as the update epilogue computes them.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_tile_aggregate_fast(const WorkItem* __restrict__ work,
                                                              const LineDesc* __restrict__ lines,
                                                              ProbState* __restrict__ ps,
                                                              Ext<float>* __restrict__ agg)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ float s_f[2 * NW];
    __shared__ int s_i[2 * NW];
    const WorkItem w = work[blockIdx.x];
    const LineDesc L = lines[w.line];
    if (ps[L.prob].done) return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const int nc = (int)(tg.c1 - tg.c0);
    const Ext<float>* __restrict__ EC = (const Ext<float>*)L.ec + tg.c0;
    const double* __restrict__ gin = L.gin + tg.c0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        if (k < nc) {
            const Ext<float> E = EC[k];
            Ext<float> lo, up;
            next_terms(gin[k], E, __builtin_amdgcn_rcpf(E.m), lo, up);
            ref_add(n1, lo);
            ref_add(n2, up);
        }
    }
    Ext<float> a1 = Ext<float>{n1.s, n1.r}, a2 = Ext<float>{n2.s, n2.r}, t1, t2;
    block_total2_ref<BLOCK, 1>(&a1, &a2, t1, t2, s_i, s_f);
    if (threadIdx.x == 0) {
        agg[(long long)(L.agg_base + w.tile) * 2 + 0] = t1;
        agg[(long long)(L.agg_base + w.tile) * 2 + 1] = t2;
    }
}

// One block per tile of a partition: flags[flag] |= 1 when the tile's
// column terms may span more than kFastBound binary orders
//   bound = (max - min of log2 mass over the tile's columns) + 2 kappa span.
struct BoundTask {
    const double* yc;       // columns
    const double* lmass;    // log2 column masses
    const int* trs;         // tile row starts
    long long R, C;
    double kappa;
    int T, ntiles;
    int flag;
    int pad;
};

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_tile_bounds(const BoundTask* __restrict__ tasks,
                                                      const int* __restrict__ first, int ntasks,
                                                      int* __restrict__ flags)
{
    __shared__ double s_red[BLOCK / kWave];
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const BoundTask tk = tasks[lo];
    const int t = blockIdx.x - first[lo];
    const long long m0 = (long long)t * tk.T;
    long long m1 = m0 + tk.T;
    if (m1 > tk.R + tk.C) m1 = tk.R + tk.C;
    const long long r0 = min(max((long long)tk.trs[t], 0LL), tk.R);
    const long long r1 = min(max((long long)tk.trs[t + 1], r0), tk.R);
    // the tile's columns plus one neighbour on each side: the carries from
    // the other tiles then lie within the bound of the tile's own terms
    const long long c0 = max(min(max(m0 - r0, 0LL), tk.C) - 1, 0LL);
    const long long c1 = min(min(max(m1 - r1, c0), tk.C) + 1, tk.C);
    if (c1 <= c0) return;
    double mx = -__builtin_inf(), mn = __builtin_inf();
    for (long long j = c0 + threadIdx.x; j < c1; j += BLOCK) {
        const double v = tk.lmass[j];
        mx = fmax(mx, v);
        mn = fmin(mn, v);
    }
    // block max of mx and of -mn
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        mx = fmax(mx, __shfl_down(mx, d, kWave));
        mn = fmin(mn, __shfl_down(mn, d, kWave));
    }
    __shared__ double s_mn[NW];
    if (lane == 0) {
        s_red[wid] = mx;
        s_mn[wid] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = s_red[0], b = s_mn[0];
        for (int v = 1; v < NW; ++v) {
            a = fmax(a, s_red[v]);
            b = fmin(b, s_mn[v]);
        }
        const double bound = (a - b) + 2.0 * tk.kappa * (tk.yc[c1 - 1] - tk.yc[c0]);
        if (!(bound <= kFastBound)) atomicOr(flags + tk.flag, 1);
    }
}

}  // namespace finom
