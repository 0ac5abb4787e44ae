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

// Wave-level total of per-lane (sum, exponent) pairs against the wave's
// largest exponent; the result is valid in every lane.
__device__ __forceinline__ Ext<float> wave_total_ref(RefAcc a)
{
    const int r = wave_max_i(a.r);
    const float v = ldexp_m(a.s, a.r - r);
    return Ext<float>{readlane_f(wave_incl_prefix_f(v), kWave - 1), r};
}

// Per-wave results of two totals go to LDS (slot wid of s_f / s_i and
// NW + wid); after a barrier every thread combines them with block_total_read.
template <int BLOCK>
__device__ __forceinline__ void block_total2_write(RefAcc a, RefAcc b, float* s_f, int* s_i)
{
    constexpr int NW = BLOCK / kWave;
    const Ext<float> wa = wave_total_ref(a), wb = wave_total_ref(b);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int wid = threadIdx.x / kWave;
        s_f[wid] = wa.m;
        s_i[wid] = wa.e;
        s_f[NW + wid] = wb.m;
        s_i[NW + wid] = wb.e;
    }
}

template <int BLOCK>
__device__ __forceinline__ Ext<float> block_total_read(const float* s_f, const int* s_i)
{
    constexpr int NW = BLOCK / kWave;
    int r = s_i[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = max(r, s_i[w]);
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += ldexp_m(s_f[w], s_i[w] - r);
    return Ext<float>{v, r};
}

// ------------------------------------------------------------ fast sweep
// Lines with unit strides (1D problems) whose tiles passed k_tile_bounds.
// Thread t owns the slots k = t + q BLOCK (q < IPT) of the tile's elements
// listed as [nc columns, nr rows]; column slots stage their terms in LDS, the
// columns are scanned in fixed chunks of IPT per thread, and row slots read
// the scans at their dividing index.

struct FastGeom {
    long long r0, c0;
    int nr, nc;
};

// The tile's row and column ranges, clamped as in tile_geom (a corrupt
// partition gives wrong values, never an access out of range), with at most
// T elements in all.
__device__ __forceinline__ FastGeom fast_geom(const LineDesc& L, int tile, int T, int ts0, int ts1)
{
    const long long m0 = (long long)tile * T;
    long long m1 = m0 + T;
    if (m1 > L.R + L.C) m1 = L.R + L.C;
    const long long r0 = min(max((long long)ts0, 0LL), L.R);
    long long r1 = min(max((long long)ts1, r0), L.R);
    const long long c0 = min(max(m0 - r0, 0LL), L.C);
    long long c1 = min(max(m1 - r1, c0), L.C);
    if (c1 - c0 > T) c1 = c0 + T;
    if ((r1 - r0) + (c1 - c0) > T) r1 = r0 + (T - (c1 - c0));
    return FastGeom{r0, c0, (int)(r1 - r0), (int)(c1 - c0)};
}

template <int BLOCK, int IPT, int EPI, bool NEXT_AGG>
__global__ __launch_bounds__(BLOCK) void k_sweep_fast(const WorkItem* __restrict__ work,
                                                     const LineDesc* __restrict__ lines,
                                                     ProbState* __restrict__ ps,
                                                     const Ext<float>* __restrict__ agg,
                                                     double* __restrict__ partial,
                                                     const double* __restrict__ dec_partial, int parity,
                                                     Ext<float>* __restrict__ agg_next)
{
    static_assert(IPT % 4 == 0, "chunks are read as float4");
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    constexpr bool CHECK = (EPI == EPI_UPDATE_CHECK);
    __shared__ __align__(16) float s_l[T + 4];
    __shared__ __align__(16) float s_u[T + 4];
    __shared__ float s_f[4 * NW];
    __shared__ int s_i[4 * NW];
    __shared__ double s_d[NW];

    const WorkItem w = work[blockIdx.x];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const FastGeom tg = fast_geom(L, w.tile, T, L.trs[w.tile], L.trs[w.tile + 1]);
    const int nc = tg.nc;
    const int nr = tg.nr;
    const bool decide = dec_partial && L.dec_part_off >= 0;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const double* __restrict__ gin = L.gin + tg.c0;
    const Ext<float>* __restrict__ EC = (const Ext<float>*)L.ec + tg.c0;
    const Ext<float>* __restrict__ ER = (const Ext<float>*)L.er + tg.r0;
    const int* __restrict__ ZT = L.zeta + tg.r0;
    const double* __restrict__ A0 = L.a0 + tg.r0;
    const bool empty = nc + nr == 0;   // only with a corrupt partition

    // ---- A. every load of the tile first. Slot k < nc is column k, slot
    // nc <= k < nc + nr is row k - nc; idle slots re-read an element in range.
    Ext<float> Eq[IPT];
    double Dq[IPT];
    int Zq[IPT];
    if (!empty) {
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int k = threadIdx.x + q * BLOCK;
            const bool col = (k < nc) || nr == 0;
            const int ic = min(k, nc - 1);
            const int ir = min(k - nc, nr - 1);
            Eq[q] = col ? EC[ic] : ER[ir];
            Dq[q] = col ? gin[ic] : A0[ir];
            Zq[q] = col ? 0 : ZT[ir];
        }
    }
    double g0 = 0.0;
    Ext<float> E0 = ext_zero<float>();
    if (nc > 0) {
        g0 = gin[0];
        E0 = EC[0];
    }
    RefAcc cl{0.f, kZeroExp}, cu{0.f, kZeroExp};
    if (L.ntiles > 1) {
        Ext<float> al = ext_zero<float>(), au = ext_zero<float>();
        for (int t = threadIdx.x; t < L.ntiles; t += BLOCK) {
            const Ext<float>* a = agg + (long long)(L.agg_base + t) * 2;
            if (t < w.tile) al = ext_add(al, a[0]);
            else if (t > w.tile) au = ext_add(au, a[1]);
        }
        cl = RefAcc{al.m, al.e};
        cu = RefAcc{au.m, au.e};
    }
    double dv = 0.0;
    if (decide)
        for (int k = threadIdx.x; k < L.dec_nparts; k += BLOCK) dv += dec_partial[L.dec_part_off + k];

    // ---- C. column terms against the tile's first column, to LDS
    int r0l = kZeroExp, r0u = kZeroExp;
    if (nc > 0) {
        const Ext<float> e0 = split_exp2(g0);
        r0l = e0.e + E0.e;
        r0u = e0.e - E0.e;
    }
    if (!empty) {
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int k = threadIdx.x + q * BLOCK;
            if (k < nc) {
                const Ext<float> eg = split_exp2(Dq[q]);
                const Ext<float> E = Eq[q];
                s_l[k] = ldexp_m(eg.m * E.m, eg.e + E.e - r0l);
                s_u[k] = ldexp_m(eg.m * __builtin_amdgcn_rcpf(E.m), eg.e - E.e - r0u);
            }
        }
    }
    // carries and the stop decision share the next barrier
    if (L.ntiles > 1) block_total2_write<BLOCK>(cl, cu, s_f + 2 * NW, s_i + 2 * NW);
    if (decide) {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) dv += __shfl_down(dv, d, kWave);
        if (lane == 0) s_d[wid] = dv;
    }
    __syncthreads();
    if (decide) {
        double err = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) err += s_d[v];
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
    if (empty) {
        if (threadIdx.x == 0) {
            if (CHECK) partial[L.part_base + w.tile] = 0.0;
            if (NEXT_AGG && L.ntiles > 1) {
                agg_next[(long long)(L.agg_base + w.tile) * 2 + 0] = ext_zero<float>();
                agg_next[(long long)(L.agg_base + w.tile) * 2 + 1] = ext_zero<float>();
            }
        }
        return;
    }
    Ext<float> CL = ext_zero<float>(), CU = ext_zero<float>();
    if (L.ntiles > 1) {
        CL = block_total_read<BLOCK>(s_f + 2 * NW, s_i + 2 * NW);
        CU = block_total_read<BLOCK>(s_f + 3 * NW, s_i + 3 * NW);
    }
    // row references: the larger of the first column's and the carry's exponent
    const int rl = max(r0l, CL.e), ru = max(r0u, CU.e);
    const float cl_rel = ldexp_m(CL.m, CL.e - rl), cu_rel = ldexp_m(CU.m, CU.e - ru);
    const int shl = r0l - rl, shu = r0u - ru;   // <= 0: rescales the in-tile sums
    double dqc[IPT];
    if (CHECK) {
        // old potential of each row for the marginal-error check, issued
        // before the scan (the weight v = 2^{log2 v} comes from the row's a0)
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int k = threadIdx.x + q * BLOCK;
            dqc[q] = (k >= nc && k < nc + nr) ? L.a2[tg.r0 + (k - nc)] : 0.0;
        }
    }

    // ---- D. scan in fixed chunks: thread t owns columns [t IPT, t IPT + IPT)
    {
        float vl[IPT], vu[IPT];
        const int base = threadIdx.x * IPT;
#pragma unroll
        for (int q = 0; q < IPT; q += 4) {
            const float4 a = *reinterpret_cast<const float4*>(s_l + base + q);
            const float4 b = *reinterpret_cast<const float4*>(s_u + base + q);
            vl[q] = a.x; vl[q + 1] = a.y; vl[q + 2] = a.z; vl[q + 3] = a.w;
            vu[q] = b.x; vu[q + 1] = b.y; vu[q + 2] = b.z; vu[q + 3] = b.w;
        }
        float sl = 0.f, su = 0.f;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const bool live = base + q < nc;
            vl[q] = live ? vl[q] : 0.f;
            vu[q] = live ? vu[q] : 0.f;
            sl += vl[q];
            su += vu[q];
        }
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
        // in place: vl becomes the exclusive prefix, vu the inclusive suffix
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const float t = vl[q];
            vl[q] = run;
            run += t;
        }
#pragma unroll
        for (int q = IPT - 1; q >= 0; --q) {
            runu += vu[q];
            vu[q] = runu;
        }
        __syncthreads();   // every chunk is read before any is overwritten
#pragma unroll
        for (int q = 0; q < IPT; q += 4) {
            *reinterpret_cast<float4*>(s_l + base + q) = make_float4(vl[q], vl[q + 1], vl[q + 2], vl[q + 3]);
            *reinterpret_cast<float4*>(s_u + base + q) = make_float4(vu[q], vu[q + 1], vu[q + 2], vu[q + 3]);
        }
        if (threadIdx.x == BLOCK - 1) {
            s_l[T] = run;      // z = nc = T: everything before
            s_u[T] = 0.f;
        }
        __syncthreads();
    }

    // ---- E. rows: p = (C_L + S_L[z]) 2^{rl - x kappa}, q = (S_U[z] + C_U) 2^{ru + x kappa}
    double red = 0.0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
    double* __restrict__ OUT = L.out + tg.r0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        if (k >= nc && k < nc + nr) {
            int z = Zq[q] - (int)tg.c0;
            z = min(max(z, 0), nc);
            const Ext<float> E = Eq[q];
            const float rE = __builtin_amdgcn_rcpf(E.m);
            const float pm = cl_rel + ldexp_m(s_l[z], shl);
            const float qm = ldexp_m(s_u[z], shu) + cu_rel;
            const double val =
                ext_log2n(ext_add(Ext<float>{pm * rE, rl - E.e}, Ext<float>{qm * E.m, ru + E.e}));
            const double pnew = Dq[q] - val;
            if (CHECK) {
                // |psi_old (K^T phi) - v| = v |2^{g_old + t - log2 v} - 1|, exponent in FP64;
                // the weight v = 2^{log2 v} from the row's operand
                const double d = (dqc[q] - Dq[q]) + val;
                const Ext<float> vv = split_exp2(Dq[q]);
                red += (double)(ldexp_m(vv.m, vv.e) * fabsf(expm1f((float)(d * 0.69314718055994530942))));
            }
            OUT[k - nc] = pnew;
            if (NEXT_AGG) {
                Ext<float> lo, up;
                next_terms(pnew, E, rE, lo, up);
                ref_add(n1, lo);
                ref_add(n2, up);
            }
        }
    }
    if (CHECK) {
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) red += __shfl_down(red, d, kWave);
        if (lane == 0) s_d[wid] = red;
    }
    if (NEXT_AGG && L.ntiles > 1) block_total2_write<BLOCK>(n1, n2, s_f, s_i);
    if (CHECK || (NEXT_AGG && L.ntiles > 1)) {
        __syncthreads();
        if (threadIdx.x == 0) {
            if (CHECK) {
                double b = 0.0;
#pragma unroll
                for (int v = 0; v < NW; ++v) b += s_d[v];
                partial[L.part_base + w.tile] = b;
            }
            if (NEXT_AGG && L.ntiles > 1) {
                agg_next[(long long)(L.agg_base + w.tile) * 2 + 0] = block_total_read<BLOCK>(s_f, s_i);
                agg_next[(long long)(L.agg_base + w.tile) * 2 + 1] = block_total_read<BLOCK>(s_f + NW, s_i + NW);
            }
        }
    }
}

// Tile totals of a fast line's column terms (the carries of its first sweep),
// computed exactly as the update epilogue of the paired sweep computes them:
// the paired sweep's rows are these columns, visited by the same threads in
// the same order (its slots are [its nc = this nr columns..., its rows]).
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
    const FastGeom tg = fast_geom(L, w.tile, T, L.trs[w.tile], L.trs[w.tile + 1]);
    const int nc = tg.nc;
    const int off = tg.nr;
    const Ext<float>* __restrict__ EC = (const Ext<float>*)L.ec + tg.c0;
    const double* __restrict__ gin = L.gin + tg.c0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int j = (int)threadIdx.x + q * BLOCK - off;
        if (j >= 0 && j < nc) {
            const Ext<float> E = EC[j];
            Ext<float> lo, up;
            next_terms(gin[j], E, __builtin_amdgcn_rcpf(E.m), lo, up);
            ref_add(n1, lo);
            ref_add(n2, up);
        }
    }
    block_total2_write<BLOCK>(n1, n2, s_f, s_i);
    __syncthreads();
    if (threadIdx.x == 0) {
        agg[(long long)(L.agg_base + w.tile) * 2 + 0] = block_total_read<BLOCK>(s_f, s_i);
        agg[(long long)(L.agg_base + w.tile) * 2 + 1] = block_total_read<BLOCK>(s_f + NW, s_i + NW);
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
