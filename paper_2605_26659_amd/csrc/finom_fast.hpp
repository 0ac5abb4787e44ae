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
// State. A fast problem keeps its scaling vectors as extended numbers
// instead of log potentials: per point c with scaling w (phi or psi) the
// state is U = w 2^{-c kappa}; the masses are kept as A = u or v and the mesh
// as B = 2^{2 c kappa}, all Ext<float> (8 bytes, as many as a log potential).
// Then a column's two terms are w 2^{+c kappa} = U B and w 2^{-c kappa} = U,
// and a row x with in-tile sums L (lower block) and R (upper block) has
//   (K w)_x = 2^{-x kappa} (L + B_x R),
// so the update w_x = A_x / (K w)_x is the state U_x = A_x / (L + B_x R):
// one multiply-add, one reciprocal, no exponential or logarithm per element.
// The marginal error of the check is |w_old (K w') - A| = |U_old W - A| with
// W = L + B R. The log potentials are formed once, when the loop has ended.
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

// Row broadcast for a reduction whose result is read in the wave's last lane:
// the rows the broadcast does not write are left undefined (no identity to
// materialise first), and none of them feeds the last lane.
template <int CTRL, int RM>
__device__ __forceinline__ float dpp_bc_f(float v)
{
    static_assert(CTRL == 0x142 || CTRL == 0x143, "row broadcasts only");
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, RM, 0xF, false));
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

// Sum over the wave (every lane gets it), in the order of the prefix above.
__device__ __forceinline__ float wave_sum_f(float v)
{
    v += dpp_f<0x111>(v);
    v += dpp_f<0x112>(v);
    v += dpp_f<0x114>(v);
    v += dpp_f<0x118>(v);
    v += dpp_bc_f<0x142, 0xA>(v);
    v += dpp_bc_f<0x143, 0xC>(v);
    return readlane_f(v, kWave - 1);
}

// Sum of lanes [0, N) (N <= 16, a power of two), read from lane N - 1.
template <int N>
__device__ __forceinline__ float first_lanes_sum_f(float v)
{
    static_assert(N >= 1 && N <= 16 && (N & (N - 1)) == 0, "one row, power of two");
    if (N > 1) v += dpp_f<0x111>(v);
    if (N > 2) v += dpp_f<0x112>(v);
    if (N > 4) v += dpp_f<0x114>(v);
    if (N > 8) v += dpp_f<0x118>(v);
    return readlane_f(v, N - 1);
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

// Maxima take INT_MIN, the identity of max, where the DPP source is missing,
// so that each step folds into a single max with a DPP operand.
constexpr int kMaxIdentity = -2147483647 - 1;

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_max_i(int v)
{
    return max(v, dpp_i<CTRL, RM>(kMaxIdentity, v));
}

__device__ __forceinline__ int wave_max_i(int v)
{
    v = dpp_max_i<0x111>(v);
    v = dpp_max_i<0x112>(v);
    v = dpp_max_i<0x114>(v);
    v = dpp_max_i<0x118>(v);
    v = dpp_max_i<0x142, 0xA>(v);
    v = dpp_max_i<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

template <int N>
__device__ __forceinline__ int first_lanes_max_i(int v)
{
    static_assert(N >= 1 && N <= 16 && (N & (N - 1)) == 0, "one row, power of two");
    if (N > 1) v = dpp_max_i<0x111>(v);
    if (N > 2) v = dpp_max_i<0x112>(v);
    if (N > 4) v = dpp_max_i<0x114>(v);
    if (N > 8) v = dpp_max_i<0x118>(v);
    return __builtin_amdgcn_readlane(v, N - 1);
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
    const float wa = wave_sum_f(a);
    const float wb = wave_sum_f(b);
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

// Mantissa into [1/2, 1) (exact). Every stored state, mass and total is kept
// normalised: the tile scans set their reference from exponents alone, which
// is only within a factor 4 of the magnitude when mantissas are normalised.
__device__ __forceinline__ Ext<float> ext_norm(Ext<float> a)
{
    return Ext<float>{__builtin_amdgcn_frexp_mantf(a.m), a.e + __builtin_amdgcn_frexp_expf(a.m)};
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
    return Ext<float>{wave_sum_f(v), r};
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
    return ext_norm(Ext<float>{v, r});
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

// The loaded operands of one tile: per slot B = 2^{2 c kappa} of its point
// and V, the column's state or the row's mass; per row slot its dividing
// index Z.
template <int IPT>
struct FastTileIn {
    FastGeom tg;
    Ext<float> B[IPT];
    Ext<float> V[IPT];
    int Z[IPT];
    Ext<float> U0, B0;  // the first column's state and B
};

// Row offset of slot k, clamped into the tile's rows (idle slots and column
// slots read row 0).
__device__ __forceinline__ unsigned fast_row_index(int k, int nc, int nr)
{
    return (unsigned)min(max(k - nc, 0), max(nr - 1, 0));
}

// Every load of a tile. Offsets are 32-bit from tile bases clamped into the
// arrays (lines have at least one row and one column, so index 0 of an
// empty part is still in range). A wave whose 64 slots are all columns or
// all rows takes a branch of its own with uniform bases; only the wave that
// straddles the boundary selects a base per lane. Every branch issues the
// same loads, so the compiler can still wait for one slot's data alone.
template <int BLOCK, int IPT>
__device__ __forceinline__ void fast_tile_load(FastTileIn<IPT>& t, const LineDesc& L)
{
    const int nc = t.tg.nc, nr = t.tg.nr;
    const long long cb = min(t.tg.c0, L.C - 1), rb = min(t.tg.r0, L.R - 1);
    const gptr<const Ext<float>> UC = gbl((const Ext<float>*)L.gin) + cb;
    const gptr<const Ext<float>> BC = gbl((const Ext<float>*)L.ec) + cb;
    const gptr<const Ext<float>> BR = gbl((const Ext<float>*)L.er) + rb;
    const gptr<const Ext<float>> AR = gbl((const Ext<float>*)L.a0) + rb;
    const gptr<const int> ZR = gbl(L.zeta) + rb;
    const unsigned ncm = (unsigned)max(nc - 1, 0);
    t.U0 = UC[0];
    t.B0 = BC[0];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        const int kw = __builtin_amdgcn_readfirstlane(k);   // slot of the wave's lane 0
        const unsigned ir = fast_row_index(k, nc, nr);
        t.Z[q] = ZR[ir];
        if (kw + kWave <= nc) {
            t.B[q] = BC[(unsigned)k];
            t.V[q] = UC[(unsigned)k];
        } else if (kw >= nc) {
            t.B[q] = BR[ir];
            t.V[q] = AR[ir];
        } else {
            const bool col = k < nc;
            const unsigned ic = min((unsigned)k, ncm);
            t.B[q] = col ? BC[ic] : BR[ir];
            t.V[q] = col ? UC[ic] : AR[ir];
        }
    }
}

// Old state of each row for the marginal-error check.
template <int BLOCK, int IPT>
__device__ __forceinline__ void fast_tile_check_loads(const FastTileIn<IPT>& t, const LineDesc& L,
                                                      Ext<float>* uold)
{
    const gptr<const Ext<float>> UO = gbl((const Ext<float>*)L.a2) + min(t.tg.r0, L.R - 1);
#pragma unroll
    for (int q = 0; q < IPT; ++q) uold[q] = UO[fast_row_index(threadIdx.x + q * BLOCK, t.tg.nc, t.tg.nr)];
}

// Column terms U B (lower block) and U (upper block) against the tile's
// first column, to LDS.
template <int BLOCK, int IPT>
__device__ __forceinline__ void fast_tile_columns(const FastTileIn<IPT>& t, float* s_l, float* s_u, int& r0l,
                                                  int& r0u)
{
    const int nc = t.tg.nc;
    r0l = kZeroExp;
    r0u = kZeroExp;
    if (nc > 0) {
        r0l = t.U0.e + t.B0.e;
        r0u = t.U0.e;
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        if (k < nc) {
            const Ext<float> U = t.V[q], B = t.B[q];
            s_l[k] = ldexp_m(U.m * B.m, U.e + B.e - r0l);
            s_u[k] = ldexp_m(U.m, U.e - r0u);
        }
    }
}

// Exclusive prefix (s_l) and inclusive suffix (s_u) of the tile's columns in
// place, thread t owning columns [t IPT, t IPT + IPT); the caller has passed a
// barrier since the columns were written. s_f holds 2 * (BLOCK / 64) entries.
// With SYNC the results are visible to the block on return; without, the
// caller passes a barrier before reading them.
template <int BLOCK, int IPT, bool SYNC = true>
__device__ __forceinline__ void fast_tile_scan(float* s_l, float* s_u, int nc, float* s_f)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    float vl[IPT], vu[IPT];
    const int base = threadIdx.x * IPT;
    // chunks wholly inside or wholly past the columns need no per-entry mask
    // (only one thread has a chunk that straddles the end)
    if (base >= nc) {
#pragma unroll
        for (int q = 0; q < IPT; ++q) vl[q] = vu[q] = 0.f;
    } else {
#pragma unroll
        for (int q = 0; q < IPT; q += 4) {
            const float4 a = *reinterpret_cast<const float4*>(s_l + base + q);
            const float4 b = *reinterpret_cast<const float4*>(s_u + base + q);
            vl[q] = a.x; vl[q + 1] = a.y; vl[q + 2] = a.z; vl[q + 3] = a.w;
            vu[q] = b.x; vu[q + 1] = b.y; vu[q + 2] = b.z; vu[q + 3] = b.w;
        }
        if (base + IPT > nc) {
#pragma unroll
            for (int q = 0; q < IPT; ++q) {
                const bool live = base + q < nc;
                vl[q] = live ? vl[q] : 0.f;
                vu[q] = live ? vu[q] : 0.f;
            }
        }
    }
    float sl = 0.f, su = 0.f;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        sl += vl[q];
        su += vu[q];
    }
    const float il = wave_incl_prefix_f(sl);
    const float iu = wave_incl_suffix_f(su);
    if (lane == kWave - 1) s_f[wid] = il;
    if (lane == 0) s_f[NW + wid] = iu;
    __syncthreads();
    // the other waves' totals: lane j < NW reads wave j's, and the lanes of the
    // waves before (prefix) / after (suffix) this one are summed across lanes
    const int j = lane & (NW - 1);
    const bool head = lane < NW;
    float a = s_f[j], b = s_f[NW + j];
    a = (head && j < wid) ? a : 0.f;
    b = (head && j > wid) ? b : 0.f;
    const float pre = first_lanes_sum_f<NW>(a);
    const float suf = first_lanes_sum_f<NW>(b);
    float run = pre + dpp_f<0x138>(il);    // wave_shr:1 -> exclusive prefix
    float runu = dpp_f<0x130>(iu) + suf;   // wave_shl:1 -> exclusive suffix
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
    // every chunk was read before the barrier above, so the chunks can be
    // overwritten in place
#pragma unroll
    for (int q = 0; q < IPT; q += 4) {
        *reinterpret_cast<float4*>(s_l + base + q) = make_float4(vl[q], vl[q + 1], vl[q + 2], vl[q + 3]);
        *reinterpret_cast<float4*>(s_u + base + q) = make_float4(vu[q], vu[q + 1], vu[q + 2], vu[q + 3]);
    }
    if (threadIdx.x == BLOCK - 1) {
        s_l[BLOCK * IPT] = run;      // z = nc = T: everything before
        s_u[BLOCK * IPT] = 0.f;
    }
    if (SYNC) __syncthreads();
}

// Rows of a scanned tile. With the carries, the row's sums are
// L = (C_L + S_L[z]) and R = (S_U[z] + C_U), against the row references rl,
// ru (the larger of the first column's and the carry's exponent); the new
// state is U = A / (L + B R). New states go to un (stored by the caller after
// the loop: a store inside it would make each later wait on the check loads
// also wait for that store), the check term |U_old W - A| to red, the next
// sweep's column terms U B and U to n1 / n2.
template <int BLOCK, int IPT, int EPI, bool NEXT_AGG>
__device__ __forceinline__ void fast_tile_rows(const FastTileIn<IPT>& t, const float* s_l, const float* s_u,
                                               Ext<float> CL, Ext<float> CU, int r0l, int r0u,
                                               const Ext<float>* uold, Ext<float>* un, double& red, RefAcc& n1,
                                               RefAcc& n2)
{
    constexpr bool CHECK = (EPI == EPI_UPDATE_CHECK);
    const int nc = t.tg.nc, nr = t.tg.nr;
    const int rl = max(r0l, CL.e), ru = max(r0u, CU.e);
    const float cl_rel = ldexp_m(CL.m, CL.e - rl), cu_rel = ldexp_m(CU.m, CU.e - ru);
    const int shl = r0l - rl, shu = r0u - ru;   // <= 0: rescales the in-tile sums
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        un[q] = ext_zero<float>();
        if (k >= nc && k < nc + nr) {
            int z = t.Z[q] - (int)t.tg.c0;
            z = min(max(z, 0), nc);
            const Ext<float> B = t.B[q], A = t.V[q];
            const float pm = cl_rel + ldexp_m(s_l[z], shl);
            const float qm = ldexp_m(s_u[z], shu) + cu_rel;
            const Ext<float> W = ext_add(Ext<float>{pm, rl}, Ext<float>{qm * B.m, ru + B.e});
            const Ext<float> U = ext_norm(Ext<float>{A.m * __builtin_amdgcn_rcpf(W.m), A.e - W.e});
            if (CHECK) {
                // |U_old W - A| with one rounding: product and difference in one
                // fused multiply-add, both operands scaled (exactly) to the larger
                // of the two exponents so that neither can overflow
                const Ext<float> O = uold[q];
                const int ep = O.e + W.e;
                const int re = max(ep, A.e);
                const float d = __builtin_fmaf(ldexp_m(O.m, ep - re), W.m, -ldexp_m(A.m, A.e - re));
                red += __builtin_amdgcn_ldexp((double)fabsf(d), re);
            }
            un[q] = U;
            if (NEXT_AGG) {
                ref_add(n1, Ext<float>{U.m * B.m, U.e + B.e});
                ref_add(n2, U);
            }
        }
    }
}

template <int BLOCK, int IPT>
__device__ __forceinline__ void fast_tile_store(const FastTileIn<IPT>& t, const LineDesc& L, const Ext<float>* un)
{
    const gptr<Ext<float>> OUT = gbl((Ext<float>*)L.out) + min(t.tg.r0, L.R - 1);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        if (k >= t.tg.nc && k < t.tg.nc + t.tg.nr) store_update(OUT + (unsigned)(k - t.tg.nc), un[q]);
    }
}

// Stop decision of the loop head from the block's sum of the checking
// sweep's partials (every block sums them in the same order). Returns true
// when the iteration stops.
__device__ __forceinline__ bool fast_decide(const LineDesc& L, int tile, ProbState* P, double err, int parity)
{
    const long long l = P->cnt[parity];
    const bool stop = (l >= P->itr_max) || !(err > P->tol);
    if (L.writes_state && tile == 0 && threadIdx.x == 0) {
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
    return stop;
}

// Two fixed slots per thread of tile aggregates and decision partials
// (loaded before the tiles, so that no wait sits between them); BIG adds
// loops over the rest, which sit in that kernel variant only because a loop
// with loads makes the compiler wait for every load issued before it.
constexpr int kFastFix = 2;

template <int BLOCK>
__device__ __forceinline__ void fast_fixed_loads(const LineDesc& L, const Ext<float>* agg,
                                                 const double* dec_partial, int np,
                                                 Ext<float> (&af)[kFastFix][2], double (&df)[kFastFix])
{
    if (np > 0) {
        const gptr<const double> DP = gbl(dec_partial) + L.dec_part_off;
#pragma unroll
        for (int f = 0; f < kFastFix; ++f) df[f] = DP[min((int)threadIdx.x + f * BLOCK, np - 1)];
    }
    const gptr<const Ext<float>> AG = gbl(agg) + (long long)L.agg_base * 2;
#pragma unroll
    for (int f = 0; f < kFastFix; ++f) {
        const int t = min((int)threadIdx.x + f * BLOCK, L.ntiles - 1);
        af[f][0] = AG[2 * t];
        af[f][1] = AG[2 * t + 1];
    }
}

// The BIG loops request kFastBatch elements per thread before adding any of
// them (one memory latency per batch, not per element), in the same order.
constexpr int kFastBatch = 8;

template <int BLOCK, bool BIG>
__device__ __forceinline__ double fast_decision_sum(const LineDesc& L, const double* dec_partial, int np,
                                                    const double (&df)[kFastFix])
{
    double dv = 0.0;
    if (np > 0) {
#pragma unroll
        for (int f = 0; f < kFastFix; ++f)
            if ((int)threadIdx.x + f * BLOCK < np) dv += df[f];
        if constexpr (BIG) {
            const gptr<const double> DP = gbl(dec_partial) + L.dec_part_off;
            for (int k0 = threadIdx.x + kFastFix * BLOCK; k0 < np; k0 += kFastBatch * BLOCK) {
                double v[kFastBatch];
#pragma unroll
                for (int u = 0; u < kFastBatch; ++u) v[u] = DP[min(k0 + u * BLOCK, np - 1)];
#pragma unroll
                for (int u = 0; u < kFastBatch; ++u)
                    if (k0 + u * BLOCK < np) dv += v[u];
            }
        }
    }
    return dv;
}

// Per-thread carries of tile `tile`: lower terms of the tiles before it,
// upper terms of the tiles after it.
template <int BLOCK, bool BIG>
__device__ __forceinline__ void fast_carries(const LineDesc& L, const Ext<float>* agg, int tile,
                                             const Ext<float> (&af)[kFastFix][2], RefAcc& cl, RefAcc& cu)
{
    const int nt = L.ntiles;
    Ext<float> al = ext_zero<float>(), au = ext_zero<float>();
#pragma unroll
    for (int f = 0; f < kFastFix; ++f) {
        const int t = threadIdx.x + f * BLOCK;
        if (t < nt && t < tile) al = ext_add(al, af[f][0]);
        if (t < nt && t > tile) au = ext_add(au, af[f][1]);
    }
    if constexpr (BIG) {
        const gptr<const Ext<float>> AG = gbl(agg) + (long long)L.agg_base * 2;
        for (int t0 = threadIdx.x + kFastFix * BLOCK; t0 < nt; t0 += kFastBatch * BLOCK) {
            Ext<float> v[kFastBatch];
#pragma unroll
            for (int u = 0; u < kFastBatch; ++u) {
                const int t = min(t0 + u * BLOCK, nt - 1);
                v[u] = AG[2 * t + (t > tile ? 1 : 0)];   // lower total before the tile, upper after
            }
#pragma unroll
            for (int u = 0; u < kFastBatch; ++u) {
                const int t = t0 + u * BLOCK;
                if (t < nt && t < tile) al = ext_add(al, v[u]);
                else if (t < nt && t > tile) au = ext_add(au, v[u]);
            }
        }
    }
    cl = RefAcc{al.m, al.e};
    cu = RefAcc{au.m, au.e};
}

template <int BLOCK>
__device__ __forceinline__ void wave_sum_to(double v, double* s)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = v;
}

template <int BLOCK>
__device__ __forceinline__ double block_read_sum(const double* s)
{
    double b = 0.0;
#pragma unroll
    for (int v = 0; v < BLOCK / kWave; ++v) b += s[v];
    return b;
}

// One tile per block.
// Lines with more tiles than kFastFix per thread take their carries from
// k_fast_carries (two numbers per tile, computed once per sweep) instead of
// every tile's totals, and that kernel takes their stop decision.
template <int BLOCK>
__device__ __forceinline__ bool fast_carried(const LineDesc& L) { return L.ntiles > kFastFix * BLOCK; }

// Tiles per thread whose totals the carries pre-pass keeps in registers:
// lines of up to kCarryRegs x BLOCK tiles read their totals once, requested
// together with the decision's partials; longer lines read them once per scan.
constexpr int kCarryRegs = 16;

// One block per carried line: the stop decision (with dec_partial) and the
// carries of every tile, the exclusive prefix of the tiles' lower totals and
// the exclusive suffix of their upper totals (carries laid out as agg).
// Each thread scans a run of consecutive tiles. On lines of up to
// kCarryRegs x BLOCK tiles the totals and the carries pass through LDS, so
// that global memory is read and written coalesced (lane k at tile k + u BLOCK,
// both numbers of a tile in one 16-byte access): a wave's access to its
// threads' runs directly would touch a separate cache line per lane.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fast_carries(const int* __restrict__ big, const LineDesc* __restrict__ lines,
                                                       ProbState* __restrict__ ps, const Ext<float>* __restrict__ agg,
                                                       Ext<float>* __restrict__ carries,
                                                       const double* __restrict__ dec_partial, int parity)
{
    constexpr int NW = BLOCK / kWave;
    constexpr int U = kFastBatch;
    constexpr int K = kCarryRegs;
    constexpr int NT = K * BLOCK;         // tiles the LDS path holds
    constexpr int NP = NT + NT / 16;      // one pad slot after every 16 tiles
    __shared__ Ext<float> s_tmp[2 * NW];
    __shared__ double s_red[NW];
    __shared__ Ext<float> s_lo[NP], s_up[NP];
    const LineDesc L = lines[big[blockIdx.x]];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const int nt = L.ntiles;
    const int ch = (nt + BLOCK - 1) / BLOCK;   // tiles per thread, consecutive
    const int t0 = threadIdx.x * ch, t1 = min(t0 + ch, nt);
    const gptr<const Ext<float>> AG = gbl(agg) + (long long)L.agg_base * 2;
    const gptr<Ext<float>> CR = gbl(carries) + (long long)L.agg_base * 2;
    const bool inreg = ch <= K;   // block-uniform
    auto pad = [](int t) { return t + (t >> 4); };
    // the totals, requested before the decision's partials so that both arrive
    // in one round trip (indices clamped into the line)
    int4 q[K];
    if (inreg) {
        const gptr<const int4> AG4 = (gptr<const int4>)AG;
#pragma unroll
        for (int u = 0; u < K; ++u) q[u] = AG4[min((int)threadIdx.x + u * BLOCK, nt - 1)];
    }
    if (dec_partial && L.dec_part_off >= 0) {
        const double err = block_sum_f64<BLOCK>(strided_sum<BLOCK>(dec_partial + L.dec_part_off, L.dec_nparts), s_red);
        if (fast_decide(L, 0, P, err, parity)) return;
    }
    Ext<float> sl = ext_zero<float>(), su = ext_zero<float>();
    Ext<float> rl[K], ru[K];
    if (inreg) {
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * BLOCK;
            if (t < nt) {
                s_lo[pad(t)] = Ext<float>{__int_as_float(q[u].x), q[u].y};
                s_up[pad(t)] = Ext<float>{__int_as_float(q[u].z), q[u].w};
            }
        }
        __syncthreads();
        // the thread's run of tiles, in tile order
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (t0 + u < t1) {
                rl[u] = s_lo[pad(t0 + u)];
                ru[u] = s_up[pad(t0 + u)];
                sl = ext_add(sl, rl[u]);
                su = ext_add(su, ru[u]);
            }
    } else {
        for (int a = t0; a < t1; a += U) {
            Ext<float> vl[U], vu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = min(a + u, t1 - 1);
                vl[u] = AG[2 * t];
                vu[u] = AG[2 * t + 1];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (a + u < t1) {
                    sl = ext_add(sl, vl[u]);
                    su = ext_add(su, vu[u]);
                }
        }
    }
    Ext<float> el, eu, tl, tu;
    block_scan_both<float, BLOCK>(sl, su, el, eu, tl, tu, s_tmp);
    // per tile: the lower totals before it, the upper totals after it
    Ext<float> run = el, runu = eu;
    if (inreg) {
        // each thread overwrites only its own run's slots, read above
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (t0 + u < t1) {
                s_lo[pad(t0 + u)] = run;
                run = ext_add(run, rl[u]);
            }
#pragma unroll
        for (int u = K - 1; u >= 0; --u)
            if (t0 + u < t1) {
                s_up[pad(t0 + u)] = runu;
                runu = ext_add(runu, ru[u]);
            }
        __syncthreads();
        const gptr<int4> CR4 = (gptr<int4>)CR;
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * BLOCK;
            if (t < nt) {
                const Ext<float> a = s_lo[pad(t)], b = s_up[pad(t)];
                CR4[t] = int4{__float_as_int(a.m), a.e, __float_as_int(b.m), b.e};
            }
        }
        return;
    }
    for (int a = t0; a < t1; a += U) {
        Ext<float> vl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vl[u] = AG[2 * min(a + u, t1 - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (a + u < t1) {
                CR[2 * (a + u)] = run;
                run = ext_add(run, vl[u]);
            }
    }
    for (int b = t1 - 1; b >= t0; b -= U) {
        Ext<float> vu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vu[u] = AG[2 * max(b - u, t0) + 1];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b - u >= t0) {
                CR[2 * (b - u) + 1] = runu;
                runu = ext_add(runu, vu[u]);
            }
    }
}

template <int BLOCK, int IPT, int EPI, bool NEXT_AGG, bool BIG>
__global__ __launch_bounds__(BLOCK) void k_sweep_fast(const WorkItem* __restrict__ work,
                                                     const LineDesc* __restrict__ lines,
                                                     ProbState* __restrict__ ps,
                                                     const Ext<float>* __restrict__ agg,
                                                     double* __restrict__ partial,
                                                     const double* __restrict__ dec_partial, int parity,
                                                     Ext<float>* __restrict__ agg_next,
                                                     const Ext<float>* __restrict__ carries)
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

    const WorkItem w = work[xcd_block(blockIdx.x, gridDim.x)];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const gptr<const int> TRS = gbl(L.trs);
    const bool carried = fast_carried<BLOCK>(L);
    const bool decide = dec_partial && L.dec_part_off >= 0 && !carried;
    const int np = decide ? L.dec_nparts : 0;
    const bool multi = L.ntiles > 1 && !carried;

    // ---- loads, in the order they are consumed (the memory counter retires
    // them in issue order)
    Ext<float> af[kFastFix][2];
    double df[kFastFix];
    Ext<float> CL = ext_zero<float>(), CU = ext_zero<float>();
    if (carried) {
        CL = carries[(long long)(L.agg_base + w.tile) * 2];
        CU = carries[(long long)(L.agg_base + w.tile) * 2 + 1];
    } else {
        fast_fixed_loads<BLOCK>(L, agg, dec_partial, np, af, df);
    }
    FastTileIn<IPT> A;
    A.tg = fast_geom(L, w.tile, T, TRS[w.tile], TRS[w.tile + 1]);
    fast_tile_load<BLOCK, IPT>(A, L);
    RefAcc cl{0.f, kZeroExp}, cu{0.f, kZeroExp};
    if (multi) fast_carries<BLOCK, BIG>(L, agg, w.tile, af, cl, cu);
    const double dv = fast_decision_sum<BLOCK, BIG>(L, dec_partial, np, df);

    // ---- columns; carries and the stop decision share the next barrier
    int r0l, r0u;
    fast_tile_columns<BLOCK, IPT>(A, s_l, s_u, r0l, r0u);
    if (multi) block_total2_write<BLOCK>(cl, cu, s_f + 2 * NW, s_i + 2 * NW);
    if (decide) wave_sum_to<BLOCK>(dv, s_d);
    __syncthreads();
    if (decide && fast_decide(L, w.tile, P, block_read_sum<BLOCK>(s_d), parity)) return;
    if (multi) {
        CL = block_total_read<BLOCK>(s_f + 2 * NW, s_i + 2 * NW);
        CU = block_total_read<BLOCK>(s_f + 3 * NW, s_i + 3 * NW);
    }
    // the check operands are issued before the scan, which covers their latency
    Ext<float> uold[IPT];
    if (CHECK) fast_tile_check_loads<BLOCK, IPT>(A, L, uold);

    // ---- scan, rows, stores
    fast_tile_scan<BLOCK, IPT>(s_l, s_u, A.tg.nc, s_f);
    double red = 0.0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
    Ext<float> un[IPT];
    fast_tile_rows<BLOCK, IPT, EPI, NEXT_AGG>(A, s_l, s_u, CL, CU, r0l, r0u, uold, un, red, n1, n2);
    fast_tile_store<BLOCK, IPT>(A, L, un);

    // ---- epilogue: the tile's check partial and next-sweep aggregates
    const bool tiles = L.ntiles > 1;
    if (CHECK) wave_sum_to<BLOCK>(red, s_d);
    if (NEXT_AGG && tiles) block_total2_write<BLOCK>(n1, n2, s_f, s_i);
    if (CHECK || (NEXT_AGG && tiles)) {
        __syncthreads();
        if (threadIdx.x == 0) {
            if (CHECK) partial[L.part_base + w.tile] = block_read_sum<BLOCK>(s_d);
            if (NEXT_AGG && tiles) {
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
    const WorkItem w = work[xcd_block(blockIdx.x, gridDim.x)];
    const LineDesc L = lines[w.line];
    if (ps[L.prob].done) return;
    const gptr<const int> TRS = gbl(L.trs);
    const FastGeom tg = fast_geom(L, w.tile, T, TRS[w.tile], TRS[w.tile + 1]);
    const int nc = tg.nc;
    const int off = tg.nr;
    const gptr<const Ext<float>> BC = gbl((const Ext<float>*)L.ec) + tg.c0;
    const gptr<const Ext<float>> UC = gbl((const Ext<float>*)L.gin) + tg.c0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int j = (int)threadIdx.x + q * BLOCK - off;
        if (j >= 0 && j < nc) {
            const Ext<float> U = UC[j], B = BC[j];
            ref_add(n1, Ext<float>{U.m * B.m, U.e + B.e});
            ref_add(n2, U);
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
    const gptr<const int> TRS = gbl(tk.trs);
    const gptr<const double> LM = gbl(tk.lmass), YC = gbl(tk.yc);
    const long long r0 = min(max((long long)TRS[t], 0LL), tk.R);
    const long long r1 = min(max((long long)TRS[t + 1], r0), tk.R);
    // the tile's columns plus one neighbour on each side: the carries from
    // the other tiles then lie within the bound of the tile's own terms
    const long long c0 = max(min(max(m0 - r0, 0LL), tk.C) - 1, 0LL);
    const long long c1 = min(min(max(m1 - r1, c0), tk.C) + 1, tk.C);
    if (c1 <= c0) return;
    double mx = -__builtin_inf(), mn = __builtin_inf();
    for (long long j = c0 + threadIdx.x; j < c1; j += BLOCK) {
        const double v = LM[j];
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
        const double bound = (a - b) + 2.0 * tk.kappa * (YC[c1 - 1] - YC[c0]);
        if (!(bound <= kFastBound)) atomicOr(flags + tk.flag, 1);
    }
}

}  // namespace finom
