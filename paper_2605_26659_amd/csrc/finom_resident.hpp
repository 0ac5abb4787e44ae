// Resident-state solver for one 1D problem on the fast sweeps.
//
// Both products of an iteration use the same merge-path partition, and tile
// t of K^T phi has as rows exactly the columns of tile t of K psi and the
// other way round (section 2.2's dividing index applied to both meshes). So
// the block that owns tile t can keep every point of the tile, x and y, in
// registers for the whole solve: its state U, its mass A, B = 2^{2 c kappa}
// and its dividing index. One cooperative launch then runs Algorithm 1's
// loop; per sweep the only data that leaves the block are the tile's totals
// of the next sweep's column terms (two extended numbers) and, for the
// checking sweep, its partial marginal error. Blocks exchange them as tagged
// records (below). Every block reads the partials of all tiles and sums them
// in the same order, so all blocks take the same stop decision and run the
// same number of sweeps.
//
// A block's slots k = t + q BLOCK (thread t, q < IPT) cover the tile's
// elements as [its nc y points, its nr x points]. In the checking sweep
// (K^T phi) the x slots are columns and the y slots rows; in K psi the other
// way round. The arithmetic per element is that of k_sweep_fast; the tile
// reference exponents come from the tile's own totals. The checking sweep's
// error terms are summed in FP32 (each term capped at 2^100, far above any
// tolerance): the sum only decides when the loop stops, and the library
// confirms a stop with an FP64 check of the returned pair.
#pragma once
#include <type_traits>

#include "finom_fast.hpp"

namespace finom {

struct ResidentArgs {
    Ext<float>* UF;           // x state (in: initial, out: final)
    Ext<float>* UG;           // y state (in: initial, out: the returned one)
    const Ext<float>* Ax;     // masses
    const Ext<float>* Ay;
    const Ext<float>* Bx;     // 2^{2 c kappa}
    const Ext<float>* By;
    const int* zx;            // x among y: #{j : y_j <= x_i}
    const int* zy;            // y among x: #{i : x_i <= y_j}
    const int* trs;           // x starts of the tiles (ntiles + 1)
    long long n, m;
    int ntiles;               // tiles of the problem (at most kResidentMaxTiles)
    int T;                    // merged points per tile (at most the block's slots)
    unsigned long long* rec;  // tagged records: [ntiles][2] x totals, [ntiles][2] y totals, [ntiles] partial errors; zero at launch
    int* fail;                // set when a wait exceeds its bound
    unsigned spin_limit;      // polls before a wait gives up
    int pad2;
    ProbState* ps;
};

// ---- exchange between blocks
// After each sweep a block publishes its tile's totals (and, for the checking
// sweep, its partial error) into one of three record buffers; in the next
// sweep every block reads the records it needs from that buffer, each thread
// one record, until they carry the expected tag. The records are the whole
// synchronisation: there is no barrier counter. They are written with
// agent-scope atomic stores and read with agent-scope atomic loads, both of
// which complete at the device's coherence point, so no cache maintenance is
// needed (a release / acquire pair would write back and invalidate the L2 of
// every XCD once per block), and the writer does not wait for its stores.
//
// Tags. The k-th write of a record carries tag k & 1. A reader waiting for
// write k can only find write k - 1 or write k there: its writer makes write
// k + 1 only after reading this reader's record in the other buffer, which
// this reader writes after this read; and having once read write k - 1, the
// reader cannot see an older write. A zeroed buffer holds tag 0, as if
// written 0 times. The tag is the sign bit of the word: a total (an
// Ext<float> whose mantissa is 0 or in [1/2, 1)) keeps its mantissa's bits in
// the high half and its exponent in the low half; a partial error is a
// non-negative double. Both are restored exactly.
constexpr unsigned kResidentSpin = 1u << 22;   // default bound of a wait, in polls (~seconds)
constexpr int kResidentMaxTiles = 512;         // tiles of one problem
// The kernels' shapes, both with tiles of up to 4096 merged points. The fast
// variant runs 512 threads of 8 slots and two blocks per CU (four waves per
// SIMD, at most 128 registers). With 256 threads of 16 slots the block-wide
// steps of a sweep cost half as much per point, but two waves per SIMD leave
// too little to issue while a wave waits: measured slower. The variant with
// extended-number scans needs twice the LDS for them and runs one block of
// 512 threads per CU.
constexpr int kResidentBlock = 512, kResidentIpt = 8, kResidentWaves = 4;
constexpr int kResidentBlockGen = 512, kResidentIptGen = 8, kResidentWavesGen = 2;
constexpr int kResidentSlots = kResidentBlock * kResidentIpt;
static_assert(kResidentSlots == kResidentBlockGen * kResidentIptGen, "both variants take the same tiles");
constexpr int kResidentErrCap = 100;           // binary exponent cap of one error term

__device__ __forceinline__ unsigned long long rec_of(Ext<float> v, unsigned tag)
{
    const unsigned hi = (__float_as_uint(v.m) & 0x7FFFFFFFu) | (tag << 31);
    return ((unsigned long long)hi << 32) | (unsigned)v.e;
}

__device__ __forceinline__ Ext<float> ext_of_rec(unsigned long long w)
{
    return Ext<float>{__uint_as_float((unsigned)(w >> 32) & 0x7FFFFFFFu), (int)(unsigned)w};
}

__device__ __forceinline__ unsigned long long rec_of(double v, unsigned tag)
{
    return ((unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull) | ((unsigned long long)tag << 63);
}

__device__ __forceinline__ double double_of_rec(unsigned long long w)
{
    return __longlong_as_double((long long)(w & 0x7FFFFFFFFFFFFFFFull));
}

__device__ __forceinline__ unsigned long long rec_load(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void resident_fail(const ResidentArgs& a, int* s_flag)
{
    __hip_atomic_store(a.fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = 0;
}

// Reads a record until it carries the expected tag, starting from a first
// read w already made. The wait is bounded: it fails after a.spin_limit polls,
// or when another block's failure shows in the fail flag (checked every 64
// polls); a failure clears the block's flag, so the block leaves its loop and
// publishes no more, and every block waiting for it fails in turn.
__device__ __forceinline__ unsigned long long rec_wait(const ResidentArgs& a, const unsigned long long* p,
                                                       unsigned long long w, unsigned tag, int* s_flag)
{
    unsigned polls = 0;
    while ((unsigned)(w >> 63) != tag) {
        ++polls;
        if (polls > a.spin_limit ||
            ((polls & 63) == 0 && __hip_atomic_load(a.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            resident_fail(a, s_flag);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        w = rec_load(p);
    }
    return w;
}

// Wave 0 of a block, with wave-uniform arguments: writes the block's records
// (lane i writes word i, n words). Nothing waits for these writes.
__device__ __forceinline__ void resident_publish(int n, unsigned long long* p0, unsigned long long w0,
                                                 unsigned long long* p1, unsigned long long w1,
                                                 unsigned long long* p2, unsigned long long w2)
{
    const int lane = threadIdx.x;
    if (lane < n) {
        unsigned long long* p = lane == 0 ? p0 : lane == 1 ? p1 : p2;
        const unsigned long long w = lane == 0 ? w0 : lane == 1 ? w1 : w2;
        __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// A block's share of the carries from one buffer of records: thread t holds
// the lower totals of tiles t + r BLOCK before the block's tile, the upper
// totals of those after it, and with PART the partial errors of all of them.
struct ResidentIn {
    Ext<float> cl, cu;
    float part;
};

// own_part: this tile's partial error, which its thread takes from the
// block rather than from its record (the same value: records keep it exactly).
// A thread waits for its totals record before it requests the partial error
// published beside it (requesting both first measured slower).
template <int BLOCK, bool PART>
__device__ __forceinline__ void resident_read(const ResidentArgs& a, int tile, const unsigned long long* tot,
                                              const unsigned long long* part, unsigned tag, int* s_flag,
                                              float own_part, ResidentIn& in)
{
    constexpr int RPT = (kResidentMaxTiles + BLOCK - 1) / BLOCK;
    const int nt = a.ntiles;
    in.cl = in.cu = ext_zero<float>();
    in.part = 0.f;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int t = threadIdx.x + r * BLOCK;
        if (t < nt && t != tile) {
            const unsigned long long* pt = tot + 2 * t + (t > tile ? 1 : 0);
            const Ext<float> v = ext_of_rec(rec_wait(a, pt, rec_load(pt), tag, s_flag));
            if (t < tile) in.cl = ext_add(in.cl, v);
            else in.cu = ext_add(in.cu, v);
            if (PART) in.part += (float)double_of_rec(rec_wait(a, part + t, rec_load(part + t), tag, s_flag));
        }
        if (PART && t == tile) in.part += own_part;
    }
}

// ---- block totals
// The per-wave parts of a block's two extended totals and, with D, of an FP32
// sum, as one interleaved sequence of DPP steps so that the independent
// reductions fill each other's wait states; lane 0 of each wave leaves them in
// LDS (each extended part normalised) for block_totals_read / block_refs_read
// after a barrier. The order of every sum is fixed.
template <int C, int R>
__device__ __forceinline__ float dpp_sum_src(float v)
{
    if constexpr (C == 0x142 || C == 0x143) return dpp_bc_f<C, R>(v);
    else return dpp_f<C, R>(v);
}

template <int C, int R, bool D>
__device__ __forceinline__ void tot_step1(int& ra, int& rb, float& d)
{
    ra = dpp_max_i<C, R>(ra);
    rb = dpp_max_i<C, R>(rb);
    if (D) d += dpp_sum_src<C, R>(d);
}

template <int C, int R>
__device__ __forceinline__ void tot_step2(float& sa, float& sb)
{
    sa += dpp_sum_src<C, R>(sa);
    sb += dpp_sum_src<C, R>(sb);
}

template <int BLOCK, bool D>
__device__ __forceinline__ void block_totals_write(RefAcc a, RefAcc b, float d, float* s_f, int* s_i, float* s_e)
{
    constexpr int NW = BLOCK / kWave;
    int ra = a.r, rb = b.r;
    tot_step1<0x111, 0xF, D>(ra, rb, d);   // row_shr:1
    tot_step1<0x112, 0xF, D>(ra, rb, d);   // row_shr:2
    tot_step1<0x114, 0xF, D>(ra, rb, d);   // row_shr:4
    tot_step1<0x118, 0xF, D>(ra, rb, d);   // row_shr:8
    tot_step1<0x142, 0xA, D>(ra, rb, d);   // row_bcast:15
    tot_step1<0x143, 0xC, D>(ra, rb, d);   // row_bcast:31
    ra = __builtin_amdgcn_readlane(ra, kWave - 1);
    rb = __builtin_amdgcn_readlane(rb, kWave - 1);
    float sa = ldexp_m(a.s, a.r - ra), sb = ldexp_m(b.s, b.r - rb);
    tot_step2<0x111, 0xF>(sa, sb);
    tot_step2<0x112, 0xF>(sa, sb);
    tot_step2<0x114, 0xF>(sa, sb);
    tot_step2<0x118, 0xF>(sa, sb);
    tot_step2<0x142, 0xA>(sa, sb);
    tot_step2<0x143, 0xC>(sa, sb);
    sa = readlane_f(sa, kWave - 1);
    sb = readlane_f(sb, kWave - 1);
    if (D) d = readlane_f(d, kWave - 1);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int wid = threadIdx.x / kWave;
        s_f[wid] = __builtin_amdgcn_frexp_mantf(sa);
        s_i[wid] = sa > 0.f ? ra + __builtin_amdgcn_frexp_expf(sa) : kZeroExp;
        s_f[NW + wid] = __builtin_amdgcn_frexp_mantf(sb);
        s_i[NW + wid] = sb > 0.f ? rb + __builtin_amdgcn_frexp_expf(sb) : kZeroExp;
        if (D) s_e[wid] = d;
    }
}

// The block's totals from the per-wave parts that block_totals_write left in
// LDS: lane w of every wave reads wave w's parts, and the waves' parts are
// combined across lanes (largest exponent, then the sum in a fixed order), so
// every thread gets the same results.
template <int BLOCK, bool D>
__device__ __forceinline__ void block_totals_read(const float* s_f, const int* s_i, const float* s_e, Ext<float>& ta,
                                                  Ext<float>& tb, float& td)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = lane & (NW - 1);
    const bool mine = lane < NW;
    const float fa = s_f[w], fb = s_f[NW + w];
    const int ea = mine ? s_i[w] : kZeroExp, eb = mine ? s_i[NW + w] : kZeroExp;
    const float d = D && mine ? s_e[w] : 0.f;
    const int ra = first_lanes_max_i<NW>(ea), rb = first_lanes_max_i<NW>(eb);
    const float sa = first_lanes_sum_f<NW>(mine ? ldexp_m(fa, ea - ra) : 0.f);
    const float sb = first_lanes_sum_f<NW>(mine ? ldexp_m(fb, eb - rb) : 0.f);
    ta = ext_norm(Ext<float>{sa, ra});
    tb = ext_norm(Ext<float>{sb, rb});
    if (D) td = first_lanes_sum_f<NW>(d);
}

// Only the references of the next sweep's column terms: the largest exponent
// of the waves' (normalised) parts of the two totals. Every term of the tile
// is below 2^ref and the tile's total below 2^(ref + 3).
template <int BLOCK>
__device__ __forceinline__ void block_refs_read(const int* s_i, int& ra, int& rb)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = lane & (NW - 1);
    const bool mine = lane < NW;
    ra = first_lanes_max_i<NW>(mine ? s_i[w] : kZeroExp);
    rb = first_lanes_max_i<NW>(mine ? s_i[NW + w] : kZeroExp);
}

// Exclusive prefix and exclusive suffix (thread order) of extended values over
// the block: wave scans, then the waves' totals combined across lanes (lane j
// of every wave reads wave j's total) rather than one after another.
template <int BLOCK>
__device__ __forceinline__ void block_scan_ext(Ext<float> vl, Ext<float> vu, Ext<float>& excl_l, Ext<float>& excl_u,
                                               Ext<float>* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    static_assert(NW == 8, "three DPP steps combine eight waves");
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const Ext<float> il = wave_incl_prefix(vl);
    const Ext<float> iu = wave_incl_suffix(vu);
    if (lane == kWave - 1) s_tmp[wid] = il;
    if (lane == 0) s_tmp[NW + wid] = iu;
    __syncthreads();
    const int j = lane & (NW - 1);
    Ext<float> a = s_tmp[j], b = s_tmp[NW + j];
    if (!(lane < NW && j < wid)) a = ext_zero<float>();
    if (!(lane < NW && j > wid)) b = ext_zero<float>();
    a = ext_add(a, dpp_ext<0x111>(a));   // row_shr:1
    b = ext_add(b, dpp_ext<0x111>(b));
    a = ext_add(a, dpp_ext<0x112>(a));   // row_shr:2
    b = ext_add(b, dpp_ext<0x112>(b));
    a = ext_add(a, dpp_ext<0x114>(a));   // row_shr:4
    b = ext_add(b, dpp_ext<0x114>(b));
    excl_l = ext_add(readlane_ext(a, NW - 1), dpp_ext<0x138>(il));   // wave_shr:1
    excl_u = ext_add(dpp_ext<0x130>(iu), readlane_ext(b, NW - 1));   // wave_shl:1
}

// Exclusive prefix (s_l) and inclusive suffix (s_u) of a tile's extended
// column terms in place, thread t owning columns [t IPT, t IPT + IPT), and the
// total before the end at s_l[BLOCK IPT]; the caller has passed a barrier
// since the columns were written, and passes another before the results are
// read. Terms past ncol count as zero.
template <int BLOCK, int IPT>
__device__ __forceinline__ void resident_scan_ext(Ext<float>* s_l, Ext<float>* s_u, int nc, Ext<float>* s_tmp)
{
    Ext<float> vl[IPT], vu[IPT];
    const int base = threadIdx.x * IPT;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const bool live = base + q < nc;
        vl[q] = live ? s_l[base + q] : ext_zero<float>();
        vu[q] = live ? s_u[base + q] : ext_zero<float>();
    }
    Ext<float> sl = ext_zero<float>(), su = ext_zero<float>();
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        sl = ext_add(sl, vl[q]);
        su = ext_add(su, vu[q]);
    }
    Ext<float> el, eu;
    block_scan_ext<BLOCK>(sl, su, el, eu, s_tmp);
    // every chunk was read before the scan's barrier: overwrite in place
    Ext<float> run = el;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const Ext<float> t = vl[q];
        s_l[base + q] = run;
        run = ext_add(run, t);
    }
    Ext<float> runu = eu;
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) {
        runu = ext_add(runu, vu[q]);
        s_u[base + q] = runu;
    }
    if (threadIdx.x == BLOCK - 1) {
        s_l[BLOCK * IPT] = run;
        s_u[BLOCK * IPT] = ext_zero<float>();
    }
}

// The local half of a sweep: the column terms (slots [c_first, c_first +
// ncol), column index k - c_first) to LDS, and their in-tile scan. Needs
// nothing from other blocks. On the fast sweeps' tiles the terms are plain
// FP32 against the references r0l, r0u (no term above 2^r); with GEN they are
// extended numbers, for tiles whose terms span more than FP32's range. The
// scan's results are visible after the caller's next barrier.
template <int BLOCK, int IPT, bool GEN, typename Term>
__device__ __forceinline__ void resident_columns(int c_first, int ncol, int r0l, int r0u, const Ext<float>* U,
                                                 const Ext<float>* B, Term* s_l, Term* s_u, float* s_f,
                                                 Ext<float>* s_tmp)
{
    // Opaque copies of the slot bounds and the thread index: without them the
    // compiler hoists every slot's masks and LDS offsets of both sweeps out of
    // the solver loop and runs out of registers. (Per-lane tests: a
    // wave-uniform test per slot runs more scalar instructions than it saves.)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    asm volatile("" : "+s"(c_first), "+s"(ncol));
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = tid + q * BLOCK - c_first;
        if ((unsigned)k < (unsigned)ncol) {
            if constexpr (GEN) {
                s_l[k] = Ext<float>{U[q].m * B[q].m, U[q].e + B[q].e};
                s_u[k] = U[q];
            } else {
                s_l[k] = ldexp_m(U[q].m * B[q].m, U[q].e + B[q].e - r0l);
                s_u[k] = ldexp_m(U[q].m, U[q].e - r0u);
            }
        }
    }
    __syncthreads();
    if constexpr (GEN) resident_scan_ext<BLOCK, IPT>(s_l, s_u, ncol, s_tmp);
    else fast_tile_scan<BLOCK, IPT, false>(s_l, s_u, ncol, s_f);
}

// The rows of a sweep (slots [r_first, r_first + nrow), dividing index Z as a
// column index of this tile) once the carries are known: replaces the rows'
// states and leaves the per-wave parts of the next sweep's tile totals (and
// for CHECK of the tile's partial error) in the block's LDS slots, visible on
// return. CHECK also keeps the rows' old states in `old` (the pair the loop
// head returns when it stops).
template <int BLOCK, int IPT, bool CHECK, bool GEN, typename Term>
__device__ __forceinline__ void resident_rows(const Ext<float> CL, const Ext<float> CU, int ncol, int r_first,
                                              int nrow, int r0l, int r0u, Ext<float>* U, const Ext<float>* s_a,
                                              const Ext<float>* B, const unsigned short* s_z, Ext<float>* old,
                                              const Term* s_l, const Term* s_u, float* s_f, int* s_i, float* s_e)
{
    constexpr int NW = BLOCK / kWave;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    asm volatile("" : "+s"(ncol), "+s"(r_first), "+s"(nrow));
    const int rl = max(r0l, CL.e), ru = max(r0u, CU.e);
    const float cl_rel = ldexp_m(CL.m, CL.e - rl), cu_rel = ldexp_m(CU.m, CU.e - ru);
    const int shl = r0l - rl, shu = r0u - ru;
    // the in-tile sums rescaled by 2^shl <= 1 in the same fused operation as
    // the carry's addition (exact products; where 2^shl is below FP32's normal
    // range the in-tile part is below 2^-126 of the carry, which is >= 1/2)
    const float scl = shl < -126 ? 0.f : ldexp_m(1.f, shl);
    const float scu = shu < -126 ? 0.f : ldexp_m(1.f, shu);
    float red = 0.f;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
    // every slot's scan values first (unconditional: each slot's dividing
    // index is within the scans), so that no row waits on its own LDS reads
    Term sl[IPT], su[IPT];
    Ext<float> A[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int z = s_z[tid + q * BLOCK];
        sl[q] = s_l[z];
        su[q] = s_u[z];
        A[q] = s_a[tid + q * BLOCK];
    }
    auto row = [&](int q) {
        const Ext<float> Aq = A[q];
        Ext<float> W;
        if constexpr (GEN) {
            const Ext<float> L = ext_add(CL, sl[q]);
            const Ext<float> R = ext_add(su[q], CU);
            W = ext_add(L, Ext<float>{R.m * B[q].m, R.e + B[q].e});
        } else {
            const float pm = __builtin_fmaf(sl[q], scl, cl_rel);
            const float qm = __builtin_fmaf(su[q], scu, cu_rel);
            W = ext_add(Ext<float>{pm, rl}, Ext<float>{qm * B[q].m, ru + B[q].e});
        }
        const Ext<float> Un = ext_norm(Ext<float>{Aq.m * __builtin_amdgcn_rcpf(W.m), Aq.e - W.e});
        if (CHECK) {
            const int ep = U[q].e + W.e;
            const int re = max(ep, Aq.e);
            const float d = __builtin_fmaf(ldexp_m(U[q].m, ep - re), W.m, -ldexp_m(Aq.m, Aq.e - re));
            red += ldexp_m(fabsf(d), min(re, kResidentErrCap));
            old[q] = U[q];
        }
        U[q] = Un;
        if constexpr (GEN) {
            // totals of terms of any range: against the largest so far
            const Ext<float> t1 = ext_add(Ext<float>{n1.s, n1.r}, Ext<float>{Un.m * B[q].m, Un.e + B[q].e});
            const Ext<float> t2 = ext_add(Ext<float>{n2.s, n2.r}, Un);
            n1 = RefAcc{t1.m, t1.e};
            n2 = RefAcc{t2.m, t2.e};
        } else {
            ref_add(n1, Ext<float>{Un.m * B[q].m, Un.e + B[q].e});
            ref_add(n2, Un);
        }
    };
#pragma unroll
    for (int q = 0; q < IPT; ++q)
        if ((unsigned)(tid + q * BLOCK - r_first) < (unsigned)nrow) row(q);
    block_totals_write<BLOCK, CHECK>(n1, n2, red, s_f + 4 * NW, s_i + 4 * NW, s_e + NW);
    __syncthreads();
}

// MINW: waves per SIMD the kernel must allow (two blocks of 512 per CU need
// four, so at most 128 registers per lane).
// The block's LDS: the tile's column scans, per-wave partial results, the
// slots' masses and their dividing indices (as rows, within the tile).
template <int BLOCK, int IPT, bool GEN>
struct ResidentLds {
    static constexpr int T = BLOCK * IPT;
    static constexpr int NW = BLOCK / kWave;
    using Term = typename std::conditional<GEN, Ext<float>, float>::type;
    __align__(16) Term l[T + 4];
    __align__(16) Term u[T + 4];
    Ext<float> tmp[GEN ? 2 * NW : 1];
    float f[6 * NW];
    int i[6 * NW];
    float e[2 * NW];   // per-wave error parts: [0, NW) of the carries, [NW, 2 NW) of the rows
    Ext<float> a[T];
    unsigned short z[T];
    float pe;   // the tile's partial error of the last checking sweep
    int flag;   // 0 once a wait of this block has failed
};

// Solves one problem's tile to the end of its loop (every tile of the problem
// must be running on some block of the grid at the same time).
template <int BLOCK, int IPT, bool GEN>
__device__ __forceinline__ void resident_solve(const ResidentArgs& a, const int tile,
                                               ResidentLds<BLOCK, IPT, GEN>& L)
{
    static_assert(IPT % 4 == 0, "chunks are read as float4");
    constexpr int NW = BLOCK / kWave;
    using Term = typename ResidentLds<BLOCK, IPT, GEN>::Term;
    Term* const s_l = L.l;
    Term* const s_u = L.u;
    Ext<float>* const s_tmp = L.tmp;
    float* const s_f = L.f;
    int* const s_i = L.i;
    float* const s_e = L.e;
    Ext<float>* const s_a = L.a;
    unsigned short* const s_z = L.z;
    int& s_flag = L.flag;
    const int T = a.T;
    const int nt = a.ntiles;
    // the loop's bounds and its first iteration (0, or where a stop that the
    // FP64 check rejected left it), read before this block publishes anything,
    // so before tile 0 can record the stop
    const long long itr_max = a.ps->itr_max;
    const double tol = a.ps->tol;
    long long l = a.ps->iters;
    unsigned long long* rec_x = a.rec;                       // totals of the x points' column terms
    unsigned long long* rec_y = a.rec + 2 * (size_t)nt;      // totals of the y points' column terms
    unsigned long long* rec_p = a.rec + 4 * (size_t)nt;      // partial errors of the checking sweep
    // the tile: x points [r0, r0 + nr), y points [c0, c0 + nc)
    const long long m0 = (long long)tile * T;
    const long long m1 = min(m0 + (long long)T, a.n + a.m);
    const long long r0 = min(max((long long)a.trs[tile], 0LL), a.n);
    const long long r1 = min(max((long long)a.trs[tile + 1], r0), a.n);
    const long long c0 = min(max(m0 - r0, 0LL), a.m);
    long long c1 = min(max(m1 - r1, c0), a.m);
    if (c1 - c0 > T) c1 = c0 + T;
    // block-uniform (scalar registers, whatever memory the bounds came from)
    const int nc = __builtin_amdgcn_readfirstlane((int)(c1 - c0));
    const int nr = __builtin_amdgcn_readfirstlane((int)min(r1 - r0, (long long)(T - nc)));

    // per slot: state and B in registers; mass and, as a row, its dividing
    // index as a column index of this tile (y rows over the tile's x, x rows
    // over its y; at most T, so 16 bits) in LDS
    Ext<float> U[IPT], B[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        const bool isy = k < nc;
        const long long jy = min(c0 + (long long)min(k, max(nc - 1, 0)), a.m - 1);
        const long long jx = min(r0 + (long long)min(max(k - nc, 0), max(nr - 1, 0)), a.n - 1);
        U[q] = isy ? a.UG[jy] : a.UF[jx];
        s_a[k] = isy ? a.Ay[jy] : a.Ax[jx];
        B[q] = isy ? a.By[jy] : a.Bx[jx];
        const long long z = isy ? (long long)a.zy[jy] - r0 : (long long)a.zx[jx] - c0;
        s_z[k] = (unsigned short)min(max(z, 0LL), (long long)(isy ? nr : nc));
    }

    // The loop. Each sweep: its columns and their scan (local, done while the
    // other blocks finish the previous sweep), the previous sweep's records
    // and the carries, the rows, publication. Two blocks share a CU, and the
    // SIMDs favour the older block's waves: a block raises its waves' issue
    // priority from its records to its publication, so that a block on the
    // critical path is not held back by its neighbour's column work.
    // Per sweep the block passes four barriers: columns written, scan's wave
    // totals, scan and carry parts written, rows' parts written. Every thread
    // takes the next sweep's column references from the rows' parts; wave 0
    // alone forms the tile's totals and partial error and publishes them.
    if (threadIdx.x == 0) s_flag = 1;
    // the first sweep's column totals (x points) from the initial state
    int refl, refu;
    {
        RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int k = threadIdx.x + q * BLOCK - nc;
            if (k >= 0 && k < nr) {
                if constexpr (GEN) {
                    const Ext<float> t1 = ext_add(Ext<float>{n1.s, n1.r}, Ext<float>{U[q].m * B[q].m, U[q].e + B[q].e});
                    const Ext<float> t2 = ext_add(Ext<float>{n2.s, n2.r}, U[q]);
                    n1 = RefAcc{t1.m, t1.e};
                    n2 = RefAcc{t2.m, t2.e};
                } else {
                    ref_add(n1, Ext<float>{U[q].m * B[q].m, U[q].e + B[q].e});
                    ref_add(n2, U[q]);
                }
            }
        }
        block_totals_write<BLOCK, false>(n1, n2, 0.f, s_f + 4 * NW, s_i + 4 * NW, s_e);
        __syncthreads();
        block_refs_read<BLOCK>(s_i + 4 * NW, refl, refu);
        if (threadIdx.x < kWave) {
            Ext<float> own_l, own_u;
            float unused;
            block_totals_read<BLOCK, false>(s_f + 4 * NW, s_i + 4 * NW, s_e, own_l, own_u, unused);
            resident_publish(2, rec_x + 2 * tile, rec_of(own_l, 1u), rec_x + 2 * tile + 1, rec_of(own_u, 1u),
                             nullptr, 0);
        }
    }

    long long it = 0;   // iterations of this launch: the records' tags count from the launch
    float err = 0.f;
    bool ok = true;
    ResidentIn in;
    Ext<float> uold[IPT];   // the y points' states the loop head checks
    for (;;) {
        // ---- K^T phi with the marginal check: columns x, rows y
        resident_columns<BLOCK, IPT, GEN>(nc, nr, refl, refu, U, B, s_l, s_u, s_f, s_tmp);
        const int rxl = refl, rxu = refu;
        // records of this iteration's sweeps: write it + 1 of their buffers
        const unsigned tag = (unsigned)((it + 1) & 1);
        __builtin_amdgcn_s_setprio(2);
        resident_read<BLOCK, false>(a, tile, rec_x, nullptr, tag, &s_flag, 0.f, in);
        block_totals_write<BLOCK, false>(RefAcc{in.cl.m, in.cl.e}, RefAcc{in.cu.m, in.cu.e}, 0.f, s_f + 2 * NW,
                                         s_i + 2 * NW, s_e);
        __syncthreads();
        ok = s_flag != 0;
        if (!ok) break;
        Ext<float> CL, CU;
        float pe;
        block_totals_read<BLOCK, false>(s_f + 2 * NW, s_i + 2 * NW, s_e, CL, CU, pe);
        resident_rows<BLOCK, IPT, true, GEN>(CL, CU, nr, 0, nc, rxl, rxu, U, s_a, B, s_z, uold, s_l, s_u, s_f, s_i, s_e);
        block_refs_read<BLOCK>(s_i + 4 * NW, refl, refu);
        if (threadIdx.x < kWave) {
            Ext<float> own_l, own_u;
            block_totals_read<BLOCK, true>(s_f + 4 * NW, s_i + 4 * NW, s_e + NW, own_l, own_u, pe);
            resident_publish(3, rec_y + 2 * tile, rec_of(own_l, tag), rec_y + 2 * tile + 1, rec_of(own_u, tag),
                             rec_p + tile, rec_of((double)pe, tag));
            if (threadIdx.x == 0) L.pe = pe;   // read by thread `tile` after the next barriers
        }
        __builtin_amdgcn_s_setprio(0);
        // ---- K psi: its columns (y) while the others finish, then the loop
        // head (every block sums the partials in the same order). No barrier
        // is needed before the columns: the scans were last read before the
        // rows' barrier, and the LDS read since then is written again only
        // after the column phase's barriers.
        resident_columns<BLOCK, IPT, GEN>(0, nc, refl, refu, U, B, s_l, s_u, s_f, s_tmp);
        const int ryl = refl, ryu = refu;
        __builtin_amdgcn_s_setprio(2);
        resident_read<BLOCK, true>(a, tile, rec_y, rec_p, tag, &s_flag, L.pe, in);
        block_totals_write<BLOCK, true>(RefAcc{in.cl.m, in.cl.e}, RefAcc{in.cu.m, in.cu.e}, in.part, s_f + 2 * NW,
                                        s_i + 2 * NW, s_e);
        __syncthreads();
        ok = s_flag != 0;
        if (!ok) break;
        block_totals_read<BLOCK, true>(s_f + 2 * NW, s_i + 2 * NW, s_e, CL, CU, err);
        if (l >= itr_max || !((double)err > tol)) {
            // the returned psi: the states the loop head checked
#pragma unroll
            for (int q = 0; q < IPT; ++q) {
                const int k = threadIdx.x + q * BLOCK;
                if (k < nc) a.UG[c0 + k] = uold[q];
            }
            break;
        }
        // ---- K psi: rows x
        resident_rows<BLOCK, IPT, false, GEN>(CL, CU, nc, nc, nr, ryl, ryu, U, s_a, B, s_z, nullptr, s_l, s_u, s_f, s_i,
                                         s_e);
        block_refs_read<BLOCK>(s_i + 4 * NW, refl, refu);
        if (threadIdx.x < kWave) {
            Ext<float> own_l, own_u;
            block_totals_read<BLOCK, false>(s_f + 4 * NW, s_i + 4 * NW, s_e, own_l, own_u, pe);
            resident_publish(2, rec_x + 2 * tile, rec_of(own_l, tag ^ 1u), rec_x + 2 * tile + 1,
                             rec_of(own_u, tag ^ 1u), nullptr, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        ++l;
        ++it;
    }
    // the returned pair: the current phi (and the psi the loop head checked,
    // written above)
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = threadIdx.x + q * BLOCK;
        if (k >= nc && k < nc + nr) a.UF[r0 + (k - nc)] = U[q];
    }
    if (tile == 0 && threadIdx.x == 0) {
        ProbState* P = a.ps;
        P->err = (double)err;
        P->iters = l;
        P->converged = (ok && (double)err <= tol) ? 1 : 0;
        P->status = (!(err == err) || err == __builtin_inff()) ? 1 : 0;
        P->done = 1;
    }
}

// One problem, one tile per block.
template <int BLOCK, int IPT, int MINW, bool GEN>
__global__ __launch_bounds__(BLOCK, MINW) void k_resident_1d(ResidentArgs a)
{
    __shared__ ResidentLds<BLOCK, IPT, GEN> L;
    resident_solve<BLOCK, IPT, GEN>(a, blockIdx.x, L);
}

// Many problems on one persistent grid. Blocks take the problems' tiles in
// order from a counter (problem p owns the tiles [first[p], first[p + 1]))
// and solve each to the end of its problem's loop before taking another. A
// block waits only for tiles of its own problem; those are handed out before
// any later problem's, and every problem has at most as many tiles as the
// grid has blocks, so the blocks of earlier problems, which wait for nothing
// that has not been handed out, finish and take the missing tiles.
static_assert(sizeof(ResidentArgs) % 4 == 0, "read as 32-bit words");

struct ResidentBatch {
    const ResidentArgs* probs;
    const int* first;         // nprob + 1 tile offsets
    int nprob;
    int total;                // first[nprob]
    int* next;                // tile counter, zero at launch
};

template <int BLOCK, int IPT, int MINW, bool GEN>
__global__ __launch_bounds__(BLOCK, MINW) void k_resident_batch(ResidentBatch b)
{
    __shared__ ResidentLds<BLOCK, IPT, GEN> L;
    __shared__ int s_g;
    for (;;) {
        __syncthreads();   // the previous tile's LDS is no longer read
        if (threadIdx.x == 0) s_g = __hip_atomic_fetch_add(b.next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        // block-uniform values in scalar registers, as in the one-problem kernel
        const int g = __builtin_amdgcn_readfirstlane(s_g);
        if (g >= b.total) break;
        int lo = 0, hi = b.nprob - 1;   // the last problem whose first tile is at most g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (__builtin_amdgcn_readfirstlane(b.first[mid]) <= g) lo = mid;
            else hi = mid - 1;
        }
        ResidentArgs a;
        const unsigned* src = reinterpret_cast<const unsigned*>(b.probs + lo);
        unsigned* dst = reinterpret_cast<unsigned*>(&a);
#pragma unroll
        for (int w = 0; w < (int)(sizeof(ResidentArgs) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
        resident_solve<BLOCK, IPT, GEN>(a, __builtin_amdgcn_readfirstlane(g - b.first[lo]), L);
    }
}

}  // namespace finom

namespace finom {

// Threads per block of the resident kernels (the fast and the extended variant).
constexpr int resident_block(bool gen) { return gen ? kResidentBlockGen : kResidentBlock; }

}  // namespace finom
