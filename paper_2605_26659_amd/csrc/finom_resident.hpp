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
// checking sweep, its partial marginal error. Blocks exchange them through a
// grid barrier (an agent-scope counter). Every block reads all totals and
// partials in the same order, so all blocks compute the same carries and take
// the same stop decision, and every block runs the same number of barriers.
//
// A block's slots k = t + q BLOCK (thread t, q < IPT) cover the tile's
// elements as [its nc y points, its nr x points]. In the checking sweep
// (K^T phi) the x slots are columns and the y slots rows; in K psi the other
// way round. The arithmetic per element is that of k_sweep_fast; the tile
// reference exponents come from the tile's own totals.
#pragma once
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
    int ntiles;               // at most the block size
    int pad;
    unsigned long long* rec;  // records: [ntiles][2] x totals, [ntiles][2] y totals, [ntiles] partial errors
    unsigned* counter;        // barrier counters (top, then one per group of blocks), zero at launch
    int* fail;                // set when a wait exceeds its bound
    unsigned spin_limit;      // polls before a wait gives up
    ProbState* ps;
};

// ---- exchange between blocks
// After each sweep every block publishes its tile's totals (and, for the
// checking sweep, its partial error) into one of three record buffers and
// counts itself in at a grid barrier; after the barrier every block reads all
// records of the buffer. Records are written with agent-scope exchanges whose
// completion the writer waits for before it arrives, and read with
// agent-scope atomic loads: both complete at the device's coherence point,
// so no cache maintenance is needed (a release / acquire pair would write
// back and invalidate the L2 of every XCD once per block). The barrier
// counts in two levels (a counter per group of blocks, the last block of a
// group counts the group in at the top counter) to spread the atomic traffic;
// every block polls the top counter. A buffer is written again only after a
// later barrier, which every block reaches only after it has read the buffer.
constexpr unsigned kResidentSpin = 1u << 22;   // default bound of a wait, in polls (~seconds)
constexpr int kResidentGroup = 16;             // blocks per first-level counter
constexpr int kResidentLine = 64;              // counters 256 bytes apart

__device__ __forceinline__ unsigned long long u64_of(Ext<float> v)
{
    unsigned long long r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

__device__ __forceinline__ Ext<float> ext_of(unsigned long long w)
{
    Ext<float> r;
    __builtin_memcpy(&r, &w, sizeof(r));
    return r;
}

__device__ __forceinline__ unsigned long long rec_load(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 of a block: writes n words and waits until the writes have
// completed at the coherence point.
__device__ __forceinline__ void resident_publish(unsigned long long* p0, unsigned long long v0,
                                                 unsigned long long* p1, unsigned long long v1,
                                                 unsigned long long* p2, unsigned long long v2)
{
    unsigned long long w = __hip_atomic_exchange(p0, v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w ^= __hip_atomic_exchange(p1, v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p2) w ^= __hip_atomic_exchange(p2, v2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" : : "v"((unsigned)w) : "memory");
}

// The grid barrier in two halves, so that a block can do its local work
// between them. Thread 0 arrives after its publication has completed; every
// block arrives and waits the same number of times. resident_wait returns
// false when the wait exceeded its bound or another block reported that;
// then every later wait returns false at once.
__device__ __forceinline__ void resident_arrive(const ResidentArgs& a, unsigned gen)
{
    const unsigned nb = gridDim.x;
    const unsigned g = blockIdx.x / kResidentGroup;
    const unsigned gsz = min((unsigned)kResidentGroup, nb - g * kResidentGroup);
    unsigned* grp = a.counter + kResidentLine * (1 + g);
    const unsigned old = __hip_atomic_fetch_add(grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == gen * gsz - 1) __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool resident_wait(const ResidentArgs& a, unsigned gen, int* s_flag)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned G = (gridDim.x + kResidentGroup - 1) / kResidentGroup;
        unsigned polls = 0;
        while (__hip_atomic_load(a.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen * G) {
            if (__hip_atomic_load(a.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++polls > a.spin_limit) {
                __hip_atomic_store(a.fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// A block's share of the carries from one buffer of records: thread t holds
// tile t's lower total when t < tile, its upper total when t > tile, and with
// PART tile t's partial error.
struct ResidentIn {
    Ext<float> cl, cu;
    double part;
};

template <bool PART>
__device__ __forceinline__ void resident_read(const ResidentArgs& a, const unsigned long long* tot,
                                              const unsigned long long* part, ResidentIn& in)
{
    const int t = threadIdx.x, tile = blockIdx.x, nt = a.ntiles;
    in.cl = in.cu = ext_zero<float>();
    in.part = 0.0;
    if (t < nt) {
        if (t < tile) in.cl = ext_of(rec_load(tot + 2 * t));
        if (t > tile) in.cu = ext_of(rec_load(tot + 2 * t + 1));
        if (PART) {
            const unsigned long long w = rec_load(part + t);
            __builtin_memcpy(&in.part, &w, sizeof(w));
        }
    }
}

// The local half of a sweep: the column terms (slots [c_first, c_first +
// ncol), column index k - c_first) against the tile's own totals, to LDS, and
// their in-tile scan. Needs nothing from other blocks.
template <int BLOCK, int IPT>
__device__ __forceinline__ void resident_columns(int c_first, int ncol, int r0l, int r0u, const Ext<float>* U,
                                                 const Ext<float>* B, float* s_l, float* s_u, float* s_f)
{
    // Opaque copies of the slot bounds and the thread index: without them the
    // compiler hoists every slot's masks and LDS offsets of both sweeps out of
    // the solver loop and runs out of registers.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    asm volatile("" : "+s"(c_first), "+s"(ncol));
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = tid + q * BLOCK - c_first;
        if (k >= 0 && k < ncol) {
            s_l[k] = ldexp_m(U[q].m * B[q].m, U[q].e + B[q].e - r0l);
            s_u[k] = ldexp_m(U[q].m, U[q].e - r0u);
        }
    }
    __syncthreads();
    fast_tile_scan<BLOCK, IPT>(s_l, s_u, ncol, s_f);
}

// The rows of a sweep (slots [r_first, r_first + nrow), dividing index Z as a
// column index of this tile) once the carries are known: replaces the rows'
// states and leaves the next sweep's tile totals (and for CHECK the tile's
// partial error) in the block's LDS slots. CHECK also keeps the rows' old
// states in `old` (the pair the loop head returns when it stops).
template <int BLOCK, int IPT, bool CHECK>
__device__ __forceinline__ void resident_rows(const ResidentIn& in, int ncol, int r_first, int nrow, int r0l,
                                              int r0u, Ext<float>* U, const Ext<float>* s_a, const Ext<float>* B,
                                              const unsigned short* s_z, Ext<float>* old, const float* s_l,
                                              const float* s_u, float* s_f, int* s_i, double* s_d)
{
    constexpr int NW = BLOCK / kWave;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    asm volatile("" : "+s"(ncol), "+s"(r_first), "+s"(nrow));
    block_total2_write<BLOCK>(RefAcc{in.cl.m, in.cl.e}, RefAcc{in.cu.m, in.cu.e}, s_f + 2 * NW, s_i + 2 * NW);
    __syncthreads();
    const Ext<float> CL = block_total_read<BLOCK>(s_f + 2 * NW, s_i + 2 * NW);
    const Ext<float> CU = block_total_read<BLOCK>(s_f + 3 * NW, s_i + 3 * NW);
    const int rl = max(r0l, CL.e), ru = max(r0u, CU.e);
    const float cl_rel = ldexp_m(CL.m, CL.e - rl), cu_rel = ldexp_m(CU.m, CU.e - ru);
    const int shl = r0l - rl, shu = r0u - ru;
    double red = 0.0;
    RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int k = tid + q * BLOCK - r_first;
        if (k >= 0 && k < nrow) {
            const int z = s_z[tid + q * BLOCK];
            const Ext<float> Aq = s_a[tid + q * BLOCK];
            const float pm = cl_rel + ldexp_m(s_l[z], shl);
            const float qm = ldexp_m(s_u[z], shu) + cu_rel;
            const Ext<float> W = ext_add(Ext<float>{pm, rl}, Ext<float>{qm * B[q].m, ru + B[q].e});
            const Ext<float> Un = ext_norm(Ext<float>{Aq.m * __builtin_amdgcn_rcpf(W.m), Aq.e - W.e});
            if (CHECK) {
                const int ep = U[q].e + W.e;
                const int re = max(ep, Aq.e);
                const float d = __builtin_fmaf(ldexp_m(U[q].m, ep - re), W.m, -ldexp_m(Aq.m, Aq.e - re));
                red += __builtin_amdgcn_ldexp((double)fabsf(d), re);
                old[q] = U[q];
            }
            U[q] = Un;
            ref_add(n1, Ext<float>{Un.m * B[q].m, Un.e + B[q].e});
            ref_add(n2, Un);
        }
    }
    if (CHECK) wave_sum_to<BLOCK>(red, s_d);
    block_total2_write<BLOCK>(n1, n2, s_f + 4 * NW, s_i + 4 * NW);
    __syncthreads();
}

// MINW: waves per SIMD the kernel must allow (two blocks of 512 per CU need
// four, so at most 128 registers per lane).
template <int BLOCK, int IPT, int MINW>
__global__ __launch_bounds__(BLOCK, MINW) void k_resident_1d(ResidentArgs a)
{
    static_assert(IPT % 4 == 0, "chunks are read as float4");
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ __align__(16) float s_l[T + 4];
    __shared__ __align__(16) float s_u[T + 4];
    __shared__ float s_f[6 * NW];
    __shared__ int s_i[6 * NW];
    __shared__ double s_d[NW];
    __shared__ Ext<float> s_a[T];           // the slots' masses
    __shared__ unsigned short s_z[T];       // the slots' dividing indices (as rows), within the tile

    const int tile = blockIdx.x;
    const int nt = a.ntiles;
    unsigned long long* rec_x = a.rec;                       // totals of the x points' column terms
    unsigned long long* rec_y = a.rec + 2 * (size_t)nt;      // totals of the y points' column terms
    unsigned long long* rec_p = a.rec + 4 * (size_t)nt;      // partial errors of the checking sweep
    // the tile: x points [r0, r0 + nr), y points [c0, c0 + nc)
    const long long m0 = (long long)tile * T;
    const long long m1 = min(m0 + T, a.n + a.m);
    const long long r0 = min(max((long long)a.trs[tile], 0LL), a.n);
    const long long r1 = min(max((long long)a.trs[tile + 1], r0), a.n);
    const long long c0 = min(max(m0 - r0, 0LL), a.m);
    long long c1 = min(max(m1 - r1, c0), a.m);
    if (c1 - c0 > T) c1 = c0 + T;
    const int nc = (int)(c1 - c0);
    const int nr = (int)min(r1 - r0, (long long)(T - nc));

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
    // other blocks finish the previous sweep), the wait for the previous
    // sweep's records, the carries, the rows, publication and arrival.
    __shared__ int s_flag;
    unsigned gen = 0;
    // the first sweep's column totals (x points) from the initial state
    Ext<float> own_l, own_u;
    {
        RefAcc n1{0.f, kZeroExp}, n2{0.f, kZeroExp};
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int k = threadIdx.x + q * BLOCK - nc;
            if (k >= 0 && k < nr) {
                ref_add(n1, Ext<float>{U[q].m * B[q].m, U[q].e + B[q].e});
                ref_add(n2, U[q]);
            }
        }
        block_total2_write<BLOCK>(n1, n2, s_f + 4 * NW, s_i + 4 * NW);
        __syncthreads();
        own_l = block_total_read<BLOCK>(s_f + 4 * NW, s_i + 4 * NW);
        own_u = block_total_read<BLOCK>(s_f + 5 * NW, s_i + 5 * NW);
        ++gen;
        if (threadIdx.x == 0) {
            resident_publish(rec_x + 2 * tile, u64_of(own_l), rec_x + 2 * tile + 1, u64_of(own_u), nullptr, 0);
            resident_arrive(a, gen);
        }
    }

    const long long itr_max = a.ps->itr_max;
    const double tol = a.ps->tol;
    long long l = 0;
    double err = 0.0;
    bool ok = true;
    ResidentIn in;
    Ext<float> uold[IPT];   // the y points' states the loop head checks
    for (;;) {
        // ---- K^T phi with the marginal check: columns x, rows y
        resident_columns<BLOCK, IPT>(nc, nr, own_l.e, own_u.e, U, B, s_l, s_u, s_f);
        const int rxl = own_l.e, rxu = own_u.e;
        ok = resident_wait(a, gen, &s_flag);
        if (!ok) break;
        resident_read<false>(a, rec_x, nullptr, in);
        resident_rows<BLOCK, IPT, true>(in, nr, 0, nc, rxl, rxu, U, s_a, B, s_z, uold, s_l, s_u, s_f, s_i, s_d);
        own_l = block_total_read<BLOCK>(s_f + 4 * NW, s_i + 4 * NW);
        own_u = block_total_read<BLOCK>(s_f + 5 * NW, s_i + 5 * NW);
        ++gen;
        if (threadIdx.x == 0) {
            const double pe = block_read_sum<BLOCK>(s_d);
            unsigned long long pb;
            __builtin_memcpy(&pb, &pe, sizeof(pb));
            resident_publish(rec_y + 2 * tile, u64_of(own_l), rec_y + 2 * tile + 1, u64_of(own_u), rec_p + tile,
                             pb);
            resident_arrive(a, gen);
        }
        // ---- K psi: its columns (y) while the others finish, then the loop
        // head (every block sums the partials in the same order)
        __syncthreads();   // s_d and the LDS scans of the checking sweep are read
        resident_columns<BLOCK, IPT>(0, nc, own_l.e, own_u.e, U, B, s_l, s_u, s_f);
        const int ryl = own_l.e, ryu = own_u.e;
        ok = resident_wait(a, gen, &s_flag);
        if (!ok) break;
        resident_read<true>(a, rec_y, rec_p, in);
        wave_sum_to<BLOCK>(in.part, s_d);
        __syncthreads();
        err = block_read_sum<BLOCK>(s_d);
        if (l >= itr_max || !(err > tol)) {
            // the returned psi: the states the loop head checked
#pragma unroll
            for (int q = 0; q < IPT; ++q) {
                const int k = threadIdx.x + q * BLOCK;
                if (k < nc) a.UG[c0 + k] = uold[q];
            }
            break;
        }
        // ---- K psi: rows x
        resident_rows<BLOCK, IPT, false>(in, nc, nc, nr, ryl, ryu, U, s_a, B, s_z, nullptr, s_l, s_u, s_f, s_i,
                                         s_d);
        own_l = block_total_read<BLOCK>(s_f + 4 * NW, s_i + 4 * NW);
        own_u = block_total_read<BLOCK>(s_f + 5 * NW, s_i + 5 * NW);
        ++gen;
        if (threadIdx.x == 0) {
            resident_publish(rec_x + 2 * tile, u64_of(own_l), rec_x + 2 * tile + 1, u64_of(own_u), nullptr, 0);
            resident_arrive(a, gen);
        }
        __syncthreads();   // the LDS scans of K psi are read
        ++l;
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
        P->err = err;
        P->iters = l;
        P->converged = (ok && err <= tol) ? 1 : 0;
        P->status = (!(err == err) || err == __builtin_inf()) ? 1 : 0;
        P->done = 1;
    }
}

}  // namespace finom
