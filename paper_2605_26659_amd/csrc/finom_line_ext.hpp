// Line sweeps on extended-number state, for the 2D loop in FP32 mode.
//
// Algorithm 2 applies the 1D product along one axis of the grid and then
// along the other (eq. 2d-kpsi / 2d-ktphi). With the grid's scalings kept as
// U = w 2^{-(a + b) kappa} for the point (a, b) (both coordinates), the 1D
// fast form of a line product carries over unchanged: along a line in which
// the coordinate c varies, the column terms are U 2^{2 c kappa} (lower block)
// and U (upper block), and a row at coordinate r gets W = L + 2^{2 r kappa} R
// from the exclusive prefix L and the suffix R of those terms at its dividing
// index. The factor 2^{-c' kappa} of the other coordinate is constant along
// the line and passes through unchanged, so
//   - the first product of a pair stores W itself as the next product's
//     column input (it is that product's U up to a factor constant along each
//     of its lines), and
//   - the second product's W is K^T phi (or K psi) times 2^{(a + b) kappa} of
//     the target point: the Sinkhorn update is U = A / W with the mass A, and
//     the loop head's marginal error |psi_old (K^T phi) - v| is |U_old W - A|.
// No exponential or logarithm is taken per point and iteration.
//
// Along a whole line of a 2D grid the terms span far more than FP32's range
// (2 kappa times the line's extent), so the in-line sums are extended numbers
// (FP32 mantissa, int32 exponent); the tile of one block is the whole line
// (lines of up to BLOCK * IPT points on each side), so there are no carries.
// One block per line; workgroups are renumbered so that each XCD takes a
// contiguous range of lines (xcd_block): the products that store their
// output with a stride then fill whole cache lines in one L2.
#pragma once
#include "finom_fast.hpp"

namespace finom {

// One product over all lines of a pass: line l reads its C column values at
// uin + l uin_line (contiguous) and writes row i at out + l out_line + i
// out_elem. Rows and columns are the same for every line (the axis meshes).
struct PassExt {
    const Ext<float>* uin;   // column input (U, or W of the previous product)
    const Ext<float>* bc;    // 2^{2 c kappa} per column
    const Ext<float>* br;    // 2^{2 r kappa} per row
    const int* zeta;         // per row: #{columns at or below it}
    Ext<float>* out;
    const Ext<float>* a;     // masses (update epilogues), row i of line l at a + l a_line + i
    const Ext<float>* uold;  // state the check reads, laid out as a
    double* partial;         // check: one partial error per line
    const double* dec;       // the stop decision sums dec[0, dec_n) (null: no decision)
    long long uin_line, out_line, out_elem, a_line;
    int R, C;
    int dec_n;
    int prob;
};

enum { LX_STORE = 0, LX_UPDATE = 1, LX_UPDATE_CHECK = 2 };

// LDS index of scan entry e: one 8-byte slot of padding after every 32
// entries, so that threads reading chunks of 4 to 8 consecutive entries
// (stride 32 to 64 bytes) fall on distinct banks.
__device__ __forceinline__ int lx_pad(int e) { return e + (e >> 5); }

template <int T>
struct LxLen {
    static constexpr int value = T + 1 + ((T + 1) >> 5) + 1;
};

// Sum of extended values in lanes [0, N) (N <= 16, a power of two), read from lane N - 1.
template <int N>
__device__ __forceinline__ Ext<float> first_lanes_sum_ext(Ext<float> v)
{
    static_assert(N >= 1 && N <= 16 && (N & (N - 1)) == 0, "one row, power of two");
    if (N > 1) v = ext_add(v, dpp_ext<0x111>(v));
    if (N > 2) v = ext_add(v, dpp_ext<0x112>(v));
    if (N > 4) v = ext_add(v, dpp_ext<0x114>(v));
    if (N > 8) v = ext_add(v, dpp_ext<0x118>(v));
    return readlane_ext(v, N - 1);
}

// Exclusive prefix (s_l) and inclusive suffix (s_u) of C extended terms in
// place (entry e at lx_pad(e)), thread t owning the chunk [t ch, t ch + ch);
// entry C gets the total in s_l and zero in s_u (a row above every column). The caller has passed a barrier
// since the terms were written, and passes another before reading.
template <int BLOCK, int IPT>
__device__ __forceinline__ void line_scan_ext(Ext<float>* s_l, Ext<float>* s_u, int C, Ext<float>* s_w)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int ch = (C + BLOCK - 1) / BLOCK;   // block-uniform, at most IPT
    const int base = threadIdx.x * ch;
    Ext<float> vl[IPT], vu[IPT];
    Ext<float> sl = ext_zero<float>(), su = ext_zero<float>();
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        vl[q] = vu[q] = ext_zero<float>();
        if (q < ch) {   // block-uniform
            if (base + q < C) {
                vl[q] = s_l[lx_pad(base + q)];
                vu[q] = s_u[lx_pad(base + q)];
            }
            sl = ext_add(sl, vl[q]);
            su = ext_add(su, vu[q]);
        }
    }
    const Ext<float> il = wave_incl_prefix(sl);
    const Ext<float> iu = wave_incl_suffix(su);
    if (lane == kWave - 1) s_w[wid] = il;
    if (lane == 0) s_w[NW + wid] = iu;
    __syncthreads();
    // the other waves' totals: lane j < NW reads wave j's
    const int j = lane & (NW - 1);
    const bool head = lane < NW;
    Ext<float> a = s_w[j], b = s_w[NW + j];
    if (!(head && j < wid)) a = ext_zero<float>();
    if (!(head && j > wid)) b = ext_zero<float>();
    a = first_lanes_sum_ext<NW>(a);
    b = first_lanes_sum_ext<NW>(b);
    Ext<float> run = ext_add(a, dpp_ext<0x138>(il));    // wave_shr:1 -> exclusive prefix
    Ext<float> runu = ext_add(dpp_ext<0x130>(iu), b);   // wave_shl:1 -> exclusive suffix
    // every entry was read before the barrier above: overwrite in place
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q < ch) {
            if (base + q < C) s_l[lx_pad(base + q)] = run;
            run = ext_add(run, vl[q]);
        }
    }
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) {
        if (q < ch) {
            runu = ext_add(runu, vu[q]);
            if (base + q < C) s_u[lx_pad(base + q)] = runu;
        }
    }
    if (threadIdx.x == BLOCK - 1) {
        s_l[lx_pad(C)] = run;   // the chunks past C are zero: run is the total
        s_u[lx_pad(C)] = ext_zero<float>();
    }
}

// ---- the in-line scan with FP64 mantissas against one reference per wave
//
// Wave w of the block owns the chunk of columns [64 IPT w, 64 IPT (w + 1)).
// Its terms are scaled to the chunk's largest exponent and summed in FP64;
// chunks are chained by extended-number carries. A term more than 2^-1022
// below its chunk's largest vanishes. For the prefix L at a row that can only
// matter if the chunk's largest lower-block term comes after the row, and
// then that term's upper-block twin enters B R at the row, damped by the
// kernel over at most the chunk's extent plus one neighbouring column: when
// 2 kappa times that extent is at most kSpan64 binary orders, B R exceeds the
// vanished part of L by more than 2^53 (and the same with the two blocks
// swapped). The host checks the extent per chunk of every axis mesh
// (ext2d_scan64); otherwise the extended-number scan runs.
constexpr double kSpan64 = 900.0;

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ double dpp_f64(double v)   // lanes without a source read 0
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, RM, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RM, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_incl_prefix_f64(double v)
{
    v += dpp_f64<0x111>(v);          // row_shr:1
    v += dpp_f64<0x112>(v);          // row_shr:2
    v += dpp_f64<0x114>(v);          // row_shr:4
    v += dpp_f64<0x118>(v);          // row_shr:8
    v += dpp_f64<0x142, 0xA>(v);     // row_bcast:15
    v += dpp_f64<0x143, 0xC>(v);     // row_bcast:31
    return v;
}

__device__ __forceinline__ double wave_incl_suffix_f64(double v)
{
    v += dpp_f64<0x101>(v);          // row_shl:1
    v += dpp_f64<0x102>(v);          // row_shl:2
    v += dpp_f64<0x104>(v);          // row_shl:4
    v += dpp_f64<0x108>(v);          // row_shl:8
    const double t1 = readlane_f64(v, 16), t2 = readlane_f64(v, 32), t3 = readlane_f64(v, 48);
    const double s1 = t2 + t3;
    const double s0 = t1 + s1;
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    const double add = (row == 0) ? s0 : (row == 1) ? s1 : (row == 2) ? t3 : 0.0;
    return v + add;
}

// Per-wave scan data: the waves' totals and reference exponents (for the
// carries) and the final reference of every chunk's stored values.
template <int NW>
struct LxWaves {
    double tot[2 * NW];
    int ref[2 * NW];
    int R[2 * NW];   // [w]: lower block, [NW + w]: upper block
};

// The scan of C terms in s_l / s_u (Ext<float>, entry e at lx_pad(e)) into
// FP64 values in the same slots: entry e of the lower block holds the
// exclusive prefix, of the upper block the inclusive suffix, each as the
// mantissa against 2^{W.R[chunk of e]}; entry C gets the total and zero. The
// caller has passed a barrier since the terms were written, and passes another
// before reading.
template <int BLOCK, int IPT>
__device__ __forceinline__ void line_scan_f64(Ext<float>* s_l, Ext<float>* s_u, int C, LxWaves<BLOCK / kWave>& W)
{
    constexpr int NW = BLOCK / kWave;
    double* const dl_out = reinterpret_cast<double*>(s_l);
    double* const du_out = reinterpret_cast<double*>(s_u);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int base = threadIdx.x * IPT;
    // the chunk's terms and their largest exponents (zero terms excluded)
    Ext<float> vl[IPT], vu[IPT];
    int ml = kZeroExp, mu = kZeroExp;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        vl[q] = vu[q] = ext_zero<float>();
        if (base + q < C) {
            vl[q] = s_l[lx_pad(base + q)];
            vu[q] = s_u[lx_pad(base + q)];
        }
        ml = max(ml, vl[q].m != 0.f ? vl[q].e : kZeroExp);
        mu = max(mu, vu[q].m != 0.f ? vu[q].e : kZeroExp);
    }
    ml = wave_max_i(ml);
    mu = wave_max_i(mu);
    double dl[IPT], du[IPT];
    double sl = 0.0, su = 0.0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        dl[q] = __builtin_amdgcn_ldexp((double)vl[q].m, vl[q].e - ml);
        du[q] = __builtin_amdgcn_ldexp((double)vu[q].m, vu[q].e - mu);
        sl += dl[q];
        su += du[q];
    }
    const double il = wave_incl_prefix_f64(sl);
    const double iu = wave_incl_suffix_f64(su);
    if (lane == kWave - 1) {
        W.tot[wid] = il;
        W.ref[wid] = ml;
    }
    if (lane == 0) {
        W.tot[NW + wid] = iu;
        W.ref[NW + wid] = mu;
    }
    __syncthreads();
    // carries: the totals of the chunks before (lower) and after (upper)
    Ext<double> CL = ext_zero<double>(), CU = ext_zero<double>();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wid) CL = ext_add(CL, Ext<double>{W.tot[w], W.ref[w]});
        if (w > wid) CU = ext_add(CU, Ext<double>{W.tot[NW + w], W.ref[NW + w]});
    }
    // the chunk's final references: the larger of its own and the carry's
    const int Rl = max(ml, CL.e), Ru = max(mu, CU.e);
    const double cl_rel = __builtin_amdgcn_ldexp(CL.m, CL.e - Rl), cu_rel = __builtin_amdgcn_ldexp(CU.m, CU.e - Ru);
    const double scl = __builtin_amdgcn_ldexp(1.0, ml - Rl), scu = __builtin_amdgcn_ldexp(1.0, mu - Ru);
    double run = dpp_f64<0x138>(il);    // wave_shr:1 -> exclusive prefix
    double runu = dpp_f64<0x130>(iu);   // wave_shl:1 -> exclusive suffix
    // every entry was read before the barrier above: overwrite in place
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (base + q < C) dl_out[lx_pad(base + q)] = __builtin_fma(run, scl, cl_rel);
        run += dl[q];
    }
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) {
        runu += du[q];
        if (base + q < C) du_out[lx_pad(base + q)] = __builtin_fma(runu, scu, cu_rel);
    }
    if (lane == 0) {
        W.R[wid] = Rl;
        W.R[NW + wid] = Ru;
    }
    // entry C (a row above every column): in the chunk that holds position C
    if (lane == 0 && wid == min(C / (kWave * IPT), NW - 1)) {
        dl_out[lx_pad(C)] = __builtin_fma(readlane_f64(il, kWave - 1), scl, cl_rel);
        du_out[lx_pad(C)] = 0.0;
    }
}

// W = L + B R at a row with dividing index z (after either scan).
template <int BLOCK, int IPT, bool S64>
__device__ __forceinline__ Ext<float> lx_row_w(const Ext<float>* s_l, const Ext<float>* s_u,
                                               const LxWaves<BLOCK / kWave>& Wv, int z, Ext<float> b)
{
    constexpr int NW = BLOCK / kWave;
    if constexpr (S64) {
        const int w = min(z / (kWave * IPT), NW - 1);
        const double lm = reinterpret_cast<const double*>(s_l)[lx_pad(z)];
        const double um = reinterpret_cast<const double*>(s_u)[lx_pad(z)];
        const Ext<double> Wd = ext_add(Ext<double>{lm, Wv.R[w]}, Ext<double>{um * (double)b.m, Wv.R[NW + w] + b.e});
        return Ext<float>{(float)__builtin_amdgcn_frexp_mant(Wd.m), Wd.e + __builtin_amdgcn_frexp_exp(Wd.m)};
    } else {
        const Ext<float> Lz = s_l[lx_pad(z)], Rz = s_u[lx_pad(z)];
        return ext_norm(ext_add(Lz, Ext<float>{Rz.m * b.m, Rz.e + b.e}));
    }
}

template <int BLOCK, int IPT, int EPI, bool S64>
__global__ __launch_bounds__(BLOCK) void k_line_ext(PassExt d, ProbState* __restrict__ ps, int parity)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    constexpr bool UPD = EPI != LX_STORE;
    constexpr bool CHECK = EPI == LX_UPDATE_CHECK;
    __shared__ Ext<float> s_l[LxLen<T>::value];
    __shared__ Ext<float> s_u[LxLen<T>::value];
    __shared__ Ext<float> s_w[2 * NW];
    __shared__ LxWaves<NW> s_wv;
    __shared__ double s_red[NW];

    const int l = xcd_block(blockIdx.x, gridDim.x);
    ProbState* P = ps + d.prob;
    if (P->done) return;
    const int R = d.R, C = d.C;

    // ---- loads (tail slots re-read the last element)
    const gptr<const Ext<float>> UI = gbl(d.uin) + (long long)l * d.uin_line;
    const gptr<const Ext<float>> BC = gbl(d.bc), BR = gbl(d.br);
    const gptr<const int> Z = gbl(d.zeta);
    Ext<float> cu[IPT], cb[IPT], rb[IPT], ra[IPT], ro[IPT];
    int rz[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= C) break;   // block-uniform
        const int k = min((int)threadIdx.x + q * BLOCK, C - 1);
        cu[q] = UI[k];
        cb[q] = BC[k];
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R) break;
        const int i = min((int)threadIdx.x + q * BLOCK, R - 1);
        rz[q] = Z[i];
        rb[q] = BR[i];
        if (UPD) ra[q] = gbl(d.a)[(long long)l * d.a_line + i];
        if (CHECK) ro[q] = gbl(d.uold)[(long long)l * d.a_line + i];
    }

    // ---- stop decision of the loop head (every block sums the same partials
    // in the same order; line 0 records it)
    if (d.dec) {
        // the partials and the count (written by earlier kernels) in one round trip
        const double v = strided_sum<BLOCK>(d.dec, d.dec_n);
        const long long it = P->cnt[parity];
        const double err = block_sum_f64<BLOCK>(v, s_red);
        const bool stop = (it >= P->itr_max) || !(err > P->tol);
        if (l == 0 && threadIdx.x == 0) {
            P->err = err;
            if (!(err == err) || err == __builtin_inf()) P->status = 1;
            if (stop) {
                P->iters = it;
                P->converged = (err <= P->tol) ? 1 : 0;
                P->done = 1;
            } else {
                P->cnt[parity ^ 1] = it + 1;
            }
        }
        if (stop) return;
    }

    // ---- column terms U 2^{2 c kappa} and U, then their in-line scans
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= C) break;
        const int k = threadIdx.x + q * BLOCK;
        if (k < C) {
            s_l[lx_pad(k)] = Ext<float>{cu[q].m * cb[q].m, cu[q].e + cb[q].e};
            s_u[lx_pad(k)] = cu[q];
        }
    }
    __syncthreads();
    if constexpr (S64) line_scan_f64<BLOCK, IPT>(s_l, s_u, C, s_wv);
    else line_scan_ext<BLOCK, IPT>(s_l, s_u, C, s_w);
    __syncthreads();

    // ---- rows: W = L + 2^{2 r kappa} R, then the epilogue
    const gptr<Ext<float>> OUT = gbl(d.out) + (long long)l * d.out_line;
    double red = 0.0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R) break;
        const int i = threadIdx.x + q * BLOCK;
        if (i < R) {
            const Ext<float> W = lx_row_w<BLOCK, IPT, S64>(s_l, s_u, s_wv, min(max(rz[q], 0), C), rb[q]);
            if (!UPD) {
                OUT[(long long)i * d.out_elem] = W;
            } else {
                const Ext<float> A = ra[q];
                const Ext<float> Un = ext_norm(Ext<float>{A.m * __builtin_amdgcn_rcpf(W.m), A.e - W.e});
                if (CHECK) {
                    // |U_old W - A| with one rounding, both operands scaled to the
                    // larger of the two exponents
                    const Ext<float> O = ro[q];
                    const int ep = O.e + W.e;
                    const int re = max(ep, A.e);
                    const float dd = __builtin_fmaf(ldexp_m(O.m, ep - re), W.m, -ldexp_m(A.m, A.e - re));
                    red += __builtin_amdgcn_ldexp((double)fabsf(dd), re);
                }
                store_update(OUT + i, Un);
            }
        }
    }
    if (CHECK) {
        const double b = block_sum_f64<BLOCK>(red, s_red);
        if (threadIdx.x == 0) d.partial[l] = b;
    }
}

// Two products of one line in one block. The first updates the line's
// scalings (U = A / W at its rows, with the marginal check when CHECK); the
// rows of the first are the columns of the second along the same axis, so the
// second takes the new U straight from the registers of the threads that
// formed it and stores its W with a stride, as the next pair's input:
//   per psi row c: psi <- v / (row c of K_x^T Phi) K_y, then row c of Psi K_y^T;
//   per phi column b: phi <- u / K_x (column b of Psi K_y^T), then K_x^T phi.
// With DECIDE the block first takes the loop head's decision from the check's
// partials (a stop leaves the line's state as it was).
struct PairExt {
    PassExt p1;              // the update (out: the line's state, contiguous)
    const Ext<float>* br2;   // rows of the second product
    const int* zeta2;
    Ext<float>* out2;
    long long out2_line, out2_elem;
    int R2;
};

// The pair of products of line l (the body of both kernels below).
template <int BLOCK, int IPT, bool CHECK, bool DECIDE, bool S64>
__device__ __forceinline__ void line_pair(const PairExt& pr, const int l, ProbState* __restrict__ ps, int parity)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NW = BLOCK / kWave;
    __shared__ Ext<float> s_l[LxLen<T>::value];
    __shared__ Ext<float> s_u[LxLen<T>::value];
    __shared__ Ext<float> s_w[2 * NW];
    __shared__ LxWaves<NW> s_wv;
    __shared__ double s_red[NW];

    const PassExt& d = pr.p1;
    ProbState* P = ps + d.prob;
    if (P->done) return;
    const int R = d.R, C = d.C, R2 = pr.R2;

    // ---- loads of both products (tail slots re-read the last element)
    const gptr<const Ext<float>> UI = gbl(d.uin) + (long long)l * d.uin_line;
    const gptr<const Ext<float>> BC = gbl(d.bc), BR = gbl(d.br), BR2 = gbl(pr.br2);
    const gptr<const int> Z = gbl(d.zeta), Z2 = gbl(pr.zeta2);
    Ext<float> cu[IPT], cb[IPT], rb[IPT], ra[IPT], ro[IPT], rb2[IPT];
    int rz[IPT], rz2[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= C) break;   // block-uniform
        const int k = min((int)threadIdx.x + q * BLOCK, C - 1);
        cu[q] = UI[k];
        cb[q] = BC[k];
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R) break;
        const int i = min((int)threadIdx.x + q * BLOCK, R - 1);
        rz[q] = Z[i];
        rb[q] = BR[i];
        ra[q] = gbl(d.a)[(long long)l * d.a_line + i];
        if (CHECK) ro[q] = gbl(d.uold)[(long long)l * d.a_line + i];
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R2) break;
        const int i = min((int)threadIdx.x + q * BLOCK, R2 - 1);
        rz2[q] = Z2[i];
        rb2[q] = BR2[i];
    }

    if (DECIDE) {
        // the partials and the count (written by earlier kernels) in one round trip
        const double v = strided_sum<BLOCK>(d.dec, d.dec_n);
        const long long it = P->cnt[parity];
        const double err = block_sum_f64<BLOCK>(v, s_red);
        const bool stop = (it >= P->itr_max) || !(err > P->tol);
        if (l == 0 && threadIdx.x == 0) {
            P->err = err;
            if (!(err == err) || err == __builtin_inf()) P->status = 1;
            if (stop) {
                P->iters = it;
                P->converged = (err <= P->tol) ? 1 : 0;
                P->done = 1;
            } else {
                P->cnt[parity ^ 1] = it + 1;
            }
        }
        if (stop) return;
    }

    // ---- first product: columns, scan, rows -> the new state
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= C) break;
        const int k = threadIdx.x + q * BLOCK;
        if (k < C) {
            s_l[lx_pad(k)] = Ext<float>{cu[q].m * cb[q].m, cu[q].e + cb[q].e};
            s_u[lx_pad(k)] = cu[q];
        }
    }
    __syncthreads();
    if constexpr (S64) line_scan_f64<BLOCK, IPT>(s_l, s_u, C, s_wv);
    else line_scan_ext<BLOCK, IPT>(s_l, s_u, C, s_w);
    __syncthreads();
    const gptr<Ext<float>> OUT = gbl(d.out) + (long long)l * d.out_line;
    Ext<float> un[IPT];
    double red = 0.0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R) break;
        const int i = threadIdx.x + q * BLOCK;
        if (i < R) {
            const Ext<float> W = lx_row_w<BLOCK, IPT, S64>(s_l, s_u, s_wv, min(max(rz[q], 0), C), rb[q]);
            const Ext<float> A = ra[q];
            un[q] = ext_norm(Ext<float>{A.m * __builtin_amdgcn_rcpf(W.m), A.e - W.e});
            if (CHECK) {
                const Ext<float> O = ro[q];
                const int ep = O.e + W.e;
                const int re = max(ep, A.e);
                const float dd = __builtin_fmaf(ldexp_m(O.m, ep - re), W.m, -ldexp_m(A.m, A.e - re));
                red += __builtin_amdgcn_ldexp((double)fabsf(dd), re);
            }
            store_update(OUT + i, un[q]);
        }
    }
    if (CHECK) {
        const double b = block_sum_f64<BLOCK>(red, s_red);   // ends with a barrier
        if (threadIdx.x == 0) d.partial[l] = b;
    } else {
        __syncthreads();   // the first scan's entries are read before they are replaced
    }

    // ---- second product: its columns are the rows just updated
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R) break;
        const int k = threadIdx.x + q * BLOCK;
        if (k < R) {
            s_l[lx_pad(k)] = Ext<float>{un[q].m * rb[q].m, un[q].e + rb[q].e};
            s_u[lx_pad(k)] = un[q];
        }
    }
    __syncthreads();
    if constexpr (S64) line_scan_f64<BLOCK, IPT>(s_l, s_u, R, s_wv);
    else line_scan_ext<BLOCK, IPT>(s_l, s_u, R, s_w);
    __syncthreads();
    const gptr<Ext<float>> OUT2 = gbl(pr.out2) + (long long)l * pr.out2_line;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q * BLOCK >= R2) break;
        const int i = threadIdx.x + q * BLOCK;
        if (i < R2)
            OUT2[(long long)i * pr.out2_elem] = lx_row_w<BLOCK, IPT, S64>(s_l, s_u, s_wv, min(max(rz2[q], 0), R),
                                                                          rb2[q]);
    }
}

// One problem: block b takes line xcd_block(b).
template <int BLOCK, int IPT, bool CHECK, bool DECIDE, bool S64>
__global__ __launch_bounds__(BLOCK) void k_line_pair_ext(PairExt pr, ProbState* __restrict__ ps, int parity)
{
    line_pair<BLOCK, IPT, CHECK, DECIDE, S64>(pr, xcd_block(blockIdx.x, gridDim.x), ps, parity);
}

// Several problems of one line shape in one launch (a batch or the server):
// work item w = xcd_block(b) is line w - first[j] of problem j, where
// first[j] <= w < first[j + 1] (first: nprob + 1 prefix sums of the line
// counts). Each line computes exactly what it computes alone.
template <int BLOCK, int IPT, bool CHECK, bool DECIDE, bool S64>
__global__ __launch_bounds__(BLOCK) void k_line_pair_ext_jobs(const PairExt* __restrict__ pairs,
                                                              const int* __restrict__ first, int nprob,
                                                              ProbState* __restrict__ ps, int parity)
{
    const int w = xcd_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= w) lo = mid;
        else hi = mid;
    }
    line_pair<BLOCK, IPT, CHECK, DECIDE, S64>(pairs[lo], w - first[lo], ps, parity);
}

// A 2D problem's arrays and launch descriptors for the extended-state loop
// (host side; filled by ext2d_bind / ext2d_setup in the library).
struct Ext2D {
    int shape = -1;                     // line shape (-1: not eligible)
    int s64 = 0;                        // every chunk of every axis mesh within kSpan64: the FP64 scan
    long long n1 = 0, m1 = 0, n2 = 0, m2 = 0;
    Ext<float>* UF = nullptr;           // phi's scalings, column-major n1 x m1
    Ext<float>* UG[2] = {nullptr, nullptr};   // psi's, row-major n2 x m2 (two buffers)
    Ext<float>* SX = nullptr;           // K_x^T phi, row-major n2 x m1
    Ext<float>* SY = nullptr;           // Psi K_y^T, column-major n2 x m1
    Ext<float>* Au = nullptr;           // masses as extended numbers (layouts of phi / psi)
    Ext<float>* Av = nullptr;
    Ext<float>* B[4] = {nullptr, nullptr, nullptr, nullptr};   // 2^{2 c kappa}: x1, x2, y1, y2
    double* part = nullptr;             // the check's partial error per psi row
    PassExt pro;                        // prologue: SX from the initial phi
    PairExt y[2], x[2];                 // per parity: psi rows, phi columns
};

// The extended-state 2D problems of one line shape and scan in a batch: per
// parity, their psi-row and phi-column pair descriptors (device arrays) and
// the prefix sums of their line counts (host side; filled by the engine).
struct Ext2DGroup {
    int shape = -1;
    int s64 = 0;
    int nprob = 0;
    const PairExt* y[2] = {nullptr, nullptr};
    const PairExt* x[2] = {nullptr, nullptr};
    const int* fy = nullptr;   // nprob + 1: prefix sums of n2 (psi rows)
    const int* fx = nullptr;   // nprob + 1: prefix sums of m1 (phi columns)
    int ny = 0, nx = 0;        // lines of each pass
};

// Conversions between a grid's log2 potentials (FP64) and its extended
// state U = 2^{g - (X_i + Y_j) kappa}, or the extended form of 2^{g}
// (masses, kappa = 0). Point k of the grid is (i, j) = (k mod nx, k / nx)
// column-major, or (k / ny, k mod ny) row-major. g may be null (the constant
// g0 everywhere).
struct GridConv {
    const double* g;         // log2 potentials (to_ext) / out (!to_ext)
    double* gout;
    Ext<float>* u;
    const Ext<float>* uin;
    const double* X;         // coordinates along the grid's first axis (null: 0)
    const double* Y;
    long long nx, ny;
    double g0, kappa;
    int row_major, to_ext;
};

constexpr int kConvBlock = 256;

template <int = 0>
__global__ __launch_bounds__(kConvBlock) void k_grid_conv(GridConv c)
{
    const long long n = c.nx * c.ny;
    for (long long k = (long long)blockIdx.x * kConvBlock + threadIdx.x; k < n;
         k += (long long)gridDim.x * kConvBlock) {
        long long i, j;
        if (c.row_major) {
            i = k / c.ny;
            j = k - i * c.ny;
        } else {
            j = k / c.nx;
            i = k - j * c.nx;
        }
        const double s = (c.X ? c.X[i] : 0.0) + (c.Y ? c.Y[j] : 0.0);
        if (c.to_ext) {
            const double g = c.g ? c.g[k] : c.g0;
            c.u[k] = ext_exp2<float>(g - s * c.kappa);
        } else {
            c.gout[k] = ext_log2(c.uin[k]) + s * c.kappa;
        }
    }
}

// 2^{2 x kappa} per point of one axis mesh, as extended numbers.
template <int = 0>
__global__ __launch_bounds__(kConvBlock) void k_axis_b(const double* __restrict__ x, long long n, double kappa,
                                                      Ext<float>* __restrict__ b)
{
    for (long long k = (long long)blockIdx.x * kConvBlock + threadIdx.x; k < n;
         k += (long long)gridDim.x * kConvBlock)
        b[k] = ext_exp2<float>(2.0 * x[k] * kappa);
}

}  // namespace finom
