// Linear-domain FINOM with the stored vector representation (precision 2).
//
// Section 2.2 represents the two quasi-collinear blocks of K by vectors: the
// ratios r_i = K_{i+1,j} / K_{i,j} = e^{-(x_{i+1}-x_i)/eps} (the same for
// both blocks, r'_i = r_i) and, per row, the entries eta_i, eta'_i of its new
// block-edge segment. Section 2.3 then evaluates K psi as p + q with
//   p_{i+1} = r_i p_i + eta_{i+1} . psi      (eq. p-DP, lower block)
//   q_i     = r'_i q_{i+1} + eta'_i . psi    (eq. q-DP, upper block)
// in the linear domain: no exponential or logarithm per iteration, only the
// stored vectors. This mode keeps them in FP64 and is valid where the kernel
// entries and the scalings phi, psi fit FP64 (the host refuses
// diam / eps > 600).
//
// Storage: every segment entry belongs to one column, so the representation
// is kept per mesh point: r_i per row, and per column j its lower-block
// weight eta_j = e^{-(x_a - y_j)/eps} against the first row a at or above it
// and its upper-block weight eta'_j = e^{-(y_j - x_{a-1})/eps} against the
// last row below it (0 where that row does not exist); a = #{i : x_i < y_j}.
// In the merged order of rows and columns (a row after the columns at or
// below it, a column after the rows strictly below it), both recurrences are
// scans of affine maps v -> alpha v + beta: forward, a column adds
// eta_j psi_j and a row reads p and then multiplies by r_i; backward, a column
// adds eta'_j psi_j and a row reads q and then multiplies by r_{i-1}. The
// composition of affine maps is associative, so the recurrences run as
// parallel scans: per merge-path tile (shared with the other modes) a blocked
// scan in LDS, and across tiles the ordered composition of the tiles' maps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <functional>
#include <vector>

#include "../../include/finom.h"
#include "finom_host.hpp"

namespace finom {

// v -> a v + b
struct Aff {
    double a, b;
};

__device__ __forceinline__ Aff aff_id() { return Aff{1.0, 0.0}; }

// first p, then q
__device__ __forceinline__ Aff aff_then(Aff p, Aff q) { return Aff{p.a * q.a, fma(q.a, p.b, q.b)}; }

__device__ __forceinline__ Aff shfl_up_aff(Aff v, int d) { return Aff{__shfl_up(v.a, d, kWave), __shfl_up(v.b, d, kWave)}; }

// Exclusive scan of the threads' maps in thread order (thread 0 first) and
// the block's total. s_tmp: 2 * BLOCK / kWave doubles.
template <int BLOCK>
__device__ __forceinline__ void block_scan_aff(Aff v, Aff& excl, Aff& total, double* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    Aff inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Aff o = shfl_up_aff(inc, d);
        if (lane >= d) inc = aff_then(o, inc);
    }
    Aff ex = shfl_up_aff(inc, 1);
    if (lane == 0) ex = aff_id();
    if (lane == kWave - 1) {
        s_tmp[wid] = inc.a;
        s_tmp[NW + wid] = inc.b;
    }
    __syncthreads();
    Aff before = aff_id();
    total = aff_id();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const Aff t{s_tmp[w], s_tmp[NW + w]};
        if (w < wid) before = aff_then(before, t);
        total = aff_then(total, t);
    }
    __syncthreads();
    excl = aff_then(before, ex);
}

// One product of the linear mode: rows xr (R), columns yc (C).
struct LinLine {
    const double* rr;      // R: r_i (the last entry unused)
    const double* eta;     // C: lower-block weight of each column
    const double* etap;    // C: upper-block weight of each column
    const int* zeta;       // R: #{j : y_j <= x_i}
    const int* above;      // C: #{i : x_i < y_j}
    const int* trs;        // tile row starts (ntiles + 1)
    const double* win;     // C: column input psi (linear)
    double* out;           // R: row output
    const double* a0;      // R: epilogue operand (masses)
    const double* a2;      // R: the check's old scaling
    long long R, C;
    int ntiles, T;
    int dec_off, dec_n;    // stop decision: partial slots (dec_n = 0: none)
    int pad0, pad1;
};

enum LinEpi { LIN_STORE = 0, LIN_UPDATE = 1, LIN_UPDATE_CHECK = 2 };

struct LinTile {
    long long r0, r1, c0, c1;
};

__device__ __forceinline__ LinTile lin_tile(const LinLine& L, int tile)
{
    // clamped as for the other sweeps: a corrupt partition gives wrong
    // values, never an out-of-range access
    LinTile g;
    const long long m0 = (long long)tile * L.T;
    long long m1 = min(m0 + (long long)L.T, L.R + L.C);
    g.r0 = min(max((long long)L.trs[tile], 0LL), L.R);
    g.r1 = min(max((long long)L.trs[tile + 1], g.r0), L.R);
    g.c0 = min(max(m0 - g.r0, 0LL), L.C);
    g.c1 = min(max(m1 - g.r1, g.c0), L.C);
    if (g.r1 - g.r0 > L.T) g.r1 = g.r0 + L.T;
    if (g.c1 - g.c0 > L.T - (g.r1 - g.r0)) g.c1 = g.c0 + (L.T - (g.r1 - g.r0));
    return g;
}

// Stop decision of Algorithm 1's loop head from the checking sweep's
// partials, as in the other modes: every block sums the same partials in the
// same order; block 0 records it. Returns true when the loop stops.
template <int BLOCK>
__device__ __forceinline__ bool lin_decide(const LinLine& L, ProbState* P, const double* dec, int parity,
                                           double* s_red)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < L.dec_n; k += BLOCK) v += dec[L.dec_off + k];
    const double err = block_sum_f64<BLOCK>(v, s_red);
    const long long l = P->cnt[parity];
    const bool stop = (l >= P->itr_max) || !(err > P->tol);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
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

template <int BLOCK, int IPT>
struct LinLds {
    static constexpr int T = BLOCK * IPT;
    double fa[T], fb[T], ba[T], bb[T];
    int row[T];
    double tmp[4 * (BLOCK / kWave)];
    double red[BLOCK / kWave];
};

// The tile's elements in merged order: slot s holds the forward map
// (fa, fb), the backward map (ba, bb) and the row index (or -1 for a column).
template <int BLOCK, int IPT>
__device__ __forceinline__ int lin_stage(const LinLine& L, const LinTile& g, LinLds<BLOCK, IPT>& S)
{
    constexpr int T = BLOCK * IPT;
    const int nr = (int)(g.r1 - g.r0), nc = (int)(g.c1 - g.c0);
    const int used = nr + nc;
    for (int k = threadIdx.x; k < T; k += BLOCK) {
        S.row[k] = -1;
        S.fa[k] = 1.0; S.fb[k] = 0.0; S.ba[k] = 1.0; S.bb[k] = 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nr; k += BLOCK) {
        const long long i = g.r0 + k;
        const int s = min(max((int)(k + (L.zeta[i] - g.c0)), 0), T - 1);
        S.row[s] = (int)(i - g.r0);
        S.fa[s] = L.rr[i];
        S.ba[s] = i > 0 ? L.rr[i - 1] : 0.0;
    }
    for (int k = threadIdx.x; k < nc; k += BLOCK) {
        const long long j = g.c0 + k;
        const int s = min(max((int)(k + (L.above[j] - g.r0)), 0), T - 1);
        const double w = L.win[j];
        S.fb[s] = L.eta[j] * w;
        S.bb[s] = L.etap[j] * w;
    }
    __syncthreads();
    return used;
}

// The ordered compositions of the other tiles' maps: the forward carry (tiles
// before `tile`, first to last) and the backward carry (tiles after it, last
// to first), each applied to 0.
template <int BLOCK>
__device__ __forceinline__ void lin_carries(const LinLine& L, int tile, const double4* __restrict__ agg, double& cf,
                                            double& cb, double* s_tmp)
{
    cf = cb = 0.0;
    if (L.ntiles <= 1) return;
    const int nf = tile, nb = L.ntiles - 1 - tile;
    const int qf = (nf + BLOCK - 1) / BLOCK, qb = (nb + BLOCK - 1) / BLOCK;
    Aff mf = aff_id(), mb = aff_id();
    for (int k = threadIdx.x * qf; k < min(nf, (int)(threadIdx.x + 1) * qf); ++k) {
        const double4 a = agg[k];
        mf = aff_then(mf, Aff{a.x, a.y});
    }
    for (int k = threadIdx.x * qb; k < min(nb, (int)(threadIdx.x + 1) * qb); ++k) {
        const double4 a = agg[L.ntiles - 1 - k];
        mb = aff_then(mb, Aff{a.z, a.w});
    }
    Aff ex, tf, tb;
    block_scan_aff<BLOCK>(mf, ex, tf, s_tmp);
    block_scan_aff<BLOCK>(mb, ex, tb, s_tmp);
    cf = tf.b;
    cb = tb.b;
}

// Per tile: the composition of its forward maps (first to last slot) and of
// its backward maps (last to first), as (fa, fb, ba, bb). With a pending stop
// decision it is taken here first (the sweep then takes none).
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_lin_aggregate(LinLine L, ProbState* __restrict__ P,
                                                         double4* __restrict__ agg, const double* __restrict__ dec,
                                                         int parity)
{
    __shared__ LinLds<BLOCK, IPT> S;
    if (P->done) return;
    if (dec && L.dec_n > 0 && lin_decide<BLOCK>(L, P, dec, parity, S.red)) return;
    const int tile = blockIdx.x;
    const LinTile g = lin_tile(L, tile);
    lin_stage<BLOCK, IPT>(L, g, S);
    const int base = threadIdx.x * IPT;
    Aff mf = aff_id(), mb = aff_id();
#pragma unroll
    for (int q = 0; q < IPT; ++q) mf = aff_then(mf, Aff{S.fa[base + q], S.fb[base + q]});
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) mb = aff_then(mb, Aff{S.ba[base + q], S.bb[base + q]});
    // backward: threads in reverse order, so scan thread BLOCK-1-t's map
    Aff ex, tf, tb;
    block_scan_aff<BLOCK>(mf, ex, tf, S.tmp);
    // reverse-order composition: gather by the mirrored thread
    __syncthreads();
    S.fa[threadIdx.x] = mb.a;
    S.fb[threadIdx.x] = mb.b;
    __syncthreads();
    const Aff mirrored{S.fa[BLOCK - 1 - threadIdx.x], S.fb[BLOCK - 1 - threadIdx.x]};
    block_scan_aff<BLOCK>(mirrored, ex, tb, S.tmp);
    if (threadIdx.x == 0) agg[tile] = make_double4(tf.a, tf.b, tb.a, tb.b);
}

// The tile sweep: both scans from the carries, then each row's product and
// the epilogue. LIN_UPDATE_CHECK also leaves the tile's partial marginal
// error |a2_i (K w)_i - a0_i| in partial[tile].
template <int BLOCK, int IPT, int EPI>
__global__ __launch_bounds__(BLOCK) void k_lin_sweep(LinLine L, ProbState* __restrict__ P,
                                                     const double4* __restrict__ agg, double* __restrict__ partial,
                                                     const double* __restrict__ dec, int parity)
{
    __shared__ LinLds<BLOCK, IPT> S;
    if (P->done) return;
    if (dec && L.dec_n > 0 && lin_decide<BLOCK>(L, P, dec, parity, S.red)) return;
    const int tile = blockIdx.x;
    const LinTile g = lin_tile(L, tile);
    double cf, cb;
    lin_carries<BLOCK>(L, tile, agg, cf, cb, S.tmp);
    lin_stage<BLOCK, IPT>(L, g, S);
    const int base = threadIdx.x * IPT;
    Aff mf = aff_id(), mb = aff_id();
#pragma unroll
    for (int q = 0; q < IPT; ++q) mf = aff_then(mf, Aff{S.fa[base + q], S.fb[base + q]});
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) mb = aff_then(mb, Aff{S.ba[base + q], S.bb[base + q]});
    Aff exf, exb, tot;
    block_scan_aff<BLOCK>(mf, exf, tot, S.tmp);
    // the backward scan runs over threads in reverse order: thread t takes the
    // map of thread BLOCK-1-t, and its exclusive result belongs to that thread
    __shared__ double s_m[2 * BLOCK];
    s_m[threadIdx.x] = mb.a;
    s_m[BLOCK + threadIdx.x] = mb.b;
    __syncthreads();
    const int mt = BLOCK - 1 - threadIdx.x;
    Aff rex;
    block_scan_aff<BLOCK>(Aff{s_m[mt], s_m[BLOCK + mt]}, rex, tot, S.tmp);
    s_m[mt] = rex.a;
    s_m[BLOCK + mt] = rex.b;
    __syncthreads();
    exb = Aff{s_m[threadIdx.x], s_m[BLOCK + threadIdx.x]};

    // forward values: p at each row slot (read before the row's map)
    double pv[IPT], qv[IPT];
    double v = fma(exf.a, cf, exf.b);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        pv[q] = v;
        v = fma(S.fa[base + q], v, S.fb[base + q]);
    }
    double w = fma(exb.a, cb, exb.b);
#pragma unroll
    for (int q = IPT - 1; q >= 0; --q) {
        qv[q] = w;
        w = fma(S.ba[base + q], w, S.bb[base + q]);
    }
    double red = 0.0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int rk = S.row[base + q];
        if (rk < 0) continue;
        const long long i = g.r0 + rk;
        const double prod = pv[q] + qv[q];
        if (EPI == LIN_STORE) {
            L.out[i] = prod;
        } else if (EPI == LIN_UPDATE) {
            L.out[i] = L.a0[i] / prod;
        } else {
            const double m = L.a0[i];
            red += fabs(fma(L.a2[i], prod, -m));
            L.out[i] = m / prod;
        }
    }
    if (EPI == LIN_UPDATE_CHECK) {
        const double b = block_sum_f64<BLOCK>(red, S.red);
        if (threadIdx.x == 0) partial[tile] = b;
    }
}

// Representation of one product (rows xr, columns yc): r per row, the two
// column weights and each column's count of rows strictly below it.
__global__ __launch_bounds__(kBlock) void k_lin_rep(const double* __restrict__ xr, long long R,
                                                    const double* __restrict__ yc, long long C, double inv_eps,
                                                    double* __restrict__ rr, double* __restrict__ eta,
                                                    double* __restrict__ etap, int* __restrict__ above)
{
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k < R) rr[k] = (k + 1 < R) ? exp(-(xr[k + 1] - xr[k]) * inv_eps) : 0.0;
    if (k < C) {
        const double y = yc[k];
        long long lo = 0, hi = R;   // #{i : x_i < y}
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            if (xr[mid] < y) lo = mid + 1;
            else hi = mid;
        }
        above[k] = (int)lo;
        eta[k] = (lo < R) ? exp(-(xr[lo] - y) * inv_eps) : 0.0;
        etap[k] = (lo > 0) ? exp(-(y - xr[lo - 1]) * inv_eps) : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_lin_fill(double* __restrict__ a, long long n, double v)
{
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) a[k] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int BLOCK, int IPT>
static void lin_launch_t(const LinLine& L, int epi, ProbState* P, double4* agg, double* partial, const double* dec,
                         int parity, hipStream_t s)
{
    if (L.ntiles > 1) {
        hipLaunchKernelGGL((k_lin_aggregate<BLOCK, IPT>), dim3(L.ntiles), dim3(BLOCK), 0, s, L, P, agg, dec, parity);
        dec = nullptr;   // the aggregate kernel took the decision
    }
    if (epi == LIN_STORE)
        hipLaunchKernelGGL((k_lin_sweep<BLOCK, IPT, LIN_STORE>), dim3(L.ntiles), dim3(BLOCK), 0, s, L, P, agg,
                           partial, dec, parity);
    else if (epi == LIN_UPDATE)
        hipLaunchKernelGGL((k_lin_sweep<BLOCK, IPT, LIN_UPDATE>), dim3(L.ntiles), dim3(BLOCK), 0, s, L, P, agg,
                           partial, dec, parity);
    else
        hipLaunchKernelGGL((k_lin_sweep<BLOCK, IPT, LIN_UPDATE_CHECK>), dim3(L.ntiles), dim3(BLOCK), 0, s, L, P,
                           agg, partial, dec, parity);
    HIPCHK(hipGetLastError());
}

// The general tile shape of cfg (the partition's T) picks the instantiation.
static void lin_launch(int cfg, const LinLine& L, int epi, ProbState* P, double4* agg, double* partial,
                       const double* dec, int parity, hipStream_t s)
{
    switch (kCfgs[cfg].general) {
        case 0: lin_launch_t<256, 4>(L, epi, P, agg, partial, dec, parity, s); return;
        case 1: lin_launch_t<256, 8>(L, epi, P, agg, partial, dec, parity, s); return;
        case 2: lin_launch_t<512, 8>(L, epi, P, agg, partial, dec, parity, s); return;
        case 3: lin_launch_t<128, 4>(L, epi, P, agg, partial, dec, parity, s); return;
    }
    throw HipError{hipErrorInvalidValue};
}

struct LinRep {
    double *rr = nullptr, *eta = nullptr, *etap = nullptr;
    int* above = nullptr;
};

static LinRep lin_rep(Alloc& al, const Part& p, double eps, hipStream_t s)
{
    LinRep r;
    r.rr = al.dev<double>(p.R);
    r.eta = al.dev<double>(p.C);
    r.etap = al.dev<double>(p.C);
    r.above = al.dev<int>(p.C);
    hipLaunchKernelGGL(k_lin_rep, dim3(blocks_for(std::max(p.R, p.C))), dim3(kBlock), 0, s, p.xr, p.R, p.yc, p.C,
                       1.0 / eps, r.rr, r.eta, r.etap, r.above);
    HIPCHK(hipGetLastError());
    return r;
}

static LinLine lin_line(const Part& p, const LinRep& r)
{
    LinLine L;
    memset(&L, 0, sizeof(L));
    L.rr = r.rr;
    L.eta = r.eta;
    L.etap = r.etap;
    L.zeta = p.zeta;
    L.above = r.above;
    L.trs = p.trs;
    L.R = p.R;
    L.C = p.C;
    L.ntiles = p.ntiles;
    L.T = p.T;
    return L;
}

// Largest diam / eps the linear mode accepts: e^{+-600} stays well inside FP64.
constexpr double kLinearSpan = 600.0;

bool linear_span_ok(double lo, double hi, double eps) { return (hi - lo) / eps <= kLinearSpan; }

// K w for one product in the linear mode (finom_matvec with precision 2).
void linear_matvec(Alloc& al, const Part& p, double eps, const double* w, double* out, int cfg, hipStream_t s)
{
    const LinRep r = lin_rep(al, p, eps, s);
    LinLine L = lin_line(p, r);
    L.win = w;
    L.out = out;
    ProbState* ps = al.dev<ProbState>(1);
    HIPCHK(hipMemsetAsync(ps, 0, sizeof(ProbState), s));
    double4* agg = al.dev<double4>(std::max(p.ntiles, 1));
    lin_launch(cfg, L, LIN_STORE, ps, agg, nullptr, nullptr, 0, s);
}

// Algorithm 1 in the linear mode. phi (n) and psi[2] (m, ping-pong) hold the
// scalings; on return phi and psi[ret_psi] are the returned pair, still
// linear. The loop runs k iterations per captured graph, one state read per
// replay, as the other modes.
int linear_loop(Alloc& al, const Part& pk, const Part& pkt, int cfg, const double* u, const double* v, double eps,
                long long itr_max, int k, double* phi, double* psi[2], ProbState* ps, ProbState* hps,
                hipStream_t s, finom_result* res, int* ret_psi)
{
    const long long n = pk.R, m = pk.C;
    const LinRep rk = lin_rep(al, pk, eps, s);     // K:   rows x, columns y
    const LinRep rkt = lin_rep(al, pkt, eps, s);   // K^T: rows y, columns x
    hipLaunchKernelGGL(k_lin_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, phi, n, 1.0 / (double)n);
    hipLaunchKernelGGL(k_lin_fill, dim3(blocks_for(m)), dim3(kBlock), 0, s, psi[0], m, 1.0 / (double)m);
    HIPCHK(hipGetLastError());
    double4* agg = al.dev<double4>(std::max(pk.ntiles, 1));
    double* partial = al.dev<double>(std::max(pkt.ntiles, 1));
    LinLine kt[2], kp[2];
    for (int b = 0; b < 2; ++b) {
        kt[b] = lin_line(pkt, rkt);   // psi = v / K^T phi, with the check of (phi, psi_old)
        kt[b].win = phi;
        kt[b].out = psi[1 - b];
        kt[b].a0 = v;
        kt[b].a2 = psi[b];
        kp[b] = lin_line(pk, rk);     // phi = u / K psi, after the stop decision
        kp[b].win = psi[1 - b];
        kp[b].out = phi;
        kp[b].a0 = u;
        kp[b].dec_off = 0;
        kp[b].dec_n = pkt.ntiles;
    }
    k += (k & 1);
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int st = FINOM_OK;
    try {
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < k; ++it) {
            const int b = it & 1;
            lin_launch(cfg, kt[b], LIN_UPDATE_CHECK, ps, agg, partial, nullptr, b, cs);
            lin_launch(cfg, kp[b], LIN_UPDATE, ps, agg, nullptr, partial, b, cs);
        }
        HIPCHK(hipStreamEndCapture(cs, &graph));
        HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        HIPCHK(hipEventCreate(&ev0));
        HIPCHK(hipEventCreate(&ev1));
        HIPCHK(hipEventRecord(ev0, s));
        const long long max_launches = itr_max / k + 2;
        long long launches = 0;
        for (;;) {
            HIPCHK(hipGraphLaunch(exec, s));
            ++launches;
            HIPCHK(hipMemcpyAsync(hps, ps, sizeof(ProbState), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hps->done) break;
            if (launches > max_launches) {   // only if the device state were corrupt
                st = FINOM_E_HIP;
                break;
            }
        }
        HIPCHK(hipEventRecord(ev1, s));
        HIPCHK(hipEventSynchronize(ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
        res->loop_ms = ms;
    } catch (...) {
        st = map_exception();
        if (cs) {
            hipStreamCaptureStatus cst;
            if (hipStreamIsCapturing(cs, &cst) == hipSuccess && cst == hipStreamCaptureStatusActive) {
                hipGraph_t g2 = nullptr;
                hipStreamEndCapture(cs, &g2);
                if (g2) hipGraphDestroy(g2);
            }
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cs) hipStreamDestroy(cs);
    *ret_psi = (int)(hps->iters & 1);
    return st;
}

}  // namespace finom
