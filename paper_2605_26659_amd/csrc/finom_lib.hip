// Host side of the FINOM library: device setup kernels (sortedness, dividing
// index, merge-path partition, log masses), workspace, sweep dispatch, the
// Sinkhorn loops of Algorithm 1 (1D) and Algorithm 2 (2D) captured in HIP
// graphs, and the C ABI of include/finom.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <functional>
#include <mutex>

#include "../../include/finom.h"
#include "finom_host.hpp"
#include "finom_resident.hpp"

namespace finom {

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// flag |= 1 if a[k] > a[k+1] or a[k] is not finite.
__global__ void k_check_sorted(const double* __restrict__ a, long long n, int* __restrict__ flag)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double v = a[k];
    bool bad = !(v == v) || fabs(v) == __builtin_inf();
    if (k + 1 < n && v > a[k + 1]) bad = true;
    if (bad) atomicOr(flag, 1);
}

// flag |= 1 if a mass is not > 0 / not finite; writes its log2.
__global__ void k_log2_mass(const double* __restrict__ a, long long n, double* __restrict__ la,
                            int* __restrict__ flag)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double v = a[k];
    if (!(v > 0.0) || v == __builtin_inf()) atomicOr(flag, 1);
    la[k] = log2(v);
}

// Per-block partial sums in FP64 (deterministic two-pass reduction).
__global__ __launch_bounds__(kBlock) void k_partial_sum(const double* __restrict__ a, long long n,
                                                        double* __restrict__ part)
{
    __shared__ double s_red[kBlock / kWave];
    double v = 0.0;
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (long long)gridDim.x * kBlock)
        v += a[k];
    v = block_sum_f64<kBlock>(v, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// zeta[i] = #{j : y_j <= x_i} (the dividing index of section 2.2, as a count)
__global__ void k_dividing_index(const double* __restrict__ xr, long long R,
                                 const double* __restrict__ yc, long long C, int* __restrict__ zeta)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R) return;
    const double x = xr[i];
    long long lo = 0, hi = C;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (yc[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    zeta[i] = (int)lo;
}

// trs[t] = #{i : i + zeta[i] < t*T}: rows among the first t*T merged elements.
__global__ void k_tile_rows(const int* __restrict__ zeta, long long R, int T, int ntiles,
                            int* __restrict__ trs)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        trs[t] = (int)R;
        return;
    }
    const long long d = (long long)t * T;
    long long lo = 0, hi = R;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (mid + zeta[mid] < d) lo = mid + 1;
        else hi = mid;
    }
    trs[t] = (int)lo;
}

// rows of the transposed pair before tile t: the columns of the base pair
__global__ void k_tile_rows_complement(const int* __restrict__ trs, int T, int ntiles, long long total,
                                       int* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    long long d = (long long)t * T;
    if (d > total) d = total;
    out[t] = (int)(d - trs[t]);
}

__global__ void k_fill(double* __restrict__ a, long long n, double v)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = v;
}

__global__ void k_scale(const double* __restrict__ a, double* __restrict__ b, long long n, double s)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = a[k] * s;
}

// Dense product, one row per thread; columns staged through LDS.
template <typename M, int INM>
__global__ __launch_bounds__(kBlock) void k_dense(const double* __restrict__ xr, long long R,
                                                  const double* __restrict__ yc, long long C,
                                                  const double* __restrict__ gin, double kappa,
                                                  double in_scale, double out_scale, int lin_out,
                                                  double* __restrict__ out)
{
    constexpr int CH = 1024;
    __shared__ double s_y[CH];
    __shared__ double s_g[CH];
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    const double x = (i < R) ? xr[i] : 0.0;
    Ext<M> acc = ext_zero<M>();
    for (long long c0 = 0; c0 < C; c0 += CH) {
        const int nc = (int)min((long long)CH, C - c0);
        __syncthreads();
        for (int k = threadIdx.x; k < nc; k += kBlock) {
            s_y[k] = yc[c0 + k];
            s_g[k] = load_in<INM>(gbl(gin) + c0 + k, in_scale);
        }
        __syncthreads();
        for (int k = 0; k < nc; ++k)
            acc = ext_add(acc, ext_exp2<M>(s_g[k] - fabs(x - s_y[k]) * kappa));
    }
    if (i < R) {
        const double v = ext_log2(acc);
        out[i] = lin_out ? exp2(v) : v * out_scale;
    }
}

// ---------------------------------------------------------------------------
// arenas
// ---------------------------------------------------------------------------
static std::mutex g_mu;
static std::map<void*, Arena*> g_arenas;

Arena* arena_for(void* stream)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_arenas.find(stream);
    if (it != g_arenas.end()) return it->second;
    Arena* a = new Arena();
    g_arenas[stream] = a;
    return a;
}

void arena_free(Arena* a)
{
    if (a->upload_done) {
        hipEventSynchronize(a->upload_done);
        hipEventDestroy(a->upload_done);
        a->upload_done = nullptr;
    }
    for (auto& b : a->dblk) hipFree(b.p);
    for (auto& b : a->hblk) hipHostFree(b.p);
    a->dblk.clear();
    a->hblk.clear();
    a->dcur = a->hcur = 0;
    a->dused = a->hused = 0;
}

void arena_release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_arenas) {
        Arena* a = kv.second;
        if (a->upload_done) {
            hipEventSynchronize(a->upload_done);
            hipEventDestroy(a->upload_done);
        }
        hipStreamSynchronize((hipStream_t)kv.first);
        for (auto& b : a->dblk) hipFree(b.p);
        for (auto& b : a->hblk) hipHostFree(b.p);
        delete a;
    }
    g_arenas.clear();
}

static thread_local char g_last_error[256] = "";

void set_last_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

int map_exception()
{
    try {
        throw;
    } catch (const std::bad_alloc&) {
        snprintf(g_last_error, sizeof(g_last_error), "allocation failed");
        return FINOM_E_NOMEM;
    } catch (const StatusError& e) {
        return e.status;
    } catch (const HipError& e) {
        snprintf(g_last_error, sizeof(g_last_error), "%s (%d)", hipGetErrorString(e.e), (int)e.e);
        if (e.e == hipErrorOutOfMemory) return FINOM_E_NOMEM;
        return FINOM_E_HIP;
    } catch (...) {
        snprintf(g_last_error, sizeof(g_last_error), "unexpected exception");
        return FINOM_E_HIP;
    }
}

// ---------------------------------------------------------------------------
// sweeps
// ---------------------------------------------------------------------------
void upload_sweep(Alloc& al, Sweep& sw, size_t ext_b)
{
    const int ns = sw.ns();
    const int tt = sw.total_tiles(), mt = sw.multi_tiles();
    WorkItem* hw = al.host<WorkItem>(tt);
    WorkItem* hm = al.host<WorkItem>(mt);
    LineDesc* hl = al.host<LineDesc>(sw.lines.size());
    int k = 0, km = 0, abase = 0;
    for (size_t li = 0; li < sw.lines.size(); ++li) {
        LineDesc& L = sw.lines[li];
        L.agg_base = (L.ntiles > 1) ? abase : 0;
        if (L.ntiles > 1) abase += L.ntiles;
        for (int t = 0; t < L.ntiles; ++t) {
            hw[k++] = WorkItem{(int)li, t};
            if (L.ntiles > 1) hm[km++] = WorkItem{(int)li, t};
        }
        hl[li] = L;
    }
    WorkItem* dw = al.dev<WorkItem>(tt);
    WorkItem* dm = al.dev<WorkItem>(mt);
    LineDesc* dl = al.dev<LineDesc>(sw.lines.size());
    void* agg = sw.agg_buf ? sw.agg_buf : (void*)al.dev<char>((size_t)std::max(mt, 1) * ns * ext_b);
    HIPCHK(hipMemcpyAsync(dw, hw, sizeof(WorkItem) * tt, hipMemcpyHostToDevice, al.s));
    if (mt > 0) HIPCHK(hipMemcpyAsync(dm, hm, sizeof(WorkItem) * mt, hipMemcpyHostToDevice, al.s));
    HIPCHK(hipMemcpyAsync(dl, hl, sizeof(LineDesc) * sw.lines.size(), hipMemcpyHostToDevice, al.s));
    sw.dev.max_tiles = 0;
    sw.dev.max_dec = 0;
    // fast sweeps: lines with more tiles than two per thread get their carries
    // from k_fast_carries (fast_carried in finom_fast.hpp)
    const int carry_limit = sw.fast ? kFastFix * kCfgs[sw.cfg].block : INT32_MAX;
    std::vector<int> big;
    for (size_t li = 0; li < sw.lines.size(); ++li) {
        const LineDesc& L = sw.lines[li];
        if (L.ntiles > carry_limit) {
            big.push_back((int)li);
            continue;
        }
        sw.dev.max_tiles = std::max(sw.dev.max_tiles, L.ntiles);
        if (L.dec_part_off >= 0) sw.dev.max_dec = std::max(sw.dev.max_dec, L.dec_nparts);
    }
    sw.dev.nbig = (int)big.size();
    sw.dev.big = nullptr;
    sw.dev.carries = nullptr;
    if (!big.empty()) {
        int* hb = al.host<int>(big.size());
        std::copy(big.begin(), big.end(), hb);
        int* db = al.dev<int>(big.size());
        HIPCHK(hipMemcpyAsync(db, hb, sizeof(int) * big.size(), hipMemcpyHostToDevice, al.s));
        sw.dev.big = db;
        sw.dev.carries = al.dev<char>((size_t)std::max(mt, 1) * ns * ext_b);
    }
    sw.dev.work = dw;
    sw.dev.nwork = tt;
    sw.dev.work_multi = dm;
    sw.dev.nwork_multi = mt;
    sw.dev.lines = dl;
    sw.dev.agg = agg;
}

template <typename M, int B, int I, int INM, bool MO>
static void launch_agg_t(const SweepDev& d, ProbState* ps, const double* dec, int parity, hipStream_t s)
{
    hipLaunchKernelGGL((k_tile_aggregate<M, B, I, INM, MO>), dim3(d.nwork_multi), dim3(B), 0, s,
                       d.work_multi, d.lines, ps, (Ext<M>*)d.agg, dec, parity);
}

template <typename M, int B, int I, int INM, int EPI, bool MO, bool NA>
static void launch_t(const Sweep& sw, ProbState* ps, double* partial, const double* dec, int parity,
                     bool agg_only, hipStream_t s)
{
    const SweepDev& d = sw.dev;
    if (d.nwork == 0) return;
    if (d.nwork_multi > 0 && (agg_only || !sw.agg_from_prev)) {
        launch_agg_t<M, B, I, INM, MO>(d, ps, agg_only ? nullptr : dec, parity, s);
        if (!agg_only) dec = nullptr;   // the aggregate kernel took the decision
    }
    if (!agg_only)
        hipLaunchKernelGGL((k_sweep<M, B, I, INM, EPI, MO, NA>), dim3(d.nwork), dim3(B), 0, s, d.work,
                           d.lines, ps, (const Ext<M>*)d.agg, partial, dec, parity, (Ext<M>*)sw.agg_next);
    HIPCHK(hipGetLastError());
}

// Sweep variants of the scan path: (input mode, epilogue, next aggregates)
#define FINOM_VARIANTS(M, B, I)                                                                    \
    switch (variant) {                                                                              \
        case 0: launch_t<M, B, I, IN_LOG2, EPI_STORE_LOG2, false, false>(sw, ps, partial, dec, parity, ao, s); return; \
        case 1: launch_t<M, B, I, IN_LOG2, EPI_UPDATE, false, false>(sw, ps, partial, dec, parity, ao, s); return;     \
        case 2: launch_t<M, B, I, IN_LOG2, EPI_UPDATE, false, true>(sw, ps, partial, dec, parity, ao, s); return;      \
        case 3: launch_t<M, B, I, IN_LOG2, EPI_UPDATE_CHECK, false, false>(sw, ps, partial, dec, parity, ao, s); return; \
        case 4: launch_t<M, B, I, IN_LOG2, EPI_UPDATE_CHECK, false, true>(sw, ps, partial, dec, parity, ao, s); return;  \
        case 5: launch_t<M, B, I, IN_NAT, EPI_STORE_NAT, false, false>(sw, ps, partial, dec, parity, ao, s); return;   \
        case 6: launch_t<M, B, I, IN_LIN, EPI_STORE_LIN, false, false>(sw, ps, partial, dec, parity, ao, s); return;   \
    }

template <int B, int I, int EPI, bool NA>
static void launch_fast_t(const Sweep& sw, ProbState* ps, double* partial, const double* dec, int parity,
                          bool agg_only, hipStream_t s)
{
    const SweepDev& d = sw.dev;
    if (d.nwork == 0) return;
    if (d.nwork_multi > 0 && (agg_only || !sw.agg_from_prev))
        hipLaunchKernelGGL((k_tile_aggregate_fast<B, I>), dim3(d.nwork_multi), dim3(B), 0, s, d.work_multi, d.lines,
                           ps, (Ext<float>*)d.agg);
    if (!agg_only) {
        // the carried lines' carries (and their stop decision) first
        if (d.nbig > 0)
            hipLaunchKernelGGL((k_fast_carries<B>), dim3(d.nbig), dim3(B), 0, s, d.big, d.lines, ps,
                               (const Ext<float>*)d.agg, (Ext<float>*)d.carries, dec, parity);
        // two fixed slots per thread cover the other lines' carries and decision
        if (d.max_tiles > kFastFix * B || d.max_dec > kFastFix * B)
            hipLaunchKernelGGL((k_sweep_fast<B, I, EPI, NA, true>), dim3(d.nwork), dim3(B), 0, s, d.work, d.lines,
                               ps, (const Ext<float>*)d.agg, partial, dec, parity, (Ext<float>*)sw.agg_next,
                               (const Ext<float>*)d.carries);
        else
            hipLaunchKernelGGL((k_sweep_fast<B, I, EPI, NA, false>), dim3(d.nwork), dim3(B), 0, s, d.work, d.lines,
                               ps, (const Ext<float>*)d.agg, partial, dec, parity, (Ext<float>*)sw.agg_next,
                               (const Ext<float>*)d.carries);
    }
    HIPCHK(hipGetLastError());
}

template <int B, int I>
static void dispatch_fast(const Sweep& sw, ProbState* ps, double* partial, const double* dec, int parity, bool ao,
                          hipStream_t s)
{
    const bool na = sw.agg_next != nullptr;
    if (sw.epi == EPI_UPDATE) {
        if (na) launch_fast_t<B, I, EPI_UPDATE, true>(sw, ps, partial, dec, parity, ao, s);
        else launch_fast_t<B, I, EPI_UPDATE, false>(sw, ps, partial, dec, parity, ao, s);
    } else if (sw.epi == EPI_UPDATE_CHECK) {
        if (na) launch_fast_t<B, I, EPI_UPDATE_CHECK, true>(sw, ps, partial, dec, parity, ao, s);
        else launch_fast_t<B, I, EPI_UPDATE_CHECK, false>(sw, ps, partial, dec, parity, ao, s);
    } else {
        throw HipError{hipErrorInvalidValue};
    }
}

static int variant_of(int inm, int epi, bool next_agg)
{
    if (inm == IN_NAT && epi == EPI_STORE_NAT) return 5;
    if (inm == IN_LIN && epi == EPI_STORE_LIN) return 6;
    if (inm != IN_LOG2) return -1;
    switch (epi) {
        case EPI_STORE_LOG2: return next_agg ? -1 : 0;
        case EPI_UPDATE: return next_agg ? 2 : 1;
        case EPI_UPDATE_CHECK: return next_agg ? 4 : 3;
        default: return -1;
    }
}

static void dispatch(int precision, int inm, const Sweep& sw, ProbState* ps, double* partial,
                     const double* dec, int parity, bool ao, hipStream_t s)
{
    if (sw.kind == 2 || sw.kind == 1) {
        const bool mo = (sw.kind == 2);
        if (mo && sw.epi == EPI_COST)
            launch_t<double, kCostBlock, kCostIpt, IN_LOG2, EPI_COST, true, false>(sw, ps, partial, dec, parity, ao, s);
        else if (mo)
            launch_t<double, kCostBlock, kCostIpt, IN_LOG2, EPI_STORE_LOG2, true, false>(sw, ps, partial, dec, parity, ao, s);
        else if (sw.epi == EPI_COST)
            launch_t<double, kCostBlock, kCostIpt, IN_LOG2, EPI_COST, false, false>(sw, ps, partial, dec, parity, ao, s);
        else
            launch_t<double, kCostBlock, kCostIpt, IN_LOG2, EPI_STORE_LOG2, false, false>(sw, ps, partial, dec, parity, ao, s);
        return;
    }
    if (sw.fast) {
        if (precision != 1 || inm != IN_LOG2) throw HipError{hipErrorInvalidValue};
        switch (sw.cfg) {
            case 0: dispatch_fast<256, 4>(sw, ps, partial, dec, parity, ao, s); return;
            case 1: dispatch_fast<256, 8>(sw, ps, partial, dec, parity, ao, s); return;
            case 2: dispatch_fast<512, 8>(sw, ps, partial, dec, parity, ao, s); return;
            case 3: dispatch_fast<128, 4>(sw, ps, partial, dec, parity, ao, s); return;
            case 4: dispatch_fast<512, 4>(sw, ps, partial, dec, parity, ao, s); return;
        }
        throw HipError{hipErrorInvalidValue};
    }
    const int variant = variant_of(inm, sw.epi, sw.agg_next != nullptr);
    if (variant < 0) throw HipError{hipErrorInvalidValue};
    if (sw.cfg < 0 || sw.cfg >= kNumCfg) throw HipError{hipErrorInvalidValue};
    const int gcfg = kCfgs[sw.cfg].general;
    if (precision == 1) {
        switch (gcfg) {
            case 0: FINOM_VARIANTS(float, 256, 4) break;
            case 1: FINOM_VARIANTS(float, 256, 8) break;
            case 2: FINOM_VARIANTS(float, 512, 8) break;
            case 3: FINOM_VARIANTS(float, 128, 4) break;
            case 5: FINOM_VARIANTS(float, 64, 4) break;
        }
    } else {
        switch (gcfg) {
            case 0: FINOM_VARIANTS(double, 256, 4) break;
            case 1: FINOM_VARIANTS(double, 256, 8) break;
            case 2: FINOM_VARIANTS(double, 512, 8) break;
            case 3: FINOM_VARIANTS(double, 128, 4) break;
            case 5: FINOM_VARIANTS(double, 64, 4) break;
        }
    }
    throw HipError{hipErrorInvalidValue};
}
#undef FINOM_VARIANTS

void launch_sweep(int precision, int inm, const Sweep& sw, ProbState* ps, double* partial,
                  const double* dec, int parity, hipStream_t s)
{
    dispatch(precision, inm, sw, ps, partial, dec, parity, false, s);
}

void launch_aggregate(int precision, int inm, const Sweep& sw, ProbState* ps, hipStream_t s)
{
    if (sw.dev.nwork_multi == 0) return;
    dispatch(precision, inm, sw, ps, nullptr, nullptr, 0, true, s);
}

static std::atomic<int> g_tuned[2][kTuneClasses];
static std::once_flag g_tuned_once;

static void tuned_init()
{
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < kTuneClasses; ++c) g_tuned[p][c].store(-1);
}

int tune_class(long long merged)
{
    int c = 0;
    while (c < kTuneClasses - 1 && merged > (512LL << c)) ++c;
    return c;
}

void set_tuned_cfg(int precision, int cls, int cfg)
{
    std::call_once(g_tuned_once, tuned_init);
    if (precision < 0 || precision > 1 || cls < 0 || cls >= kTuneClasses) return;
    g_tuned[precision][cls].store((cfg >= 0 && cfg < kNumTunedCfg) ? cfg : -1);
}

int get_tuned_cfg(int precision, int cls)
{
    std::call_once(g_tuned_once, tuned_init);
    if (precision < 0 || precision > 1 || cls < 0 || cls >= kTuneClasses) return -1;
    return g_tuned[precision][cls].load();
}

static int forced_cfg()
{
    const char* e = getenv("FINOM_TILE_CFG");
    if (e && *e) {
        const int c = atoi(e);
        if (c >= 0 && c < kNumTunedCfg) return c;
    }
    return -1;
}

int short_line_cfg(int precision, long long merged)
{
    if (forced_cfg() < 0 && merged <= kCfgs[kShortCfg].T()) return kShortCfg;
    return tuned_cfg(precision, merged);
}

int tuned_cfg(int precision, long long merged)
{
    if (const int c = forced_cfg(); c >= 0) return c;
    const int t = get_tuned_cfg(precision, tune_class(merged));
    if (t >= 0) return t;
    return default_cfg(precision, merged);
}

int default_cfg(int precision, long long merged)
{
    // one tile per line when it fits; otherwise tiles of 2048, and of 4096
    // once 2048 would give more tiles than the resident solver holds at once
    if (merged <= 1024) return 0;
    (void)precision;
    return merged <= 512LL * 2048 ? 1 : 2;
}

// ---------------------------------------------------------------------------
// partitions and validation
// ---------------------------------------------------------------------------
Part make_part(Alloc& al, const double* xr, long long R, const double* yc, long long C, int T,
               hipStream_t s)
{
    Part p;
    p.xr = xr;
    p.R = R;
    p.yc = yc;
    p.C = C;
    p.T = T;
    p.ntiles = ntiles_for(R, C, T);
    p.zeta = al.dev<int>(R);
    p.trs = al.dev<int>(p.ntiles + 1);
    enqueue_partition(xr, R, yc, C, T, p.zeta, p.trs, s);
    return p;
}

void enqueue_partition(const double* xr, long long R, const double* yc, long long C, int T, int* zeta,
                       int* trs, hipStream_t s)
{
    const int ntiles = ntiles_for(R, C, T);
    hipLaunchKernelGGL(k_dividing_index, dim3(blocks_for(R)), dim3(kBlock), 0, s, xr, R, yc, C, zeta);
    hipLaunchKernelGGL(k_tile_rows, dim3(blocks_for(ntiles + 1)), dim3(kBlock), 0, s, zeta, R, T, ntiles, trs);
    HIPCHK(hipGetLastError());
}

Part make_part_like(Alloc& al, const Part& base, int T, hipStream_t s)
{
    Part p = base;
    p.T = T;
    p.ntiles = ntiles_for(p.R, p.C, T);
    p.trs = al.dev<int>(p.ntiles + 1);
    hipLaunchKernelGGL(k_tile_rows, dim3(blocks_for(p.ntiles + 1)), dim3(kBlock), 0, s, p.zeta, p.R, T,
                       p.ntiles, p.trs);
    HIPCHK(hipGetLastError());
    return p;
}

Part make_part_transposed(Alloc& al, const Part& base, hipStream_t s)
{
    Part p;
    p.xr = base.yc;
    p.R = base.C;
    p.yc = base.xr;
    p.C = base.R;
    p.T = base.T;
    p.ntiles = base.ntiles;
    p.zeta = al.dev<int>(p.R);
    p.trs = al.dev<int>(p.ntiles + 1);
    hipLaunchKernelGGL(k_dividing_index, dim3(blocks_for(p.R)), dim3(kBlock), 0, s, p.xr, p.R, p.yc, p.C,
                       p.zeta);
    hipLaunchKernelGGL(k_tile_rows_complement, dim3(blocks_for(p.ntiles + 1)), dim3(kBlock), 0, s, base.trs,
                       base.T, base.ntiles, base.R + base.C, p.trs);
    HIPCHK(hipGetLastError());
    return p;
}

void enqueue_sorted_check(const double* a, long long n, int* dflag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, dflag);
}

void enqueue_log2_mass(const double* a, long long n, double* la, int* dflag, hipStream_t s)
{
    hipLaunchKernelGGL(k_log2_mass, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, la, dflag);
}

void enqueue_sum(Alloc& al, const double* a, long long n, double* dsum, hipStream_t s)
{
    const int nb = 64;
    double* part = al.dev<double>(nb);
    hipLaunchKernelGGL(k_partial_sum, dim3(nb), dim3(kBlock), 0, s, a, n, part);
    hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, part, 0, nb, dsum);
}

void enqueue_fill(double* a, long long n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, v);
}

void enqueue_scale(const double* a, double* b, long long n, double f, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, b, n, f);
}

__global__ __launch_bounds__(kBlock) void k_fast_state(const FastStateTask* __restrict__ tasks,
                                                      const int* __restrict__ first, int ntasks)
{
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const FastStateTask t = tasks[lo];
    const long long k = (long long)(blockIdx.x - first[lo]) * kBlock + threadIdx.x;
    if (k >= t.n) return;
    if (t.mode == 0) {
        ((Ext<float>*)t.out)[k] = split_exp2(t.a + t.b * t.in[k]);
    } else if (t.mode == 1) {
        int e = 0;
        const double fr = frexp(t.in[k], &e);
        ((Ext<float>*)t.out)[k] = Ext<float>{(float)fr, e};
    } else if (t.mode == 2) {
        const Ext<float> u = ((const Ext<float>*)t.out)[k];
        ((double*)t.out)[k] =
            (u.m > 0.f) ? log2((double)u.m) + (double)u.e + t.b * t.mesh[k] : -__builtin_inf();
    } else if (t.mode == 3) {
        ((double*)t.out)[k] = log2(t.in[k]);
    } else {
        // the inverse of mode 2 in FP64: 2^(s - floor s) in [1, 2) rounded to
        // FP32 and normalised. A state that mode 2 converted comes back with
        // the same bits: the log form is off by at most 2^-27 in absolute
        // terms (|c kappa| < 2^25), well inside half an FP32 unit.
        const double s = ((const double*)t.out)[k] - t.b * t.mesh[k];
        Ext<float> u = ext_zero<float>();
        if (s > -__builtin_inf()) {
            const double fl = floor(s);
            u = ext_norm(Ext<float>{(float)exp2(s - fl), (int)fl});
        }
        ((Ext<float>*)t.out)[k] = u;
    }
}

void enqueue_fast_state(Alloc& al, const std::vector<FastStateTask>& tasks, hipStream_t s)
{
    if (tasks.empty()) return;
    const int nt = (int)tasks.size();
    FastStateTask* ht = al.host<FastStateTask>(nt);
    int* hf = al.host<int>(nt + 1);
    hf[0] = 0;
    for (int i = 0; i < nt; ++i) {
        ht[i] = tasks[i];
        hf[i + 1] = hf[i] + (int)blocks_for(tasks[i].n);
    }
    FastStateTask* dt = al.dev<FastStateTask>(nt);
    int* df = al.dev<int>(nt + 1);
    HIPCHK(hipMemcpyAsync(dt, ht, sizeof(FastStateTask) * nt, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(df, hf, sizeof(int) * (nt + 1), hipMemcpyHostToDevice, s));
    if (hf[nt] > 0) hipLaunchKernelGGL(k_fast_state, dim3(hf[nt]), dim3(kBlock), 0, s, dt, df, nt);
    HIPCHK(hipGetLastError());
}

__global__ void k_rearm(ProbState* __restrict__ p, long long l, long long itr_stop)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p->done = 0;
        p->converged = 0;
        p->tol = -1.0;
        p->itr_max = itr_stop;
        p->cnt[0] = l;
        p->cnt[1] = l;
        p->iters = l;
    }
}

void enqueue_rearm(ProbState* ps, long long l, long long itr_stop, hipStream_t s)
{
    hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, s, ps, l, itr_stop);
    HIPCHK(hipGetLastError());
}

bool fast_allowed()
{
    const char* e = getenv("FINOM_FAST");
    return !(e && e[0] == '0');
}


bool setup_fast_1d(Alloc& al, const Part& pk, const Part& pkt, double* lu, double* lv, const double* u,
                   const double* v, double eps, Ext<float>** Bx, Ext<float>** By, hipStream_t s,
                   bool convert_always)
{
    *Bx = *By = nullptr;
    const double kappa = 1.0 / (eps * kLn2);
    BoundTask* ht = al.host<BoundTask>(2);
    int* hfirst = al.host<int>(3);
    int* hflag = al.host<int>(1);
    memset(ht, 0, 2 * sizeof(BoundTask));
    // K psi: columns y with masses v; K^T phi: columns x with masses u
    ht[0].yc = pk.yc;
    ht[0].lmass = lv;
    ht[0].trs = pk.trs;
    ht[0].R = pk.R;
    ht[0].C = pk.C;
    ht[0].kappa = kappa;
    ht[0].T = pk.T;
    ht[0].ntiles = pk.ntiles;
    ht[1].yc = pkt.yc;
    ht[1].lmass = lu;
    ht[1].trs = pkt.trs;
    ht[1].R = pkt.R;
    ht[1].C = pkt.C;
    ht[1].kappa = kappa;
    ht[1].T = pkt.T;
    ht[1].ntiles = pkt.ntiles;
    hfirst[0] = 0;
    hfirst[1] = pk.ntiles;
    hfirst[2] = pk.ntiles + pkt.ntiles;
    BoundTask* dt = al.dev<BoundTask>(2);
    int* dfirst = al.dev<int>(3);
    int* dflag = al.dev<int>(1);
    HIPCHK(hipMemcpyAsync(dt, ht, 2 * sizeof(BoundTask), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dfirst, hfirst, 3 * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), s));
    hipLaunchKernelGGL((k_tile_bounds<kBlock>), dim3(hfirst[2]), dim3(kBlock), 0, s, dt, dfirst, 2, dflag);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const bool bounded = hflag[0] == 0;
    if (!bounded && !convert_always) return false;
    *Bx = al.dev<Ext<float>>(pk.R);
    *By = al.dev<Ext<float>>(pk.C);
    std::vector<FastStateTask> ft(4);
    memset(ft.data(), 0, ft.size() * sizeof(FastStateTask));
    ft[0].out = *Bx; ft[0].in = pk.xr; ft[0].n = pk.R; ft[0].b = 2.0 * kappa; ft[0].mode = 0;
    ft[1].out = *By; ft[1].in = pk.yc; ft[1].n = pk.C; ft[1].b = 2.0 * kappa; ft[1].mode = 0;
    ft[2].out = lu; ft[2].in = u; ft[2].n = pk.R; ft[2].mode = 1;
    ft[3].out = lv; ft[3].in = v; ft[3].n = pk.C; ft[3].mode = 1;
    enqueue_fast_state(al, ft, s);
    return bounded;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Reads the end points of the (sorted) meshes and checks that every exponent
// |coordinate| / (eps ln 2) stays below 2^25, the range the device exponent
// arithmetic is written for. Returns FINOM_OK or FINOM_E_ARG.
static int check_coord_range(Alloc& al, const double* const* meshes, const long long* sizes, int count,
                             double eps)
{
    double* h = al.host<double>(2 * count);
    for (int k = 0; k < count; ++k) {
        HIPCHK(hipMemcpyAsync(h + 2 * k, meshes[k], sizeof(double), hipMemcpyDeviceToHost, al.s));
        HIPCHK(hipMemcpyAsync(h + 2 * k + 1, meshes[k] + sizes[k] - 1, sizeof(double), hipMemcpyDeviceToHost,
                              al.s));
    }
    HIPCHK(hipStreamSynchronize(al.s));
    const double kappa = 1.0 / (eps * kLn2);
    for (int k = 0; k < 2 * count; ++k)
        if (!(fabs(h[k]) * kappa < kCoordLimit)) return FINOM_E_ARG;
    return FINOM_OK;
}

// ---------------------------------------------------------------------------
// the iteration loop: k iterations per captured graph, one state read per graph
// ---------------------------------------------------------------------------
// Sums the first n partial slots into slot n in the order of a block of dec's
// general sweep, so that the sum equals what each of its blocks would form
// (the decision's pre-reduction, wire_decision below).
static void launch_pre_reduce(const Sweep& dec, double* partial, int n, ProbState* ps, int parity, hipStream_t s)
{
    if (dec.cfg < 0 || dec.cfg >= kNumCfg || dec.lines.empty()) throw HipError{hipErrorInvalidValue};
    ProbState* P = ps + dec.lines[0].prob;
    switch (kCfgs[kCfgs[dec.cfg].general].block) {
        case 64: hipLaunchKernelGGL((k_reduce_partials_wide<64, 1024>), dim3(1), dim3(1024), 0, s, partial, 0, n, partial + n, P, parity); break;
        case 128: hipLaunchKernelGGL((k_reduce_partials_wide<128, 1024>), dim3(1), dim3(1024), 0, s, partial, 0, n, partial + n, P, parity); break;
        case 256: hipLaunchKernelGGL((k_reduce_partials_wide<256, 1024>), dim3(1), dim3(1024), 0, s, partial, 0, n, partial + n, P, parity); break;
        case 512: hipLaunchKernelGGL((k_reduce_partials_wide<512, 1024>), dim3(1), dim3(1024), 0, s, partial, 0, n, partial + n, P, parity); break;
        default: throw HipError{hipErrorInvalidValue};
    }
    HIPCHK(hipGetLastError());
}

struct LoopSpec {
    std::vector<Sweep*> seq[2];        // sweeps of one iteration, by iteration parity
    std::vector<bool> decides[2];      // sweep takes the stop decision
    std::vector<int> pre[2];           // partials summed ahead of the sweep (wire_decision), or 0
};

// on_stop (optional) runs when the state reports a stop; it returns true
// after re-arming the state for more iterations (a stop that the FP64 check
// rejected), and the replays go on.
// The loop of Algorithm 1 / 2: k iterations (body(parity, stream) enqueues
// one) captured in a HIP graph, replayed until the device state records a
// stop; on_stop may veto a stop and re-arm the state (the loop then goes on).
static int run_loop_fn(const std::function<void(int, hipStream_t)>& body, ProbState* ps, long long itr_max, int k,
                       hipStream_t s, ProbState* hps, finom_result* res, const std::function<bool()>& on_stop = {})
{
    k += (k & 1);   // even, so every replay starts on parity 0
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evs = nullptr;
    int st = FINOM_OK;
    try {
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < k; ++it) body(it & 1, cs);
        HIPCHK(hipStreamEndCapture(cs, &graph));
        HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        HIPCHK(hipEventCreate(&ev0));
        HIPCHK(hipEventCreate(&ev1));
        HIPCHK(hipEventCreateWithFlags(&evs, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev0, s));
        // One replay stays queued behind each state read, so the GPU runs it
        // while the host reads the state after the previous one. Once that
        // state records a stop, the queued replay changes nothing: every
        // kernel of the loop returns at once for a stopped problem.
        long long max_launches = itr_max / k + 3;
        long long launches = 0;
        auto replay = [&] {
            HIPCHK(hipGraphLaunch(exec, s));
            ++launches;
        };
        replay();
        for (;;) {
            HIPCHK(hipMemcpyAsync(hps, ps, sizeof(ProbState), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(evs, s));
            replay();
            HIPCHK(hipEventSynchronize(evs));
            if (hps->done) {
                HIPCHK(hipStreamSynchronize(s));   // the queued replay has run before the state is touched
                if (on_stop && on_stop()) {
                    ++max_launches;   // the resumed iteration may start a replay of its own
                    replay();
                    continue;
                }
                break;
            }
            if (launches > max_launches) {   // only if the device state were corrupt
                HIPCHK(hipStreamSynchronize(s));
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
        hipStreamSynchronize(s);   // no replay may still run once its graph is destroyed
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
    if (evs) hipEventDestroy(evs);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cs) hipStreamDestroy(cs);
    return st;
}

static int run_loop(const LoopSpec& lp, int precision, ProbState* ps, double* partial,
                    long long itr_max, int k, hipStream_t s, ProbState* hps, finom_result* res,
                    const std::function<bool()>& on_stop = {})
{
    auto body = [&](int b, hipStream_t cs) {
        for (size_t q = 0; q < lp.seq[b].size(); ++q) {
            if (q < lp.pre[b].size() && lp.pre[b][q] > 0) launch_pre_reduce(*lp.seq[b][q], partial, lp.pre[b][q], ps, b, cs);
            launch_sweep(precision, IN_LOG2, *lp.seq[b][q], ps, partial, lp.decides[b][q] ? partial : nullptr, b, cs);
        }
    };
    return run_loop_fn(body, ps, itr_max, k, s, hps, res, on_stop);
}

// ---- 2D loop on extended-number state (FP32 mode): line shapes (threads
// per line x points per thread), one block per line and the whole line one
// tile. By default the smallest shape that holds the longest axis mesh;
// FINOM_LINE_SHAPE (0..4) picks another that holds it.
struct LineShape {
    int block, ipt;
};
constexpr int kNumLineShapes = 5;
constexpr LineShape kLineShapes[kNumLineShapes] = {{64, 4}, {256, 4}, {256, 8}, {128, 8}, {64, 16}};

static int line_ext_shape(long long longest)
{
    int sh = longest <= 256 ? 0 : longest <= 1024 ? 1 : longest <= 2048 ? 2 : -1;
    if (sh < 0) return -1;
    if (const char* e = getenv("FINOM_LINE_SHAPE")) {
        const int v = atoi(e);
        if (v >= 0 && v < kNumLineShapes && kLineShapes[v].block * kLineShapes[v].ipt >= longest) sh = v;
    }
    return sh;
}

template <int B, int I>
static void launch_line_ext_t(const PassExt& d, bool s64, int nlines, ProbState* ps, hipStream_t s)
{
    if (s64) hipLaunchKernelGGL((k_line_ext<B, I, LX_STORE, true>), dim3(nlines), dim3(B), 0, s, d, ps, 0);
    else hipLaunchKernelGGL((k_line_ext<B, I, LX_STORE, false>), dim3(nlines), dim3(B), 0, s, d, ps, 0);
    HIPCHK(hipGetLastError());
}

template <int B, int I, bool S64>
static void launch_line_pair_s(const PairExt& pr, bool check, int nlines, ProbState* ps, int parity, hipStream_t s)
{
    if (check)
        hipLaunchKernelGGL((k_line_pair_ext<B, I, true, false, S64>), dim3(nlines), dim3(B), 0, s, pr, ps, parity);
    else
        hipLaunchKernelGGL((k_line_pair_ext<B, I, false, true, S64>), dim3(nlines), dim3(B), 0, s, pr, ps, parity);
}

template <int B, int I>
static void launch_line_pair_t(const PairExt& pr, bool s64, bool check, int nlines, ProbState* ps, int parity,
                               hipStream_t s)
{
    if (s64) launch_line_pair_s<B, I, true>(pr, check, nlines, ps, parity, s);
    else launch_line_pair_s<B, I, false>(pr, check, nlines, ps, parity, s);
    HIPCHK(hipGetLastError());
}

template <int B, int I, bool S64>
static void launch_line_pair_jobs_s(const PairExt* pairs, const int* first, int nprob, bool check, int nlines,
                                    ProbState* ps, int parity, hipStream_t s)
{
    if (check)
        hipLaunchKernelGGL((k_line_pair_ext_jobs<B, I, true, false, S64>), dim3(nlines), dim3(B), 0, s, pairs, first,
                           nprob, ps, parity);
    else
        hipLaunchKernelGGL((k_line_pair_ext_jobs<B, I, false, true, S64>), dim3(nlines), dim3(B), 0, s, pairs, first,
                           nprob, ps, parity);
}

template <int B, int I>
static void launch_line_pair_jobs_t(const PairExt* pairs, const int* first, int nprob, bool s64, bool check,
                                    int nlines, ProbState* ps, int parity, hipStream_t s)
{
    if (s64) launch_line_pair_jobs_s<B, I, true>(pairs, first, nprob, check, nlines, ps, parity, s);
    else launch_line_pair_jobs_s<B, I, false>(pairs, first, nprob, check, nlines, ps, parity, s);
    HIPCHK(hipGetLastError());
}

// One product storing W (the loop's prologue).
static void launch_line_ext(int shape, bool s64, const PassExt& d, int nlines, ProbState* ps, hipStream_t s)
{
    switch (shape) {
        case 0: launch_line_ext_t<64, 4>(d, s64, nlines, ps, s); break;
        case 1: launch_line_ext_t<256, 4>(d, s64, nlines, ps, s); break;
        case 2: launch_line_ext_t<256, 8>(d, s64, nlines, ps, s); break;
        case 3: launch_line_ext_t<128, 8>(d, s64, nlines, ps, s); break;
        default: launch_line_ext_t<64, 16>(d, s64, nlines, ps, s); break;
    }
}

// A pair of products per line: the update with the check (psi rows), or the
// update after the loop head's decision (phi columns).
static void launch_line_pair(int shape, bool s64, const PairExt& pr, bool check, int nlines, ProbState* ps,
                             int parity, hipStream_t s)
{
    switch (shape) {
        case 0: launch_line_pair_t<64, 4>(pr, s64, check, nlines, ps, parity, s); break;
        case 1: launch_line_pair_t<256, 4>(pr, s64, check, nlines, ps, parity, s); break;
        case 2: launch_line_pair_t<256, 8>(pr, s64, check, nlines, ps, parity, s); break;
        case 3: launch_line_pair_t<128, 8>(pr, s64, check, nlines, ps, parity, s); break;
        default: launch_line_pair_t<64, 16>(pr, s64, check, nlines, ps, parity, s); break;
    }
}

// The pairs of several problems of one line shape (k_line_pair_ext_jobs).
static void launch_line_pair_jobs(int shape, bool s64, const PairExt* pairs, const int* first, int nprob, bool check,
                                  int nlines, ProbState* ps, int parity, hipStream_t s)
{
    switch (shape) {
        case 0: launch_line_pair_jobs_t<64, 4>(pairs, first, nprob, s64, check, nlines, ps, parity, s); break;
        case 1: launch_line_pair_jobs_t<256, 4>(pairs, first, nprob, s64, check, nlines, ps, parity, s); break;
        case 2: launch_line_pair_jobs_t<256, 8>(pairs, first, nprob, s64, check, nlines, ps, parity, s); break;
        case 3: launch_line_pair_jobs_t<128, 8>(pairs, first, nprob, s64, check, nlines, ps, parity, s); break;
        default: launch_line_pair_jobs_t<64, 16>(pairs, first, nprob, s64, check, nlines, ps, parity, s); break;
    }
}

static void enqueue_grid_conv(const GridConv& c, hipStream_t s)
{
    const long long n = c.nx * c.ny;
    const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>((n + kConvBlock - 1) / kConvBlock, 65536));
    hipLaunchKernelGGL(k_grid_conv<0>, dim3(grid), dim3(kConvBlock), 0, s, c);
    HIPCHK(hipGetLastError());
}

// log2 potentials g <-> the extended state of a grid (see GridConv)
static void grid_to_ext(const double* g, double g0, Ext<float>* u, const double* X, const double* Y, long long nx,
                        long long ny, bool row_major, double kappa, hipStream_t s)
{
    GridConv c{};
    c.g = g;
    c.u = u;
    c.X = X;
    c.Y = Y;
    c.nx = nx;
    c.ny = ny;
    c.g0 = g0;
    c.kappa = kappa;
    c.row_major = row_major ? 1 : 0;
    c.to_ext = 1;
    enqueue_grid_conv(c, s);
}

static void grid_to_log2(const Ext<float>* u, double* g, const double* X, const double* Y, long long nx, long long ny,
                         bool row_major, double kappa, hipStream_t s)
{
    GridConv c{};
    c.gout = g;
    c.uin = u;
    c.X = X;
    c.Y = Y;
    c.nx = nx;
    c.ny = ny;
    c.kappa = kappa;
    c.row_major = row_major ? 1 : 0;
    c.to_ext = 0;
    enqueue_grid_conv(c, s);
}

int ext2d_shape(long long n1, long long m1, long long n2, long long m2, int precision)
{
    if (precision != 1 || !fast_allowed()) return -1;
    return line_ext_shape(std::max(std::max(n1, n2), std::max(m1, m2)));
}

size_t ext2d_bytes(long long n1, long long m1, long long n2, long long m2)
{
    const long long na = n1 * m1, nb = n2 * m2, ns = n2 * m1;
    const long long ext = 2 * na + 3 * nb + 2 * ns + n1 + n2 + m1 + m2;
    return sizeof(Ext<float>) * (size_t)ext + sizeof(double) * (size_t)n2 + 256 * 12;
}

void ext2d_bind(Ext2D& e, char* mem, long long n1, long long m1, long long n2, long long m2, int shape)
{
    e.shape = shape;
    e.n1 = n1;
    e.m1 = m1;
    e.n2 = n2;
    e.m2 = m2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = (off + 255) / 256 * 256;
        off = o + bytes;
        return mem + o;
    };
    const size_t eb = sizeof(Ext<float>);
    e.UF = (Ext<float>*)take(eb * n1 * m1);
    e.UG[0] = (Ext<float>*)take(eb * n2 * m2);
    e.UG[1] = (Ext<float>*)take(eb * n2 * m2);
    e.SX = (Ext<float>*)take(eb * n2 * m1);
    e.SY = (Ext<float>*)take(eb * n2 * m1);
    e.Au = (Ext<float>*)take(eb * n1 * m1);
    e.Av = (Ext<float>*)take(eb * n2 * m2);
    e.B[0] = (Ext<float>*)take(eb * n1);
    e.B[1] = (Ext<float>*)take(eb * n2);
    e.B[2] = (Ext<float>*)take(eb * m1);
    e.B[3] = (Ext<float>*)take(eb * m2);
    e.part = (double*)take(sizeof(double) * n2);
}

void ext2d_setup(Ext2D& e, const Part& px, const Part& px_t, const Part& py, const Part& py_t, int prob)
{
    const long long n1 = e.n1, m1 = e.m1, n2 = e.n2, m2 = e.m2;
    Ext<float>* const Bx1 = e.B[0];
    Ext<float>* const Bx2 = e.B[1];
    Ext<float>* const By1 = e.B[2];
    Ext<float>* const By2 = e.B[3];
    // prologue: SX = K_x^T phi along x (line b < m1: column b of phi) into
    // the row-major intermediate
    PassExt& t0 = e.pro;
    t0 = PassExt{};
    t0.uin = e.UF; t0.uin_line = n1; t0.bc = Bx1; t0.br = Bx2; t0.zeta = px_t.zeta;
    t0.out = e.SX; t0.out_line = 1; t0.out_elem = m1; t0.R = (int)n2; t0.C = (int)n1; t0.prob = prob;
    for (int b = 0; b < 2; ++b) {
        // per psi row c < n2: psi = v / (row c of SX) K_y with the check, then
        // row c of Psi K_y^T into the column-major SY
        PairExt& y = e.y[b];
        y = PairExt{};
        PassExt& t = y.p1;
        t.uin = e.SX; t.uin_line = m1; t.bc = By1; t.br = By2; t.zeta = py_t.zeta;
        t.out = e.UG[1 - b]; t.out_line = m2; t.out_elem = 1; t.a = e.Av; t.a_line = m2; t.uold = e.UG[b];
        t.partial = e.part; t.R = (int)m2; t.C = (int)m1; t.prob = prob;
        y.br2 = By1; y.zeta2 = py.zeta; y.out2 = e.SY; y.out2_line = 1; y.out2_elem = n2; y.R2 = (int)m1;
        // per phi column b < m1, after the loop head's decision: phi = u / K_x
        // (column b of SY), then K_x^T phi into SX for the next pair
        PairExt& x = e.x[b];
        x = PairExt{};
        PassExt& k = x.p1;
        k.uin = e.SY; k.uin_line = n2; k.bc = Bx2; k.br = Bx1; k.zeta = px.zeta;
        k.out = e.UF; k.out_line = n1; k.out_elem = 1; k.a = e.Au; k.a_line = n1; k.R = (int)n1; k.C = (int)n2;
        k.dec = e.part; k.dec_n = (int)n2; k.prob = prob;
        x.br2 = Bx2; x.zeta2 = px_t.zeta; x.out2 = e.SX; x.out2_line = 1; x.out2_elem = m1; x.R2 = (int)n2;
    }
}

// Whether every chunk of every axis mesh (64 IPT consecutive columns of a
// line, plus one neighbour on each side) spans at most kSpan64 binary orders
// of kernel decay: 2 kappa (c_last - c_first) (FINOM_LINE_SCAN=ext turns
// the FP64 scan off).
static bool ext2d_scan64(const double* const* axes, const long long* lens, int chunk, double kappa)
{
    if (const char* e = getenv("FINOM_LINE_SCAN"))
        if (strcmp(e, "ext") == 0) return false;
    for (int a = 0; a < 4; ++a) {
        std::vector<double> h((size_t)lens[a]);
        HIPCHK(hipMemcpy(h.data(), axes[a], sizeof(double) * lens[a], hipMemcpyDeviceToHost));
        for (long long c0 = 0; c0 < lens[a]; c0 += chunk) {
            const long long lo = std::max(c0 - 1, 0LL), hi = std::min(c0 + chunk, lens[a] - 1);
            if (!(2.0 * kappa * (h[hi] - h[lo]) <= kSpan64)) return false;
        }
    }
    return true;
}

void ext2d_init(Ext2D& e, const double* x1, const double* x2, const double* y1, const double* y2,
                const double* lu, const double* lvr, double kappa, hipStream_t s)
{
    const double* axes[4] = {x1, x2, y1, y2};
    const long long lens[4] = {e.n1, e.n2, e.m1, e.m2};
    HIPCHK(hipStreamSynchronize(s));   // the meshes are read on the host (they are inputs: nothing pending writes them)
    e.s64 = ext2d_scan64(axes, lens, kWave * kLineShapes[e.shape].ipt, kappa) ? 1 : 0;
    for (int a = 0; a < 4; ++a)
        hipLaunchKernelGGL(k_axis_b<0>, dim3(std::max(1u, std::min(blocks_for(lens[a], kConvBlock), 65536u))),
                           dim3(kConvBlock), 0, s, axes[a], lens[a], kappa, e.B[a]);
    HIPCHK(hipGetLastError());
    const long long na = e.n1 * e.m1, nb = e.n2 * e.m2;
    grid_to_ext(nullptr, -log2((double)na), e.UF, x1, y1, e.n1, e.m1, false, kappa, s);
    grid_to_ext(nullptr, -log2((double)nb), e.UG[0], x2, y2, e.n2, e.m2, true, kappa, s);
    grid_to_ext(lu, 0.0, e.Au, nullptr, nullptr, e.n1, e.m1, false, 0.0, s);
    grid_to_ext(lvr, 0.0, e.Av, nullptr, nullptr, e.n2, e.m2, true, 0.0, s);
}

void ext2d_prologue(const Ext2D& e, ProbState* ps, hipStream_t s)
{
    launch_line_ext(e.shape, e.s64 != 0, e.pro, (int)e.m1, ps, s);
}

void ext2d_group_iteration(const Ext2DGroup& g, int parity, ProbState* ps, hipStream_t s)
{
    if (g.nprob == 0) return;
    launch_line_pair_jobs(g.shape, g.s64 != 0, g.y[parity], g.fy, g.nprob, true, g.ny, ps, parity, s);
    launch_line_pair_jobs(g.shape, g.s64 != 0, g.x[parity], g.fx, g.nprob, false, g.nx, ps, parity, s);
}

void ext2d_iteration(const Ext2D& e, int parity, ProbState* ps, hipStream_t s)
{
    launch_line_pair(e.shape, e.s64 != 0, e.y[parity], true, (int)e.n2, ps, parity, s);
    launch_line_pair(e.shape, e.s64 != 0, e.x[parity], false, (int)e.m1, ps, parity, s);
}



void ext2d_to_log2(const Ext2D& e, int bo, double* F, double* G, const double* x1, const double* x2,
                   const double* y1, const double* y2, double kappa, hipStream_t s)
{
    grid_to_log2(e.UF, F, x1, y1, e.n1, e.m1, false, kappa, s);
    grid_to_log2(e.UG[bo], G, x2, y2, e.n2, e.m2, true, kappa, s);
}

static int default_graph_iters(long long points)
{
    if (points <= (1 << 14)) return 64;
    if (points <= (1 << 18)) return 32;
    return 16;
}

static void init_state(Alloc& al, ProbState* ps, ProbState* hps, int count, long long itr_max,
                       double tol)
{
    for (int i = 0; i < count; ++i) {
        memset(hps + i, 0, sizeof(ProbState));
        hps[i].itr_max = itr_max;
        hps[i].tol = tol;
    }
    HIPCHK(hipMemcpyAsync(ps, hps, count * sizeof(ProbState), hipMemcpyHostToDevice, al.s));
}

// Reads the validation flags and mass sums; returns a status.
static int read_checks(Alloc& al, int* dflag, double* dsum)
{
    int* hflag = al.host<int>(4);
    double* hsum = al.host<double>(2);
    HIPCHK(hipMemcpyAsync(hflag, dflag, 4 * sizeof(int), hipMemcpyDeviceToHost, al.s));
    HIPCHK(hipMemcpyAsync(hsum, dsum, 2 * sizeof(double), hipMemcpyDeviceToHost, al.s));
    HIPCHK(hipStreamSynchronize(al.s));
    if (hflag[0]) return FINOM_E_UNSORTED;
    if (hflag[1]) return FINOM_E_MASS;
    if (!(fabs(hsum[0] - hsum[1]) <= 1e-12 * std::max(fabs(hsum[0]), fabs(hsum[1]))))
        return FINOM_E_MASS;
    return FINOM_OK;
}

static void finish_result(finom_result* res, const ProbState& st, double w1)
{
    res->w1 = w1;
    res->marginal_err = st.err;
    res->iters = st.iters;
    res->sweeps = 2 * st.iters + 1;
    res->converged = st.converged;
}

static void set_decision(Sweep& sw, int off, int n)
{
    for (size_t i = 0; i < sw.lines.size(); ++i) {
        sw.lines[i].dec_part_off = off;
        sw.lines[i].dec_nparts = n;
        sw.lines[i].writes_state = (i == 0) ? 1 : 0;
    }
}

// A checking sweep of many lines leaves one partial error per tile, and every
// block of the deciding sweep would sum all of them (quadratic in the lines:
// 16384 blocks x 16384 partials on a 128^3 grid). Beyond kPreReduceMin
// partials one block sums them first, in the order a deciding block uses (the
// same value), and takes the decision from it as every deciding block would;
// the deciding sweep's blocks then only test whether the problem has stopped.
constexpr int kPreReduceMin = 1024;

// Wires the decision of sweep dec to the nchk partials of its checking sweep
// (slots [0, nchk)). Returns how many to sum ahead of it into slot nchk, or 0.
static int wire_decision(Sweep& dec, int nchk)
{
    const bool pre = nchk > kPreReduceMin && dec.kind == 0 && !dec.fast;
    // pre-reduced: the summing kernel takes the decision, the sweep none
    set_decision(dec, pre ? -1 : 0, pre ? 0 : nchk);
    return pre ? nchk : 0;
}


// ---- resident solver: eligibility

bool resident_allowed()
{
    const char* e = getenv("FINOM_RESIDENT");
    return !(e && e[0] == '0');
}

const void* resident_kernel(bool gen)
{
    return gen ? (const void*)k_resident_1d<kResidentBlockGen, kResidentIptGen, kResidentWavesGen, true>
               : (const void*)k_resident_1d<kResidentBlock, kResidentIpt, kResidentWaves, false>;
}

// The smaller of the two kernels' capacities, so that a problem is resident
// alone exactly when it is resident in a batch. Computed once per process on
// the device current at the first call.
int resident_capacity(bool gen)
{
    static int cap[2] = {-1, -1};
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    int& c = cap[gen ? 1 : 0];
    if (c < 0) {
        int dev = 0, coop = 0, cus = 0, per_cu = 0;
        c = 0;
        const void* k = resident_kernel(gen);
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, resident_block(gen), 0) == hipSuccess)
            c = std::min(cus * per_cu, resident_batch_capacity(gen));
    }
    return c;
}

// Tiles of T (at most the kernel's slots per block), at most one record per
// thread and all resident at once.
bool resident_fits(long long n, long long m, int T, bool gen)
{
    if (!resident_allowed() || T < 1 || T > kResidentSlots) return false;
    const long long nt = (n + m + T - 1) / T;
    return nt >= 1 && nt <= kResidentMaxTiles && nt <= resident_capacity(gen);
}

}  // namespace finom

using namespace finom;

// ---------------------------------------------------------------------------
// matvec
// ---------------------------------------------------------------------------
static int matvec_impl(bool dense, const double* x, int64_t n, const double* y, int64_t m,
                       double eps, const double* in, double* out, const finom_opts* opts,
                       void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!x || !y || !in || !out || n < 1 || m < 1 || !finite_pos(eps)) return FINOM_E_ARG;
    if (o.precision < 0 || o.precision > 2) return FINOM_E_ARG;
    if (o.domain != 0 && o.domain != 1) return FINOM_E_ARG;
    if (o.precision == 2 && (dense || o.domain != 0)) return FINOM_E_ARG;   // the linear mode is linear
    if (n + m > (int64_t)INT32_MAX) return FINOM_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        if (!o.skip_checks) {
            int* dflag = al.dev<int>(1);
            int* hflag = al.host<int>(1);
            HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), s));
            enqueue_sorted_check(x, n, dflag, s);
            enqueue_sorted_check(y, m, dflag, s);
            HIPCHK(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hflag[0]) return FINOM_E_UNSORTED;
            const double* ms[2] = {x, y};
            const long long ns[2] = {n, m};
            if (check_coord_range(al, ms, ns, 2, eps) != FINOM_OK) return FINOM_E_ARG;
        }
        const int inm = (o.domain == 1) ? IN_NAT : IN_LIN;
        const double kappa = 1.0 / (eps * kLn2);
        if (dense) {
#define DK(M, I, LIN)                                                                               \
    hipLaunchKernelGGL((k_dense<M, I>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, y, \
                       (long long)m, in, kappa, kappa, eps * kLn2, LIN, out)
            if (o.precision == 1) {
                if (inm == IN_NAT) DK(float, IN_NAT, 0);
                else DK(float, IN_LIN, 1);
            } else {
                if (inm == IN_NAT) DK(double, IN_NAT, 0);
                else DK(double, IN_LIN, 1);
            }
#undef DK
            HIPCHK(hipGetLastError());
            return FINOM_OK;
        }
        if (o.precision == 2) {
            const int cfg = tuned_cfg(0, n + m);
            const Part p = make_part(al, x, n, y, m, kCfgs[cfg].T(), s);
            linear_matvec(al, p, eps, in, out, cfg, s);
            al.uploaded();
            return FINOM_OK;
        }
        const int cfg = tuned_cfg(o.precision, n + m);
        const int T = kCfgs[cfg].T();
        Part p = make_part(al, x, n, y, m, T, s);
        ProbState* ps = al.dev<ProbState>(1);
        HIPCHK(hipMemsetAsync(ps, 0, sizeof(ProbState), s));
        Sweep sw;
        sw.kind = 0;
        sw.cfg = cfg;
        sw.epi = (o.domain == 1) ? EPI_STORE_NAT : EPI_STORE_LIN;
        LineDesc L = make_line(x, n, y, m, p.zeta, p.trs, T, eps);
        L.gin = in;
        L.out = out;
        L.dec_part_off = -1;
        sw.lines.push_back(L);
        upload_sweep(al, sw, ext_bytes(o.precision));
        al.uploaded();
        launch_sweep(o.precision, inm, sw, ps, nullptr, nullptr, 0, s);
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

extern "C" {

int finom_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m, double eps,
                 const double* in, double* out, const finom_opts* opts, void* stream)
{
    return matvec_impl(false, x_rows, n, y_cols, m, eps, in, out, opts, stream);
}

int dense_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m, double eps,
                 const double* in, double* out, const finom_opts* opts, void* stream)
{
    return matvec_impl(true, x_rows, n, y_cols, m, eps, in, out, opts, stream);
}

// ---------------------------------------------------------------------------
// Resident-state solver (one cooperative launch per solve)
// ---------------------------------------------------------------------------


// Runs the whole loop; the final phi is left in UF and the returned psi in UG
// (both as the fast state).
static int run_resident(Alloc& al, const Part& pk, const Part& pkt, Ext<float>* UF, Ext<float>* UG,
                        const Ext<float>* Ax, const Ext<float>* Ay, const Ext<float>* Bx, const Ext<float>* By,
                        ProbState* ps, ProbState* hps, hipStream_t s, finom_result* res, bool gen)
{
    ResidentArgs a;
    memset(&a, 0, sizeof(a));
    a.UF = UF;
    a.UG = UG;
    a.Ax = Ax;
    a.Ay = Ay;
    a.Bx = Bx;
    a.By = By;
    a.zx = pk.zeta;
    a.zy = pkt.zeta;
    a.trs = pk.trs;
    a.n = pk.R;
    a.m = pk.C;
    a.ntiles = pk.ntiles;
    a.T = pk.T;
    a.rec = al.dev<unsigned long long>(5 * (size_t)pk.ntiles);
    a.fail = al.dev<int>(1);
    // records start at zero (tag 0: written 0 times)
    HIPCHK(hipMemsetAsync(a.rec, 0, 5 * (size_t)pk.ntiles * sizeof(unsigned long long), s));
    HIPCHK(hipMemsetAsync(a.fail, 0, sizeof(int), s));
    a.ps = ps;
    a.spin_limit = kResidentSpin;
    if (const char* e = getenv("FINOM_RESIDENT_SPIN")) a.spin_limit = (unsigned)strtoul(e, nullptr, 10);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int st = FINOM_OK;
    try {
        HIPCHK(hipEventCreate(&ev0));
        HIPCHK(hipEventCreate(&ev1));
        HIPCHK(hipEventRecord(ev0, s));
        void* args[] = {&a};
        HIPCHK(hipLaunchCooperativeKernel(resident_kernel(gen), dim3(pk.ntiles), dim3(resident_block(gen)), args, 0,
                                          s));
        HIPCHK(hipEventRecord(ev1, s));
        int* hfail = al.host<int>(1);
        HIPCHK(hipMemcpyAsync(hfail, a.fail, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hps, ps, sizeof(ProbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
        res->loop_ms = ms;
        if (*hfail) {
            st = FINOM_E_HIP;
            snprintf(g_last_error, sizeof(g_last_error), "resident solver: a grid wait exceeded its bound");
        }
    } catch (...) {
        st = map_exception();
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    return st;
}

// ---------------------------------------------------------------------------
// Algorithm 1
// ---------------------------------------------------------------------------
int sinkhorn_w1_1d(const double* x, int64_t n, const double* y, int64_t m, const double* u,
                   const double* v, double eps, double tol, int64_t itr_max, const finom_opts* opts,
                   double* f_out, double* g_out, finom_result* res, void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!res) return FINOM_E_ARG;
    memset(res, 0, sizeof(*res));
    auto fail = [&](int st) {
        res->status = st;
        return st;
    };
    if (!x || !y || !u || !v || n < 1 || m < 1 || !finite_pos(eps)) return fail(FINOM_E_ARG);
    if (!(tol >= 0.0) || !std::isfinite(tol) || itr_max < 0) return fail(FINOM_E_ARG);
    if (o.precision < 0 || o.precision > 2) return fail(FINOM_E_ARG);
    if (n + m > (int64_t)INT32_MAX) return fail(FINOM_E_ARG);
    hipStream_t s = (hipStream_t)stream;
    const bool linear = o.precision == 2;
    try {
        Alloc al(stream);
        // the tile shape does not depend on the kernel that runs the tiles,
        // so a problem gets the same tiles alone and in a batch (the linear
        // mode takes the FP64 table's shapes)
        const int cfg = tuned_cfg(linear ? 0 : o.precision, n + m);
        const int T = kCfgs[cfg].T();
        const bool try_resident = o.precision == 1 && fast_allowed() && resident_fits(n, m, T, false);
        const bool try_gen = o.precision == 1 && fast_allowed() && resident_fits(n, m, T, true);
        const size_t eb = ext_bytes(o.precision);

        // validation and log masses
        int* dflag = al.dev<int>(4);
        double* dsum = al.dev<double>(2);
        double* lu = al.dev<double>(n);
        double* lv = al.dev<double>(m);
        HIPCHK(hipMemsetAsync(dflag, 0, 4 * sizeof(int), s));
        if (!o.skip_checks) {
            enqueue_sorted_check(x, n, dflag, s);
            enqueue_sorted_check(y, m, dflag, s);
        }
        enqueue_log2_mass(u, n, lu, dflag + 1, s);
        enqueue_log2_mass(v, m, lv, dflag + 1, s);
        enqueue_sum(al, u, n, dsum, s);
        enqueue_sum(al, v, m, dsum + 1, s);
        if (!o.skip_checks) {
            int st = read_checks(al, dflag, dsum);
            if (st == FINOM_OK) {
                const double* ms[2] = {x, y};
                const long long ns[2] = {n, m};
                st = check_coord_range(al, ms, ns, 2, eps);
            }
            if (st != FINOM_OK) return fail(st);
        }
        if (linear) {
            // the linear mode's scalings fit FP64 only for diam / eps <= 600
            double* h = al.host<double>(4);
            HIPCHK(hipMemcpyAsync(h, x, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(h + 1, x + n - 1, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(h + 2, y, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(h + 3, y + m - 1, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!linear_span_ok(std::min(h[0], h[2]), std::max(h[1], h[3]), eps)) {
                set_last_error("linear mode (precision 2): diam / eps exceeds 600");
                return fail(FINOM_E_ARG);
            }
        }

        // dividing indices (Algorithm 1, first step) on one merge-path
        // partition shared by both products
        const Part pk = make_part(al, x, n, y, m, T, s);      // K psi:   rows x, columns y
        const Part pkt = make_part_transposed(al, pk, s);     // K^T phi: rows y, columns x
        const Part pc = make_part_like(al, pk, cost_tile_size(), s);
        Ext<float>* Bx = nullptr;
        Ext<float>* By = nullptr;
        const bool fast = o.precision == 1 && fast_allowed() &&
                          setup_fast_1d(al, pk, pkt, lu, lv, u, v, eps, &Bx, &By, s, try_gen);
        // tiles beyond the fast bound: the resident solver's extended-number
        // variant, on the same state representation
        const bool gen = !fast && try_gen;
        const bool ext_state = fast || gen;
        const double kappa = 1.0 / (eps * kLn2);

        // state: phi = 1/n, psi = 1/m, as log2 potentials, or for the fast
        // sweeps as U = w 2^{-c kappa} in the same buffers
        double* F = al.dev<double>(n);
        double* G[2] = {al.dev<double>(m), al.dev<double>(m)};
        if (ext_state) {
            std::vector<FastStateTask> ft(2);
            memset(ft.data(), 0, ft.size() * sizeof(FastStateTask));
            ft[0].out = F; ft[0].in = x; ft[0].n = n; ft[0].a = -log2((double)n); ft[0].b = -kappa;
            ft[1].out = G[0]; ft[1].in = y; ft[1].n = m; ft[1].a = -log2((double)m); ft[1].b = -kappa;
            enqueue_fast_state(al, ft, s);
        } else if (!linear) {
            enqueue_fill(F, n, -log2((double)n), s);
            enqueue_fill(G[0], m, -log2((double)m), s);
        }
        ProbState* ps = al.dev<ProbState>(2);      // [0] iteration, [1] cost
        ProbState* hps = al.host<ProbState>(2);
        init_state(al, ps, hps, 2, itr_max, tol);
        const bool resident = (try_resident && fast) || gen;
        const int nparts = std::max(pkt.ntiles, pc.ntiles);
        double* partial = al.dev<double>(nparts);

        // FP32 mode: every stop is confirmed by the FP64 check of the pair it
        // returns (K^T phi with FP64 scans), with the state in log form
        const bool confirm = o.precision == 1;
        double* part64 = confirm ? al.dev<double>(pkt.ntiles) : nullptr;
        double* err64_d = confirm ? al.dev<double>(1) : nullptr;
        double* err64_h = confirm ? al.host<double>(1) : nullptr;
        Sweep chk64[2];   // by the buffer holding the checked psi
        for (int bo = 0; bo < 2 && confirm; ++bo) {
            chk64[bo].epi = EPI_UPDATE_CHECK;
            chk64[bo].cfg = cfg;
            LineDesc a = make_line(y, m, x, n, pkt.zeta, pkt.trs, T, eps);
            a.gin = F; a.out = G[1 - bo]; a.a0 = lv; a.a1 = v; a.a2 = G[bo];
            a.prob = 1;
            a.dec_part_off = -1;
            chk64[bo].lines.push_back(a);
            assign_parts(chk64[bo], 0);
            upload_sweep(al, chk64[bo], sizeof(Ext<double>));
        }
        int shift = 0;          // psi of iteration l in G[(l & 1) ^ shift] (streaming loop)
        int resumes = 0;
        long long last_l = -1;   // iteration of the last rejected stop
        long long step = 0;      // iterations run after it
        double err64 = 0.0;
        // the pair in (F, G[bo]) to FP64 log form (and log2 v beside it) or back
        auto ext_convert = [&](int bo, bool to_log) {
            std::vector<FastStateTask> ft(3);
            memset(ft.data(), 0, ft.size() * sizeof(FastStateTask));
            ft[0].out = F; ft[0].mesh = x; ft[0].n = n; ft[0].b = kappa; ft[0].mode = to_log ? 2 : 4;
            ft[1].out = G[bo]; ft[1].mesh = y; ft[1].n = m; ft[1].b = kappa; ft[1].mode = to_log ? 2 : 4;
            ft[2].out = lv; ft[2].in = v; ft[2].n = m; ft[2].mode = to_log ? 3 : 1;
            enqueue_fast_state(al, ft, s);
        };
        // Called at a stop (hps[0] read): true when the loop is re-armed
        auto on_stop = [&]() -> bool {
            const long long l = hps[0].iters;
            const int bo = resident ? 0 : psi_slot(l, shift);
            if (ext_state) ext_convert(bo, true);
            launch_sweep(0, IN_LOG2, chk64[bo], ps, part64, nullptr, 0, s);
            hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, part64, 0, pkt.ntiles,
                               err64_d);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(err64_h, err64_d, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            err64 = *err64_h;
            if (!(err64 > tol) || l >= itr_max || !std::isfinite(err64) || hps[0].status ||
                !may_resume(l, last_l))
                return false;
            // resume from the same pair, in its own representation
            if (ext_state) ext_convert(bo, false);
            if (bo == 1) HIPCHK(hipMemcpyAsync(G[0], G[1], sizeof(double) * m, hipMemcpyDeviceToDevice, s));
            shift = (int)(l & 1);
            step = resume_step(step);
            enqueue_rearm(ps, l, resume_until(l, step, itr_max), s);
            last_l = l;
            ++resumes;
            return true;
        };
        if (resident) {
            al.uploaded();
            double ms_total = 0.0;
            for (;;) {
                const int st = run_resident(al, pk, pkt, (Ext<float>*)F, (Ext<float>*)G[0], (const Ext<float>*)lu,
                                            (const Ext<float>*)lv, Bx, By, ps, hps, s, res, gen);
                if (st != FINOM_OK) return fail(st);
                ms_total += res->loop_ms;
                if (!on_stop()) break;
            }
            res->loop_ms = ms_total;
        }
        int lin_psi = 0;
        if (linear) {
            al.uploaded();
            const int kit = o.graph_iters > 0 ? o.graph_iters : default_graph_iters((n + m) / 2);
            const int st = linear_loop(al, pk, pkt, cfg, u, v, eps, itr_max, kit, F, G, ps, hps, s, res, &lin_psi);
            if (st != FINOM_OK) return fail(st);
            // the returned pair to log2 potentials for the cost and the outputs
            std::vector<FastStateTask> ft(2);
            memset(ft.data(), 0, ft.size() * sizeof(FastStateTask));
            ft[0].out = F; ft[0].in = F; ft[0].n = n; ft[0].mode = 3;
            ft[1].out = G[lin_psi]; ft[1].in = G[lin_psi]; ft[1].n = m; ft[1].mode = 3;
            enqueue_fast_state(al, ft, s);
        }
        // tile aggregates: each product's epilogue writes the other's
        const bool multi = pk.ntiles > 1;
        void* agg_k = multi ? (void*)al.dev<char>((size_t)pk.ntiles * 2 * eb) : nullptr;
        void* agg_kt = multi ? (void*)al.dev<char>((size_t)pk.ntiles * 2 * eb) : nullptr;

        Sweep kt[2], kk[2];
        for (int b = 0; b < 2 && !resident && !linear; ++b) {
            kt[b].epi = EPI_UPDATE_CHECK;
            kt[b].cfg = cfg;
            kt[b].agg_from_prev = multi;
            kt[b].agg_buf = agg_kt;
            kt[b].agg_next = agg_k;
            LineDesc a = make_line(y, m, x, n, pkt.zeta, pkt.trs, T, eps);
            a.gin = F; a.out = G[1 - b]; a.a0 = lv; a.a1 = v; a.a2 = G[b];
            a.er = By; a.ec = Bx;
            a.dec_part_off = -1;
            kt[b].fast = kk[b].fast = fast;
            kt[b].lines.push_back(a);
            assign_parts(kt[b], 0);
            kk[b].epi = EPI_UPDATE;
            kk[b].cfg = cfg;
            kk[b].agg_from_prev = multi;
            kk[b].agg_buf = agg_k;
            kk[b].agg_next = agg_kt;
            LineDesc c = make_line(x, n, y, m, pk.zeta, pk.trs, T, eps);
            c.gin = G[1 - b]; c.out = F; c.a0 = lu;
            c.er = Bx; c.ec = By;
            kk[b].lines.push_back(c);
            set_decision(kk[b], 0, pkt.ntiles);
            upload_sweep(al, kt[b], eb);
            upload_sweep(al, kk[b], eb);
        }
        if (!resident && !linear) {
            al.uploaded();
            // aggregates of the initial phi for the first K^T phi
            launch_aggregate(o.precision, IN_LOG2, kt[0], ps, s);

            LoopSpec lp;
            for (int b = 0; b < 2; ++b) {
                lp.seq[b] = {&kt[b], &kk[b]};
                lp.decides[b] = {false, true};
            }
            const int kit = o.graph_iters > 0 ? o.graph_iters : default_graph_iters((n + m) / 2);
            const int st = run_loop(lp, o.precision, ps, partial, itr_max, kit, s, hps, res,
                                    confirm ? std::function<bool()>(on_stop) : std::function<bool()>());
            if (st != FINOM_OK) return fail(st);
        }

        // returned pair (F, G[psi_slot]) (the resident solver leaves it in
        // (F, G[0])), in log form (the FP64 check has converted it already);
        // <C, Gamma> from the FP64 moment sums
        double* Gf = linear ? G[lin_psi] : resident ? G[0] : G[psi_slot(hps[0].iters, shift)];
        if (ext_state && !confirm) {
            std::vector<FastStateTask> ft(2);
            memset(ft.data(), 0, ft.size() * sizeof(FastStateTask));
            ft[0].out = F; ft[0].mesh = x; ft[0].n = n; ft[0].b = kappa; ft[0].mode = 2;
            ft[1].out = Gf; ft[1].mesh = y; ft[1].n = m; ft[1].b = kappa; ft[1].mode = 2;
            enqueue_fast_state(al, ft, s);
        }
        Sweep kc;
        kc.kind = 2;
        kc.epi = EPI_COST;
        LineDesc c = make_line(x, n, y, m, pc.zeta, pc.trs, pc.T, eps);
        c.gin = Gf; c.a0 = F; c.prob = 1; c.dec_part_off = -1;
        kc.lines.push_back(c);
        const int ncp = assign_parts(kc, 0);
        upload_sweep(al, kc, sizeof(Ext<double>));
        al.uploaded();
        launch_sweep(o.precision, IN_LOG2, kc, ps, partial, nullptr, 0, s);
        hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, partial, 0, ncp,
                           &ps[1].w1);
        if (f_out) enqueue_scale(F, f_out, n, eps * kLn2, s);
        if (g_out) enqueue_scale(Gf, g_out, m, eps * kLn2, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hps, ps, 2 * sizeof(ProbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (confirm) {
            hps[0].err = err64;
            hps[0].converged = (err64 <= tol) ? 1 : 0;
            if (!std::isfinite(err64)) hps[0].status = 1;
        }
        finish_result(res, hps[0], hps[1].w1);
        res->sweeps += resumes;
        res->resumes = resumes;
        res->fast = fast ? (resident ? 2 : 1) : (gen ? 3 : 0);
        if (hps[0].status) return fail(FINOM_E_NUMERIC);
        return fail(hps[0].converged ? FINOM_OK : FINOM_NOT_CONVERGED);
    } catch (...) {
        return fail(map_exception());
    }
}

// ---------------------------------------------------------------------------
// Algorithm 2 with the decoupled stabilised sweeps of the appendix
// ---------------------------------------------------------------------------
int sinkhorn_w1_2d(const double* x1, int64_t n1, const double* y1, int64_t m1, const double* x2,
                   int64_t n2, const double* y2, int64_t m2, const double* u, const double* v,
                   double eps, double tol, int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!res) return FINOM_E_ARG;
    memset(res, 0, sizeof(*res));
    auto fail = [&](int st) {
        res->status = st;
        return st;
    };
    if (!x1 || !y1 || !x2 || !y2 || !u || !v) return fail(FINOM_E_ARG);
    if (n1 < 1 || m1 < 1 || n2 < 1 || m2 < 1 || !finite_pos(eps)) return fail(FINOM_E_ARG);
    if (!(tol >= 0.0) || !std::isfinite(tol) || itr_max < 0) return fail(FINOM_E_ARG);
    if (o.precision != 0 && o.precision != 1) return fail(FINOM_E_ARG);
    const long long na = (long long)n1 * m1, nb = (long long)n2 * m2;
    if (n1 + n2 > INT32_MAX || m1 + m2 > INT32_MAX || na > (1LL << 40) || nb > (1LL << 40))
        return fail(FINOM_E_ARG);
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        const int cfg_x = short_line_cfg(o.precision, n1 + n2);
        const int cfg_y = short_line_cfg(o.precision, m1 + m2);
        const int Tx = kCfgs[cfg_x].T(), Ty = kCfgs[cfg_y].T();
        const int Tc = cost_tile_size();
        const size_t eb = ext_bytes(o.precision);

        int* dflag = al.dev<int>(4);
        double* dsum = al.dev<double>(2);
        double* lu = al.dev<double>(na);
        double* lv = al.dev<double>(nb);
        HIPCHK(hipMemsetAsync(dflag, 0, 4 * sizeof(int), s));
        if (!o.skip_checks) {
            enqueue_sorted_check(x1, n1, dflag, s);
            enqueue_sorted_check(y1, m1, dflag, s);
            enqueue_sorted_check(x2, n2, dflag, s);
            enqueue_sorted_check(y2, m2, dflag, s);
        }
        enqueue_log2_mass(u, na, lu, dflag + 1, s);
        enqueue_log2_mass(v, nb, lv, dflag + 1, s);
        enqueue_sum(al, u, na, dsum, s);
        enqueue_sum(al, v, nb, dsum + 1, s);
        if (!o.skip_checks) {
            int st = read_checks(al, dflag, dsum);
            if (st == FINOM_OK) {
                const double* ms[4] = {x1, y1, x2, y2};
                const long long ns[4] = {n1, m1, n2, m2};
                st = check_coord_range(al, ms, ns, 4, eps);
            }
            if (st != FINOM_OK) return fail(st);
        }

        // 1D kernels of both axes (eq. 2d-1d-kernels) and their transposes
        const Part px = make_part(al, x1, n1, x2, n2, Tx, s);    // K_x:   rows x1, cols x2
        const Part px_t = make_part_transposed(al, px, s);       // K_x^T: rows x2, cols x1
        const Part py = make_part(al, y1, m1, y2, m2, Ty, s);    // K_y:   rows y1, cols y2
        const Part py_t = make_part_transposed(al, py, s);       // K_y^T: rows y2, cols y1
        const Part pxc = make_part_like(al, px, Tc, s);
        const Part pyc = make_part_like(al, py, Tc, s);

        // phi column-major; psi, log2 v and v row-major (element (l, j) at j + l m2)
        double* F = al.dev<double>(na);
        double* G[2] = {al.dev<double>(nb), al.dev<double>(nb)};
        double* S = al.dev<double>((long long)n2 * m1);
        double* lvr = al.dev<double>(nb);
        double* vr = al.dev<double>(nb);
        enqueue_transpose_scale(lv, lvr, n2, m2, true, 1.0, s);
        enqueue_transpose_scale(v, vr, n2, m2, true, 1.0, s);
        enqueue_fill(F, na, -log2((double)na), s);
        enqueue_fill(G[0], nb, -log2((double)nb), s);
        ProbState* ps = al.dev<ProbState>(2);
        ProbState* hps = al.host<ProbState>(2);
        init_state(al, ps, hps, 2, itr_max, tol);

        // FP32 mode on lines of at most 2048 points: the loop keeps the
        // grids' scalings as extended numbers (finom_line_ext.hpp), with no
        // exponential or logarithm per point and iteration
        const int lx_shape = ext2d_shape(n1, m1, n2, m2, o.precision);
        const bool ext2d = lx_shape >= 0;
        const double kappa = 1.0 / (eps * kLn2);

        Sweep ktx[2], kty[2], ky[2], kx[2];
        int nchk = 0, pre2d = 0;
        if (!ext2d) {
            for (int b = 0; b < 2; ++b) {
                ktx[b].cfg = kx[b].cfg = cfg_x;
                kty[b].cfg = ky[b].cfg = cfg_y;
                // K^T phi = vec(K_x^T Phi K_y): S = K_x^T Phi (columns), then S K_y (rows of S into rows of psi)
                ktx[b].epi = EPI_STORE_LOG2;
                add_2d_kt_x_lines(ktx[b], px_t, eps, F, n1, S, m1);
                kty[b].epi = EPI_UPDATE_CHECK;
                add_2d_kt_y_lines(kty[b], py_t, eps, S, m1, G[1 - b], m2, lvr, vr, G[b], n2);
                nchk = assign_parts(kty[b], 0);
                // K psi = vec(K_x Psi K_y^T): S = Psi K_y^T (rows of psi), then K_x S (columns into phi)
                ky[b].epi = EPI_STORE_LOG2;
                add_2d_k_y_lines(ky[b], py, eps, G[1 - b], m2, S, m1, n2);
                kx[b].epi = EPI_UPDATE;
                add_2d_k_x_lines(kx[b], px, eps, S, n2, F, n1, lu, m1);
            }
            for (int b = 0; b < 2; ++b) {
                pre2d = wire_decision(ky[b], nchk);
                upload_sweep(al, ktx[b], eb);
                upload_sweep(al, kty[b], eb);
                upload_sweep(al, ky[b], eb);
                upload_sweep(al, kx[b], eb);
            }
        }

        // FP32 mode: every stop is confirmed by the FP64 check of the pair it
        // returns (K^T phi along x then y with FP64 scans)
        const bool confirm = o.precision == 1;
        Sweep ktx64, kty64[2];   // kty64 by the buffer holding the checked psi
        if (confirm) {
            ktx64.cfg = cfg_x;
            ktx64.epi = EPI_STORE_LOG2;
            add_2d_kt_x_lines(ktx64, px_t, eps, F, n1, S, m1, 1);
            upload_sweep(al, ktx64, sizeof(Ext<double>));
            for (int bo = 0; bo < 2; ++bo) {
                kty64[bo].cfg = cfg_y;
                kty64[bo].epi = EPI_UPDATE_CHECK;
                add_2d_kt_y_lines(kty64[bo], py_t, eps, S, m1, G[1 - bo], m2, lvr, vr, G[bo], n2, 1);
                nchk = assign_parts(kty64[bo], 0);
                upload_sweep(al, kty64[bo], sizeof(Ext<double>));
            }
        }
        const long long ncost = 2LL * m1 * pxc.ntiles;
        double* partial = al.dev<double>(std::max<long long>(std::max<long long>(nchk + 1, ncost), n2));
        double* part64 = confirm ? al.dev<double>(nchk) : nullptr;
        double* err64_d = confirm ? al.dev<double>(1) : nullptr;
        double* err64_h = confirm ? al.host<double>(1) : nullptr;

        // the extended-state loop's arrays and launches
        Ext2D e;
        if (ext2d) {
            ext2d_bind(e, al.dev<char>(ext2d_bytes(n1, m1, n2, m2)), n1, m1, n2, m2, lx_shape);
            ext2d_setup(e, px, px_t, py, py_t, 0);
            ext2d_init(e, x1, x2, y1, y2, lu, lvr, kappa, s);
        }
        al.uploaded();
        int shift = 0;          // psi of iteration l in G[(l & 1) ^ shift]
        int resumes = 0;
        long long last_l = -1;   // iteration of the last rejected stop
        long long step = 0;      // iterations run after it
        double err64 = 0.0;
        // the extended state as log2 potentials (F, and psi's slot bo of G)
        auto ext_to_log2 = [&](int bo) { ext2d_to_log2(e, bo, F, G[bo], x1, x2, y1, y2, kappa, s); };
        auto on_stop = [&]() -> bool {
            const long long l = hps[0].iters;
            const int bo = psi_slot(l, shift);
            if (ext2d) ext_to_log2(bo);
            launch_sweep(0, IN_LOG2, ktx64, ps, nullptr, nullptr, 0, s);
            launch_sweep(0, IN_LOG2, kty64[bo], ps, part64, nullptr, 0, s);
            hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, part64, 0, nchk, err64_d);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(err64_h, err64_d, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            err64 = *err64_h;
            if (!(err64 > tol) || l >= itr_max || !std::isfinite(err64) || hps[0].status ||
                !may_resume(l, last_l))
                return false;
            if (bo == 1) {
                if (ext2d) HIPCHK(hipMemcpyAsync(e.UG[0], e.UG[1], sizeof(Ext<float>) * nb, hipMemcpyDeviceToDevice, s));
                else HIPCHK(hipMemcpyAsync(G[0], G[1], sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
            }
            shift = (int)(l & 1);
            step = resume_step(step);
            enqueue_rearm(ps, l, resume_until(l, step, itr_max), s);
            last_l = l;
            ++resumes;
            return true;
        };

        const int kit = o.graph_iters > 0 ? o.graph_iters : default_graph_iters((na + nb) / 2);
        int st;
        if (ext2d) {
            // the prologue's S holds K_x^T phi for the first pair; each phi pair
            // leaves it for the next (a stop keeps phi and S as they were)
            ext2d_prologue(e, ps, s);
            auto body = [&](int b, hipStream_t cs) { ext2d_iteration(e, b, ps, cs); };
            st = run_loop_fn(body, ps, itr_max, kit, s, hps, res,
                             confirm ? std::function<bool()>(on_stop) : std::function<bool()>());
            if (st == FINOM_OK) ext_to_log2(psi_slot(hps[0].iters, shift));
        } else {
            LoopSpec lp;
            for (int b = 0; b < 2; ++b) {
                lp.seq[b] = {&ktx[b], &kty[b], &ky[b], &kx[b]};
                lp.decides[b] = {false, false, true, false};
                lp.pre[b] = {0, 0, pre2d, 0};
            }
            st = run_loop(lp, o.precision, ps, partial, itr_max, kit, s, hps, res,
                          confirm ? std::function<bool()>(on_stop) : std::function<bool()>());
        }
        if (st != FINOM_OK) return fail(st);

        // <C, Gamma> = sum Phi o (M_x Psi K_y^T) + sum Phi o (K_x Psi M_y^T), M = C o K,
        // each product along y first, as in the loop
        double* Gf = G[psi_slot(hps[0].iters, shift)];
        Sweep cy_p, cx_m, cy_m, cx_p;
        cy_p.kind = 1; cy_p.epi = EPI_STORE_LOG2;
        add_2d_k_y_lines(cy_p, pyc, eps, Gf, m2, S, m1, n2);
        cx_m.kind = 2; cx_m.epi = EPI_COST;
        add_2d_k_x_lines(cx_m, pxc, eps, S, n2, nullptr, n1, F, m1);
        cy_m.kind = 2; cy_m.epi = EPI_STORE_LOG2;
        add_2d_k_y_lines(cy_m, pyc, eps, Gf, m2, S, m1, n2);
        cx_p.kind = 1; cx_p.epi = EPI_COST;
        add_2d_k_x_lines(cx_p, pxc, eps, S, n2, nullptr, n1, F, m1);
        for (Sweep* c : {&cy_p, &cx_m, &cy_m, &cx_p})
            for (auto& L : c->lines) L.prob = 1;
        const int n_a = assign_parts(cx_m, 0);
        const int n_b = assign_parts(cx_p, n_a);
        for (Sweep* c : {&cy_p, &cx_m, &cy_m, &cx_p}) upload_sweep(al, *c, sizeof(Ext<double>));
        al.uploaded();
        launch_sweep(o.precision, IN_LOG2, cy_p, ps, partial, nullptr, 0, s);
        launch_sweep(o.precision, IN_LOG2, cx_m, ps, partial, nullptr, 0, s);
        launch_sweep(o.precision, IN_LOG2, cy_m, ps, partial, nullptr, 0, s);
        launch_sweep(o.precision, IN_LOG2, cx_p, ps, partial, nullptr, 0, s);
        hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, partial, 0,
                           n_a + n_b, &ps[1].w1);
        if (f_out) enqueue_scale(F, f_out, na, eps * kLn2, s);
        if (g_out) enqueue_transpose_scale(Gf, g_out, n2, m2, false, eps * kLn2, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hps, ps, 2 * sizeof(ProbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (confirm) {
            hps[0].err = err64;
            hps[0].converged = (err64 <= tol) ? 1 : 0;
            if (!std::isfinite(err64)) hps[0].status = 1;
        }
        finish_result(res, hps[0], hps[1].w1);
        res->sweeps = 4 * hps[0].iters + 2 + 2 * resumes;
        res->resumes = resumes;
        res->fast = ext2d ? 4 : 0;
        if (hps[0].status) return fail(FINOM_E_NUMERIC);
        return fail(hps[0].converged ? FINOM_OK : FINOM_NOT_CONVERGED);
    } catch (...) {
        return fail(map_exception());
    }
}

// ---------------------------------------------------------------------------
// d-dimensional tensor meshes: the remark closing section 3 applies each
// product axis by axis, the 1D method along every coordinate direction
// ---------------------------------------------------------------------------
int sinkhorn_w1_nd(int32_t d, const int64_t* n_src, const double* const* x_src, const int64_t* n_tgt,
                   const double* const* x_tgt, const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out, double* g_out, finom_result* res,
                   void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!res) return FINOM_E_ARG;
    memset(res, 0, sizeof(*res));
    auto fail = [&](int st) {
        res->status = st;
        return st;
    };
    if (d < 1 || d > FINOM_MAX_DIMS || !n_src || !x_src || !n_tgt || !x_tgt || !u || !v) return fail(FINOM_E_ARG);
    if (!finite_pos(eps) || !(tol >= 0.0) || !std::isfinite(tol) || itr_max < 0) return fail(FINOM_E_ARG);
    if (o.precision != 0 && o.precision != 1) return fail(FINOM_E_ARG);
    long long na = 1, nb = 1;
    for (int a = 0; a < d; ++a) {
        if (!x_src[a] || !x_tgt[a] || n_src[a] < 1 || n_tgt[a] < 1) return fail(FINOM_E_ARG);
        if (n_src[a] + n_tgt[a] > INT32_MAX) return fail(FINOM_E_ARG);
        if (n_src[a] > (1LL << 40) / na || n_tgt[a] > (1LL << 40) / nb) return fail(FINOM_E_ARG);
        na *= n_src[a];
        nb *= n_tgt[a];
    }
    // one and two axes have their own paths (the resident and fast 1D sweeps;
    // the 2D layout with psi row-major)
    if (d == 1)
        return sinkhorn_w1_1d(x_src[0], n_src[0], x_tgt[0], n_tgt[0], u, v, eps, tol, itr_max, opts, f_out, g_out,
                              res, stream);
    if (d == 2)
        return sinkhorn_w1_2d(x_src[0], n_src[0], x_src[1], n_src[1], x_tgt[0], n_tgt[0], x_tgt[1], n_tgt[1], u, v,
                              eps, tol, itr_max, opts, f_out, g_out, res, stream);
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        const int Tc = cost_tile_size();
        const size_t eb = ext_bytes(o.precision);

        int* dflag = al.dev<int>(4);
        double* dsum = al.dev<double>(2);
        double* lu = al.dev<double>(na);
        double* lv = al.dev<double>(nb);
        HIPCHK(hipMemsetAsync(dflag, 0, 4 * sizeof(int), s));
        if (!o.skip_checks)
            for (int a = 0; a < d; ++a) {
                enqueue_sorted_check(x_src[a], n_src[a], dflag, s);
                enqueue_sorted_check(x_tgt[a], n_tgt[a], dflag, s);
            }
        enqueue_log2_mass(u, na, lu, dflag + 1, s);
        enqueue_log2_mass(v, nb, lv, dflag + 1, s);
        enqueue_sum(al, u, na, dsum, s);
        enqueue_sum(al, v, nb, dsum + 1, s);
        if (!o.skip_checks) {
            int st = read_checks(al, dflag, dsum);
            if (st == FINOM_OK) {
                const double* ms[2 * FINOM_MAX_DIMS];
                long long ns[2 * FINOM_MAX_DIMS];
                for (int a = 0; a < d; ++a) {
                    ms[2 * a] = x_src[a];
                    ns[2 * a] = n_src[a];
                    ms[2 * a + 1] = x_tgt[a];
                    ns[2 * a + 1] = n_tgt[a];
                }
                st = check_coord_range(al, ms, ns, 2 * d, eps);
            }
            if (st != FINOM_OK) return fail(st);
        }

        // per axis: K_a (rows source, columns target), K_a^T, and the cost partition
        std::vector<int> cfg(d);
        std::vector<Part> pk(d), pkt(d), pc(d);
        for (int a = 0; a < d; ++a) {
            cfg[a] = short_line_cfg(o.precision, n_src[a] + n_tgt[a]);
            pk[a] = make_part(al, x_src[a], n_src[a], x_tgt[a], n_tgt[a], kCfgs[cfg[a]].T(), s);
            pkt[a] = make_part_transposed(al, pk[a], s);
            pc[a] = make_part_like(al, pk[a], Tc, s);
        }

        // Grid layouts: rot(r) stores the axes in the order r, r+1, ..., d-1,
        // 0, ..., r-1, the first fastest. K^T phi runs along axes 0, 1, ...,
        // d-1 and K psi along d-1, ..., 0. A step along axis a reads its input
        // in rot(a), so that every line is contiguous, and stores its output
        // in the layout the next step reads, strided along a; the last step of
        // a product stores in rot(a), contiguously. So phi lives in rot(0),
        // the caller's column-major order, and psi in rot(d-1), with the
        // copies of log2 v and v that the check reads.
        auto strides_of = [&](const std::vector<long long>& sz, int r, std::vector<long long>& st) {
            st.assign(d, 0);
            long long acc = 1;
            for (int q = 0; q < d; ++q) {
                const int ax = (r + q) % d;
                st[ax] = acc;
                acc *= sz[ax];
            }
        };
        long long smax = 1;
        for (int dir = 0; dir < 2; ++dir) {
            const bool tt = dir == 0;
            std::vector<long long> sz(d);
            for (int q = 0; q < d; ++q) sz[q] = tt ? n_src[q] : n_tgt[q];
            for (int k = 0; k + 1 < d; ++k) {
                const int a = tt ? k : d - 1 - k;
                sz[a] = tt ? n_tgt[a] : n_src[a];
                long long tot = 1;
                for (int q = 0; q < d; ++q) tot *= sz[q];
                smax = std::max(smax, tot);
            }
        }
        const long long rows_t = nb / n_tgt[d - 1];   // psi in rot(d-1): the column-major grid transposed as
                                                      // rows_t x n_tgt[d-1]
        double* S[2] = {al.dev<double>(smax), al.dev<double>(smax)};
        double* F = al.dev<double>(na);
        double* G[2] = {al.dev<double>(nb), al.dev<double>(nb)};
        double* lvr = al.dev<double>(nb);
        double* vr = al.dev<double>(nb);
        enqueue_transpose_scale(lv, lvr, rows_t, n_tgt[d - 1], true, 1.0, s);
        enqueue_transpose_scale(v, vr, rows_t, n_tgt[d - 1], true, 1.0, s);
        enqueue_fill(F, na, -log2((double)na), s);
        enqueue_fill(G[0], nb, -log2((double)nb), s);
        ProbState* ps = al.dev<ProbState>(2);
        ProbState* hps = al.host<ProbState>(2);
        init_state(al, ps, hps, 2, itr_max, tol);

        // Step k of a product (axis a): a line is one multi-index over the
        // other axes; it reads its contiguous run of the input (axis a
        // fastest there) and writes at the output offset of the same
        // multi-index with the stride of axis a in the output layout. The
        // epilogue operands of the last step are indexed as its output.
        auto add_product = [&](Sweep* sw, bool to_target, const std::vector<Part>& parts, const double* in,
                               double* out, const double* a0, const double* a1, const double* a2, int prob) {
            std::vector<long long> sz(d), st_in, st_out, idx(d);
            for (int q = 0; q < d; ++q) sz[q] = to_target ? n_src[q] : n_tgt[q];
            for (int k = 0; k < d; ++k) {
                const int a = to_target ? k : d - 1 - k;
                const bool last = k == d - 1;
                strides_of(sz, a, st_in);   // the input: axis a fastest (contiguous lines)
                sz[a] = to_target ? n_tgt[a] : n_src[a];
                const int r = last ? a : (to_target ? (a + 1) % d : (a + d - 1) % d);
                strides_of(sz, r, st_out);
                long long nlines = 1;
                for (int q = 0; q < d; ++q)
                    if (q != a) nlines *= sz[q];
                const double* src = k == 0 ? in : S[(k - 1) & 1];
                double* dst = last ? out : S[k & 1];
                const Part& p = parts[a];
                // every line of the step shares the meshes and the partition
                LineDesc base = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
                base.ostride = st_out[a];
                base.dec_part_off = -1;
                base.prob = prob;
                sw[k].lines.reserve(sw[k].lines.size() + (size_t)nlines);
                // lines in the order of the output's layout (its stride-one axis
                // fastest), so that neighbouring workgroups store neighbouring
                // elements and fill cache lines together in one L2; each line
                // reads its input, a contiguous run, wherever it lies
                std::vector<int> ord;
                for (int q = 0; q < d; ++q)
                    if ((r + q) % d != a) ord.push_back((r + q) % d);
                std::fill(idx.begin(), idx.end(), 0);
                for (long long L = 0; L < nlines; ++L) {
                    long long oo = 0, io = 0;
                    for (int q = 0; q < d; ++q)
                        if (q != a) {
                            oo += idx[q] * st_out[q];
                            io += idx[q] * st_in[q];
                        }
                    LineDesc Ld = base;
                    Ld.gin = src + io;
                    Ld.out = dst ? dst + oo : nullptr;
                    if (last) {
                        Ld.a0 = a0 ? a0 + oo : nullptr;
                        Ld.a1 = a1 ? a1 + oo : nullptr;
                        Ld.a2 = a2 ? a2 + oo : nullptr;
                    }
                    sw[k].lines.push_back(Ld);
                    for (const int ax : ord) {
                        if (++idx[ax] < sz[ax]) break;
                        idx[ax] = 0;
                    }
                }
            }
        };

        // K^T phi: every axis in turn from the source grid to the target grid,
        // the last step with the psi update and the marginal check; K psi back,
        // its first step taking the stop decision and its last the phi update
        std::vector<Sweep> kt[2], kp[2];
        int nchk = 0;
        for (int b = 0; b < 2; ++b) {
            kt[b].resize(d);
            kp[b].resize(d);
            for (int k = 0; k < d; ++k) {
                kt[b][k].cfg = cfg[k];
                kp[b][k].cfg = cfg[d - 1 - k];
                kt[b][k].epi = kp[b][k].epi = EPI_STORE_LOG2;
            }
            kt[b][d - 1].epi = EPI_UPDATE_CHECK;
            kp[b][d - 1].epi = EPI_UPDATE;
            add_product(kt[b].data(), true, pkt, F, G[1 - b], lvr, vr, G[b], 0);
            nchk = assign_parts(kt[b][d - 1], 0);
            add_product(kp[b].data(), false, pk, G[1 - b], F, lu, nullptr, nullptr, 0);
        }
        int prend = 0;
        for (int b = 0; b < 2; ++b) {
            prend = wire_decision(kp[b][0], nchk);
            for (int k = 0; k < d; ++k) upload_sweep(al, kt[b][k], eb);
            for (int k = 0; k < d; ++k) upload_sweep(al, kp[b][k], eb);
        }
        const long long ncost = (long long)d * (na / n_src[0]) * pc[0].ntiles;
        double* partial = al.dev<double>(std::max<long long>(nchk + 1, ncost));

        // FP32 mode: every stop is confirmed by the FP64 check of the pair it
        // returns (K^T phi along every axis with FP64 scans)
        const bool confirm = o.precision == 1;
        std::vector<Sweep> kt64[2];   // by the buffer holding the checked psi
        double* part64 = confirm ? al.dev<double>(nchk) : nullptr;
        double* err64_d = confirm ? al.dev<double>(1) : nullptr;
        double* err64_h = confirm ? al.host<double>(1) : nullptr;
        for (int bo = 0; bo < 2 && confirm; ++bo) {
            kt64[bo].resize(d);
            for (int k = 0; k < d; ++k) {
                kt64[bo][k].cfg = cfg[k];
                kt64[bo][k].epi = k == d - 1 ? EPI_UPDATE_CHECK : EPI_STORE_LOG2;
            }
            add_product(kt64[bo].data(), true, pkt, F, G[1 - bo], lvr, vr, G[bo], 1);
            assign_parts(kt64[bo][d - 1], 0);
            for (int k = 0; k < d; ++k) upload_sweep(al, kt64[bo][k], sizeof(Ext<double>));
        }
        al.uploaded();
        int shift = 0;          // psi of iteration l in G[(l & 1) ^ shift]
        int resumes = 0;
        long long last_l = -1;   // iteration of the last rejected stop
        long long step = 0;      // iterations run after it
        double err64 = 0.0;
        auto on_stop = [&]() -> bool {
            const long long l = hps[0].iters;
            const int bo = psi_slot(l, shift);
            for (int k = 0; k < d; ++k)
                launch_sweep(0, IN_LOG2, kt64[bo][k], ps, k == d - 1 ? part64 : nullptr, nullptr, 0, s);
            hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, part64, 0, nchk, err64_d);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(err64_h, err64_d, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            err64 = *err64_h;
            if (!(err64 > tol) || l >= itr_max || !std::isfinite(err64) || hps[0].status ||
                !may_resume(l, last_l))
                return false;
            if (bo == 1) HIPCHK(hipMemcpyAsync(G[0], G[1], sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
            shift = (int)(l & 1);
            step = resume_step(step);
            enqueue_rearm(ps, l, resume_until(l, step, itr_max), s);
            last_l = l;
            ++resumes;
            return true;
        };

        LoopSpec lp;
        for (int b = 0; b < 2; ++b) {
            for (int a = 0; a < d; ++a) {
                lp.seq[b].push_back(&kt[b][a]);
                lp.decides[b].push_back(false);
            }
            lp.pre[b].assign(d, 0);
            for (int a = 0; a < d; ++a) {
                lp.seq[b].push_back(&kp[b][a]);
                lp.decides[b].push_back(a == 0);
                lp.pre[b].push_back(a == 0 ? prend : 0);
            }
        }
        const int kit = o.graph_iters > 0 ? o.graph_iters : default_graph_iters((na + nb) / 2);
        const int st = run_loop(lp, o.precision, ps, partial, itr_max, kit, s, hps, res,
                                confirm ? std::function<bool()>(on_stop) : std::function<bool()>());
        if (st != FINOM_OK) return fail(st);

        // <C, Gamma> with C = sum_c |x_c - y_c|: pass c is the product K psi
        // with the moment kernel C_c o K_c along axis c, summed against phi
        double* Gf = G[psi_slot(hps[0].iters, shift)];
        std::vector<Sweep> cs((size_t)d * d);
        int nparts = 0;
        for (int c = 0; c < d; ++c) {
            Sweep* w = cs.data() + (size_t)c * d;
            for (int k = 0; k < d; ++k) {
                w[k].kind = d - 1 - k == c ? 2 : 1;
                w[k].epi = k == d - 1 ? EPI_COST : EPI_STORE_LOG2;
            }
            add_product(w, false, pc, Gf, nullptr, F, nullptr, nullptr, 1);
            nparts += assign_parts(w[d - 1], nparts);
        }
        for (auto& w : cs) upload_sweep(al, w, sizeof(Ext<double>));
        al.uploaded();
        for (auto& w : cs) launch_sweep(o.precision, IN_LOG2, w, ps, partial, nullptr, 0, s);
        hipLaunchKernelGGL((k_reduce_partials<kBlock>), dim3(1), dim3(kBlock), 0, s, partial, 0, nparts,
                           &ps[1].w1);
        if (f_out) enqueue_scale(F, f_out, na, eps * kLn2, s);
        if (g_out) enqueue_transpose_scale(Gf, g_out, rows_t, n_tgt[d - 1], false, eps * kLn2, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hps, ps, 2 * sizeof(ProbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (confirm) {
            hps[0].err = err64;
            hps[0].converged = (err64 <= tol) ? 1 : 0;
            if (!std::isfinite(err64)) hps[0].status = 1;
        }
        finish_result(res, hps[0], hps[1].w1);
        res->sweeps = 2LL * d * hps[0].iters + d + (long long)d * resumes;
        res->resumes = resumes;
        if (hps[0].status) return fail(FINOM_E_NUMERIC);
        return fail(hps[0].converged ? FINOM_OK : FINOM_NOT_CONVERGED);
    } catch (...) {
        return fail(map_exception());
    }
}

const char* finom_strerror(int status)
{
    switch (status) {
        case FINOM_OK: return "ok";
        case FINOM_NOT_CONVERGED: return "iteration cap reached before the tolerance";
        case FINOM_E_ARG: return "invalid argument";
        case FINOM_E_UNSORTED: return "mesh is not non-decreasing or holds a non-finite value";
        case FINOM_E_MASS: return "masses must be positive, finite and balanced";
        case FINOM_E_NOMEM: return "out of device or pinned host memory";
        case FINOM_E_HIP: return "HIP runtime error";
        case FINOM_E_ADMIT: return "request exceeds the serving memory budget";
        case FINOM_E_NUMERIC: return "non-finite marginal error";
        default: return "unknown status";
    }
}

void finom_release(void) { arena_release_all(); }

const char* finom_version(void) { return "finom-gfx950 0.3"; }

const char* finom_last_error(void) { return g_last_error; }

}  // extern "C"
