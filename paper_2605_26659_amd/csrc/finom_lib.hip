// Host side of the FINOM library: argument checks, device setup kernels
// (sortedness, dividing index, merge-path partition, log masses), workspace,
// sweep dispatch, the Sinkhorn loop of Algorithm 1 captured in HIP graphs,
// and the C ABI of include/finom.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/finom.h"
#include "finom_kernels.hpp"

namespace finom {

constexpr int kBlock = 256;
constexpr int kIptF32 = 8;    // T = 2048 merged elements per tile
constexpr int kIptF64 = 4;    // T = 1024
constexpr int kIptCost = 2;   // T = 512, FP64 moment sums (four LDS arrays)
constexpr double kLn2 = 0.69314718055994530942;

struct HipError {
    hipError_t e;
};

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t _e = (x);                       \
        if (_e != hipSuccess) throw HipError{_e};  \
    } while (0)

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

// flags[0] |= 1 if a[k] > a[k+1] or a[k] is not finite.
__global__ void k_check_sorted(const double* __restrict__ a, long long n, int* __restrict__ flag)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double v = a[k];
    bool bad = !(v == v) || fabs(v) == __builtin_inf();
    if (k + 1 < n && v > a[k + 1]) bad = true;
    if (bad) atomicOr(flag, 1);
}

// flags |= 1 if a mass is not > 0 / not finite; writes log2 of it.
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

__global__ __launch_bounds__(kBlock) void k_final_sum(const double* __restrict__ part, int np,
                                                      double* __restrict__ out)
{
    __shared__ double s_red[kBlock / kWave];
    double v = 0.0;
    for (int k = threadIdx.x; k < np; k += kBlock) v += part[k];
    v = block_sum_f64<kBlock>(v, s_red);
    if (threadIdx.x == 0) *out = v;
}

// zeta[i] = #{j : y_j <= x_i} (the dividing index of section 2.2, 0-based count)
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
            s_g[k] = load_in<INM>(gin + c0 + k, in_scale);
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
// workspace: one growable device arena and one pinned host arena per stream
// ---------------------------------------------------------------------------
struct Arena {
    char* dev = nullptr;
    size_t dcap = 0, dused = 0;
    char* host = nullptr;
    size_t hcap = 0, hused = 0;
    hipEvent_t upload_done = nullptr;
};

static std::mutex g_mu;
static std::map<void*, Arena*> g_arenas;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Alloc {
    Arena* a;
    hipStream_t s;
    Alloc(void* stream) : s((hipStream_t)stream)
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_arenas.find(stream);
        if (it == g_arenas.end()) {
            a = new Arena();
            g_arenas[stream] = a;
        } else {
            a = it->second;
        }
    }
    // Reserve (bytes) of device and host memory for this call; reallocates when
    // the arena is too small (after the stream has drained).
    void reserve(size_t dbytes, size_t hbytes)
    {
        if (a->upload_done) HIPCHK(hipEventSynchronize(a->upload_done));
        if (dbytes > a->dcap) {
            HIPCHK(hipStreamSynchronize(s));
            if (a->dev) HIPCHK(hipFree(a->dev));
            a->dev = nullptr;
            a->dcap = 0;
            size_t cap = std::max(dbytes, a->dcap * 3 / 2);
            if (hipMalloc((void**)&a->dev, cap) != hipSuccess) throw std::bad_alloc();
            a->dcap = cap;
        }
        if (hbytes > a->hcap) {
            HIPCHK(hipStreamSynchronize(s));
            if (a->host) HIPCHK(hipHostFree(a->host));
            a->host = nullptr;
            a->hcap = 0;
            size_t cap = std::max(hbytes, (size_t)1 << 16);
            if (hipHostMalloc((void**)&a->host, cap, hipHostMallocDefault) != hipSuccess)
                throw std::bad_alloc();
            a->hcap = cap;
        }
        if (!a->upload_done) HIPCHK(hipEventCreateWithFlags(&a->upload_done, hipEventDisableTiming));
        a->dused = 0;
        a->hused = 0;
    }
    template <typename T>
    T* dev(size_t count)
    {
        size_t off = align_up(a->dused, 256);
        a->dused = off + align_up(sizeof(T) * std::max<size_t>(count, 1), 256);
        if (a->dused > a->dcap) throw std::bad_alloc();
        return reinterpret_cast<T*>(a->dev + off);
    }
    template <typename T>
    T* host(size_t count)
    {
        size_t off = align_up(a->hused, 64);
        a->hused = off + align_up(sizeof(T) * std::max<size_t>(count, 1), 64);
        if (a->hused > a->hcap) throw std::bad_alloc();
        return reinterpret_cast<T*>(a->host + off);
    }
};

// Byte counter used to size the arena before carving it.
struct Sizer {
    size_t d = 0, h = 0;
    template <typename T>
    void dev(size_t count) { d = align_up(d, 256) + align_up(sizeof(T) * std::max<size_t>(count, 1), 256); }
    template <typename T>
    void host(size_t count) { h = align_up(h, 64) + align_up(sizeof(T) * std::max<size_t>(count, 1), 64); }
};

static unsigned blocks_for(long long n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

static int ntiles_for(long long R, long long C, int T) { return (int)((R + C + T - 1) / T); }

static int tile_size(int precision) { return kBlock * (precision == 1 ? kIptF32 : kIptF64); }

// ---------------------------------------------------------------------------
// sweep dispatch
// ---------------------------------------------------------------------------
struct SweepDev {
    const WorkItem* work = nullptr;        // all tiles
    int nwork = 0;
    const WorkItem* work_multi = nullptr;  // tiles of lines with more than one tile
    int nwork_multi = 0;
    const LineDesc* lines = nullptr;
    void* agg = nullptr;
    void* carry = nullptr;
    unsigned int* line_ctr = nullptr;
};

template <typename M, int IPT, int INM, int EPI, bool MOMENT>
static void launch_sweep_t(const SweepDev& sw, ProbState* ps, double* partial, hipStream_t s)
{
    if (sw.nwork_multi > 0) {
        hipLaunchKernelGGL((k_tile_aggregate<M, kBlock, IPT, INM, MOMENT>), dim3(sw.nwork_multi),
                           dim3(kBlock), 0, s, sw.work_multi, sw.lines, ps, (Ext<M>*)sw.agg,
                           (Ext<M>*)sw.carry, sw.line_ctr);
    }
    hipLaunchKernelGGL((k_sweep<M, kBlock, IPT, INM, EPI, MOMENT>), dim3(sw.nwork), dim3(kBlock), 0, s,
                       sw.work, sw.lines, ps, (const Ext<M>*)sw.carry, partial);
    HIPCHK(hipGetLastError());
}

static void launch_sweep(int precision, int inm, int epi, const SweepDev& sw, ProbState* ps,
                         double* partial, hipStream_t s)
{
#define SW(M, IPT, I, E) launch_sweep_t<M, IPT, I, E, false>(sw, ps, partial, s)
    if (precision == 1) {
        switch (inm * 16 + epi) {
            case IN_LOG2 * 16 + EPI_STORE_LOG2: SW(float, kIptF32, IN_LOG2, EPI_STORE_LOG2); return;
            case IN_LOG2 * 16 + EPI_UPDATE: SW(float, kIptF32, IN_LOG2, EPI_UPDATE); return;
            case IN_LOG2 * 16 + EPI_UPDATE_CHECK: SW(float, kIptF32, IN_LOG2, EPI_UPDATE_CHECK); return;
            case IN_NAT * 16 + EPI_STORE_NAT: SW(float, kIptF32, IN_NAT, EPI_STORE_NAT); return;
            case IN_LIN * 16 + EPI_STORE_LIN: SW(float, kIptF32, IN_LIN, EPI_STORE_LIN); return;
        }
    } else {
        switch (inm * 16 + epi) {
            case IN_LOG2 * 16 + EPI_STORE_LOG2: SW(double, kIptF64, IN_LOG2, EPI_STORE_LOG2); return;
            case IN_LOG2 * 16 + EPI_UPDATE: SW(double, kIptF64, IN_LOG2, EPI_UPDATE); return;
            case IN_LOG2 * 16 + EPI_UPDATE_CHECK: SW(double, kIptF64, IN_LOG2, EPI_UPDATE_CHECK); return;
            case IN_NAT * 16 + EPI_STORE_NAT: SW(double, kIptF64, IN_NAT, EPI_STORE_NAT); return;
            case IN_LIN * 16 + EPI_STORE_LIN: SW(double, kIptF64, IN_LIN, EPI_STORE_LIN); return;
        }
    }
#undef SW
    throw HipError{hipErrorInvalidValue};
}

static void launch_cost_sweep(int epi, const SweepDev& sw, ProbState* ps, double* partial, hipStream_t s)
{
    if (epi == EPI_COST)
        launch_sweep_t<double, kIptCost, IN_LOG2, EPI_COST, true>(sw, ps, partial, s);
    else
        launch_sweep_t<double, kIptCost, IN_LOG2, EPI_STORE_LOG2, true>(sw, ps, partial, s);
}

// Host-side description of the lines of one sweep, turned into device arrays.
struct SweepHost {
    std::vector<LineDesc> lines;
    int T = 0;
    int total_tiles() const
    {
        int t = 0;
        for (auto& l : lines) t += l.ntiles;
        return t;
    }
    int multi_tiles() const
    {
        int t = 0;
        for (auto& l : lines)
            if (l.ntiles > 1) t += l.ntiles;
        return t;
    }
    int max_lines() const { return (int)lines.size(); }
};

// Sizes the device/host buffers a sweep needs (NS = sums per column).
static void size_sweep(Sizer& z, const SweepHost& sh, int ns, size_t ext_bytes)
{
    z.dev<WorkItem>(sh.total_tiles());
    z.dev<WorkItem>(sh.multi_tiles());
    z.dev<LineDesc>(sh.lines.size());
    z.dev<char>((size_t)sh.multi_tiles() * ns * ext_bytes);
    z.dev<char>((size_t)sh.multi_tiles() * ns * ext_bytes);
    z.dev<unsigned int>(sh.lines.size());
    z.host<WorkItem>(sh.total_tiles());
    z.host<WorkItem>(sh.multi_tiles());
    z.host<LineDesc>(sh.lines.size());
}

// Assigns agg slots, fills work lists, uploads (async, from pinned memory).
static SweepDev upload_sweep(Alloc& al, SweepHost& sh, int ns, size_t ext_bytes, hipStream_t s)
{
    SweepDev d;
    const int tt = sh.total_tiles(), mt = sh.multi_tiles();
    WorkItem* hw = al.host<WorkItem>(tt);
    WorkItem* hm = al.host<WorkItem>(mt);
    LineDesc* hl = al.host<LineDesc>(sh.lines.size());
    int k = 0, km = 0, abase = 0;
    for (size_t li = 0; li < sh.lines.size(); ++li) {
        LineDesc& L = sh.lines[li];
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
    LineDesc* dl = al.dev<LineDesc>(sh.lines.size());
    void* agg = al.dev<char>((size_t)mt * ns * ext_bytes);
    void* carry = al.dev<char>((size_t)mt * ns * ext_bytes);
    unsigned int* ctr = al.dev<unsigned int>(sh.lines.size());
    HIPCHK(hipMemcpyAsync(dw, hw, sizeof(WorkItem) * std::max(tt, 1), hipMemcpyHostToDevice, s));
    if (mt > 0) HIPCHK(hipMemcpyAsync(dm, hm, sizeof(WorkItem) * mt, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dl, hl, sizeof(LineDesc) * sh.lines.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(ctr, 0, sizeof(unsigned int) * sh.lines.size(), s));
    d.work = dw;
    d.nwork = tt;
    d.work_multi = dm;
    d.nwork_multi = mt;
    d.lines = dl;
    d.agg = agg;
    d.carry = carry;
    d.line_ctr = ctr;
    return d;
}

static LineDesc make_line(const double* xr, long long R, const double* yc, long long C,
                          const int* zeta, const int* trs, int T, double eps)
{
    LineDesc L;
    memset(&L, 0, sizeof(L));
    L.xr = xr;
    L.yc = yc;
    L.zeta = zeta;
    L.trs = trs;
    L.R = R;
    L.C = C;
    L.gstride = 1;
    L.ostride = 1;
    L.kappa = 1.0 / (eps * kLn2);
    L.in_scale = L.kappa;
    L.out_scale = eps * kLn2;
    L.shift = 0.0;
    L.ntiles = ntiles_for(R, C, T);
    return L;
}

static void setup_partition(const double* xr, long long R, const double* yc, long long C, int T,
                            int* zeta, int* trs, hipStream_t s)
{
    hipLaunchKernelGGL(k_dividing_index, dim3(blocks_for(R)), dim3(kBlock), 0, s, xr, R, yc, C, zeta);
    const int nt = ntiles_for(R, C, T);
    hipLaunchKernelGGL(k_tile_rows, dim3(blocks_for(nt + 1)), dim3(kBlock), 0, s, zeta, R, T, nt, trs);
    HIPCHK(hipGetLastError());
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int map_exception()
{
    try {
        throw;
    } catch (const std::bad_alloc&) {
        return FINOM_E_NOMEM;
    } catch (const HipError& e) {
        if (e.e == hipErrorOutOfMemory) return FINOM_E_NOMEM;
        return FINOM_E_HIP;
    } catch (...) {
        return FINOM_E_HIP;
    }
}

// ---------------------------------------------------------------------------
// matvec entry points
// ---------------------------------------------------------------------------
static int matvec_impl(bool dense, const double* x, int64_t n, const double* y, int64_t m,
                       double eps, const double* in, double* out, const finom_opts* opts,
                       void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!x || !y || !in || !out || n < 1 || m < 1 || !finite_pos(eps)) return FINOM_E_ARG;
    if (o.precision != 0 && o.precision != 1) return FINOM_E_ARG;
    if (o.domain != 0 && o.domain != 1) return FINOM_E_ARG;
    if (n + m > (int64_t)INT32_MAX) return FINOM_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        const int T = tile_size(o.precision);
        SweepHost sh;
        sh.T = T;
        sh.lines.push_back(make_line(x, n, y, m, nullptr, nullptr, T, eps));
        const size_t eb = (o.precision == 1) ? sizeof(Ext<float>) : sizeof(Ext<double>);
        Sizer z;
        z.dev<int>(2);
        z.dev<int>(n);
        z.dev<int>(sh.lines[0].ntiles + 1);
        z.dev<ProbState>(1);
        z.host<int>(2);
        size_sweep(z, sh, 2, eb);
        al.reserve(z.d, z.h);
        int* dflag = al.dev<int>(2);
        int* zeta = al.dev<int>(n);
        int* trs = al.dev<int>(sh.lines[0].ntiles + 1);
        ProbState* ps = al.dev<ProbState>(1);
        if (!o.skip_checks) {
            int* hflag = al.host<int>(2);
            HIPCHK(hipMemsetAsync(dflag, 0, 2 * sizeof(int), s));
            hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, dflag);
            hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(m)), dim3(kBlock), 0, s, y, (long long)m, dflag);
            HIPCHK(hipMemcpyAsync(hflag, dflag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hflag[0]) return FINOM_E_UNSORTED;
        }
        const int inm = (o.domain == 1) ? IN_NAT : IN_LIN;
        if (dense) {
            const double kappa = 1.0 / (eps * kLn2);
            if (o.precision == 1) {
                if (inm == IN_NAT)
                    hipLaunchKernelGGL((k_dense<float, IN_NAT>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, y,
                                       (long long)m, in, kappa, kappa, eps * kLn2, 0, out);
                else
                    hipLaunchKernelGGL((k_dense<float, IN_LIN>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, y,
                                       (long long)m, in, kappa, kappa, eps * kLn2, 1, out);
            } else {
                if (inm == IN_NAT)
                    hipLaunchKernelGGL((k_dense<double, IN_NAT>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, y,
                                       (long long)m, in, kappa, kappa, eps * kLn2, 0, out);
                else
                    hipLaunchKernelGGL((k_dense<double, IN_LIN>), dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, y,
                                       (long long)m, in, kappa, kappa, eps * kLn2, 1, out);
            }
            HIPCHK(hipGetLastError());
            return FINOM_OK;
        }
        setup_partition(x, n, y, m, T, zeta, trs, s);
        LineDesc& L = sh.lines[0];
        L.zeta = zeta;
        L.trs = trs;
        L.gin = in;
        L.out = out;
        HIPCHK(hipMemsetAsync(ps, 0, sizeof(ProbState), s));
        SweepDev sw = upload_sweep(al, sh, 2, eb, s);
        HIPCHK(hipEventRecord(al.a->upload_done, s));
        launch_sweep(o.precision, inm, (o.domain == 1) ? EPI_STORE_NAT : EPI_STORE_LIN, sw, ps, nullptr, s);
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

// ---------------------------------------------------------------------------
// 1D Sinkhorn (Algorithm 1)
// ---------------------------------------------------------------------------

// Checks masses (> 0, finite), writes log2 masses, returns |sum u - sum v| test
// through the host flag block. Sums are reduced deterministically.
struct MassCheck {
    double* dsum;   // 2 doubles
    double* part;   // 2 * nb doubles
    int nb;
};

static void enqueue_mass(const double* a, long long n, double* la, int* dflag, double* part,
                         int nb, double* dsum, hipStream_t s)
{
    hipLaunchKernelGGL(k_log2_mass, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, la, dflag);
    hipLaunchKernelGGL(k_partial_sum, dim3(nb), dim3(kBlock), 0, s, a, n, part);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, s, part, nb, dsum);
}

static int default_graph_iters(long long points)
{
    if (points <= (1 << 14)) return 64;
    if (points <= (1 << 18)) return 32;
    return 16;
}

}  // namespace finom

using namespace finom;

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
    if (o.precision != 0 && o.precision != 1) return fail(FINOM_E_ARG);
    if (n + m > (int64_t)INT32_MAX) return fail(FINOM_E_ARG);
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        const int T = tile_size(o.precision);
        const int Tc = kBlock * kIptCost;
        const size_t eb = (o.precision == 1) ? sizeof(Ext<float>) : sizeof(Ext<double>);
        const size_t ebc = sizeof(Ext<double>);
        const int nt_kt = ntiles_for(m, n, T), nt_k = ntiles_for(n, m, T), nt_c = ntiles_for(n, m, Tc);
        const int nb = 64;

        // lines: K^T phi (rows y, cols x, reads F, updates G with the check),
        //        K psi (rows x, cols y, reads G, updates F), cost (rows x, cols y)
        SweepHost kt[2], kk[2], kc;
        for (int b = 0; b < 2; ++b) {
            kt[b].lines.push_back(make_line(y, m, x, n, nullptr, nullptr, T, eps));
            kk[b].lines.push_back(make_line(x, n, y, m, nullptr, nullptr, T, eps));
        }
        kc.lines.push_back(make_line(x, n, y, m, nullptr, nullptr, Tc, eps));

        Sizer z;
        z.dev<int>(4);
        z.dev<int>(n);
        z.dev<int>(m);
        z.dev<int>(nt_k + 1);
        z.dev<int>(nt_kt + 1);
        z.dev<int>(nt_c + 1);
        z.dev<double>(n);
        z.dev<double>(m);
        z.dev<double>(n);
        z.dev<double>(m);
        z.dev<double>(m);
        z.dev<double>(std::max(nt_kt, nt_c));
        z.dev<double>(2);
        z.dev<double>(2 * nb);
        z.dev<ProbState>(2);
        for (int b = 0; b < 2; ++b) {
            size_sweep(z, kt[b], 2, eb);
            size_sweep(z, kk[b], 2, eb);
        }
        size_sweep(z, kc, 4, ebc);
        z.host<ProbState>(2);
        z.host<int>(4);
        z.host<double>(2);
        al.reserve(z.d, z.h);

        int* dflag = al.dev<int>(4);
        int* zx = al.dev<int>(n);
        int* zy = al.dev<int>(m);
        int* tx = al.dev<int>(nt_k + 1);
        int* ty = al.dev<int>(nt_kt + 1);
        int* tc = al.dev<int>(nt_c + 1);
        double* lu = al.dev<double>(n);
        double* lv = al.dev<double>(m);
        double* F = al.dev<double>(n);
        double* G[2] = {al.dev<double>(m), al.dev<double>(m)};
        double* partial = al.dev<double>(std::max(nt_kt, nt_c));
        double* dsum = al.dev<double>(2);
        double* mpart = al.dev<double>(2 * nb);
        ProbState* ps = al.dev<ProbState>(2);      // [0] iteration, [1] cost reduction
        ProbState* hps = al.host<ProbState>(2);
        int* hflag = al.host<int>(4);
        double* hsum = al.host<double>(2);

        // --- validation (device) and setup
        HIPCHK(hipMemsetAsync(dflag, 0, 4 * sizeof(int), s));
        if (!o.skip_checks) {
            hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, (long long)n, dflag);
            hipLaunchKernelGGL(k_check_sorted, dim3(blocks_for(m)), dim3(kBlock), 0, s, y, (long long)m, dflag);
        }
        enqueue_mass(u, n, lu, dflag + 1, mpart, nb, dsum, s);
        enqueue_mass(v, m, lv, dflag + 1, mpart + nb, nb, dsum + 1, s);
        if (!o.skip_checks) {
            HIPCHK(hipMemcpyAsync(hflag, dflag, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hsum, dsum, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hflag[0]) return fail(FINOM_E_UNSORTED);
            if (hflag[1]) return fail(FINOM_E_MASS);
            if (!(fabs(hsum[0] - hsum[1]) <= 1e-12 * std::max(fabs(hsum[0]), fabs(hsum[1]))))
                return fail(FINOM_E_MASS);
        }
        setup_partition(x, n, y, m, T, zx, tx, s);
        setup_partition(y, m, x, n, T, zy, ty, s);
        hipLaunchKernelGGL(k_tile_rows, dim3(blocks_for(nt_c + 1)), dim3(kBlock), 0, s, zx, (long long)n, Tc, nt_c, tc);
        // Algorithm 1 initialisation: phi = 1/n, psi = 1/m (log2 units)
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, F, (long long)n, -log2((double)n));
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(m)), dim3(kBlock), 0, s, G[0], (long long)m, -log2((double)m));
        HIPCHK(hipGetLastError());
        ProbState init;
        memset(&init, 0, sizeof(init));
        init.itr_max = itr_max;
        init.tol = tol;
        hps[0] = init;
        memset(hps + 1, 0, sizeof(ProbState));
        HIPCHK(hipMemcpyAsync(ps, hps, 2 * sizeof(ProbState), hipMemcpyHostToDevice, s));

        // sweeps; buffer b: G[b] is the old psi, G[1-b] the new one
        SweepDev dkt[2], dk[2];
        for (int b = 0; b < 2; ++b) {
            LineDesc& a = kt[b].lines[0];
            a.zeta = zy; a.trs = ty; a.gin = F; a.out = G[1 - b];
            a.a0 = lv; a.a1 = v; a.a2 = G[b];
            a.part_base = 0; a.prob_part_off = 0; a.prob_nparts = a.ntiles;
            LineDesc& c = kk[b].lines[0];
            c.zeta = zx; c.trs = tx; c.gin = G[1 - b]; c.out = F; c.a0 = lu;
            dkt[b] = upload_sweep(al, kt[b], 2, eb, s);
            dk[b] = upload_sweep(al, kk[b], 2, eb, s);
        }
        HIPCHK(hipEventRecord(al.a->upload_done, s));

        // --- the loop: graphs of k iterations, one flag read per graph
        int k = o.graph_iters > 0 ? o.graph_iters : default_graph_iters((long long)(n + m) / 2);
        k += (k & 1);   // even, so every replay starts on buffer 0
        hipStream_t cs;
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = true;
        try {
            HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            for (int it = 0; it < k; ++it) {
                const int b = it & 1;
                launch_sweep(o.precision, IN_LOG2, EPI_UPDATE_CHECK, dkt[b], ps, partial, cs);
                launch_sweep(o.precision, IN_LOG2, EPI_UPDATE, dk[b], ps, nullptr, cs);
            }
            HIPCHK(hipStreamEndCapture(cs, &graph));
            HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        } catch (...) {
            ok = false;
        }
        if (!ok) {
            if (graph) hipGraphDestroy(graph);
            hipStreamDestroy(cs);
            return fail(FINOM_E_HIP);
        }
        long long launches = 0;
        const long long max_launches = itr_max / k + 2;
        int st = FINOM_OK;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        try {
            HIPCHK(hipEventCreate(&ev0));
            HIPCHK(hipEventCreate(&ev1));
            HIPCHK(hipEventRecord(ev0, s));
            for (;;) {
                HIPCHK(hipGraphLaunch(exec, s));
                ++launches;
                HIPCHK(hipMemcpyAsync(hps, ps, sizeof(ProbState), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (hps->done) break;
                if (launches > max_launches) {   // cannot happen unless the device state is corrupt
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
        }
        if (ev0) hipEventDestroy(ev0);
        if (ev1) hipEventDestroy(ev1);
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        hipStreamDestroy(cs);
        if (st != FINOM_OK) return fail(st);

        // --- returned pair: F and G[l % 2]; cost <C, Gamma> (moment sums, FP64)
        double* Gf = G[hps->iters & 1];
        LineDesc& c = kc.lines[0];
        c.zeta = zx; c.trs = tc; c.gin = Gf; c.a0 = F; c.out = nullptr;
        c.prob = 1;
        c.part_base = 0; c.prob_part_off = 0; c.prob_nparts = c.ntiles;
        SweepDev dc = upload_sweep(al, kc, 4, ebc, s);
        HIPCHK(hipEventRecord(al.a->upload_done, s));
        launch_cost_sweep(EPI_COST, dc, ps, partial, s);
        if (f_out)
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, s, F, f_out, (long long)n, eps * kLn2);
        if (g_out)
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(m)), dim3(kBlock), 0, s, Gf, g_out, (long long)m, eps * kLn2);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hps, ps, 2 * sizeof(ProbState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        res->w1 = hps[1].w1;
        res->marginal_err = hps->err;
        res->iters = hps->iters;
        res->sweeps = 2 * hps->iters + 1;
        res->converged = hps->converged;
        if (hps->status) return fail(FINOM_E_NUMERIC);
        return fail(hps->converged ? FINOM_OK : FINOM_NOT_CONVERGED);
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

void finom_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_arenas) {
        Arena* a = kv.second;
        if (a->upload_done) {
            hipEventSynchronize(a->upload_done);
            hipEventDestroy(a->upload_done);
        }
        if (a->dev) hipFree(a->dev);
        if (a->host) hipHostFree(a->host);
        delete a;
    }
    g_arenas.clear();
}

const char* finom_version(void) { return "finom-gfx950 0.1"; }

}  // extern "C"
