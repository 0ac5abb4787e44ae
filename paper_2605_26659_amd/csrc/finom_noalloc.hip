// finom_matvec_noalloc: the product K psi of finom_matvec (section 2.1's
// kernel, split at the dividing index of section 2.2 and evaluated by the
// recurrences of section 2.3) for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops). Everything the product
// needs beyond the caller's inputs and output - the dividing index, the
// merge-path tile starts, the work list, the line descriptor, the iteration
// state the sweep kernels read and the tile aggregates - lives in one
// file-scope device array of fixed size, so a call enqueues kernels only.
//
// The array is reached through its device address, which the host takes once
// per device with hipGetSymbolAddress (the array's name in host code is a
// host-side stand-in, not a device address). Each device holds its own copy
// until the process ends. Calls on one device share it: two calls that
// overlap on a device (different streams, or different host threads without
// ordering) race on it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/finom.h"
#include "finom_host.hpp"

namespace finom {
namespace {

// Layout of the scratch array. Tiles hold at least 512 merged points (the
// smallest tile shape), so FINOM_NOALLOC_MAX_POINTS merged points give at
// most kMaxTiles tiles.
constexpr long long kMaxMerged = FINOM_NOALLOC_MAX_POINTS;
constexpr int kMinTile = 512;
constexpr long long kMaxTiles = (kMaxMerged + kMinTile - 1) / kMinTile;
constexpr size_t al256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kOffState = 0;
constexpr size_t kOffLine = al256(kOffState + sizeof(ProbState));
constexpr size_t kOffWork = al256(kOffLine + sizeof(LineDesc));
constexpr size_t kOffTrs = al256(kOffWork + sizeof(WorkItem) * kMaxTiles);
constexpr size_t kOffAgg = al256(kOffTrs + sizeof(int) * (kMaxTiles + 1));
constexpr size_t kOffZeta = al256(kOffAgg + 2 * sizeof(Ext<double>) * kMaxTiles);
constexpr size_t kScratchBytes = al256(kOffZeta + sizeof(int) * kMaxMerged);
static_assert(kScratchBytes <= (17u << 20), "the scratch array stays below 17 MiB");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, taken once per
// device; nullptr (and the last-error text set) on failure.
unsigned char* scratch_address()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_last_error("finom_matvec_noalloc: no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[160];
            snprintf(msg, sizeof(msg), "finom_matvec_noalloc: hipGetSymbolAddress failed: %s (%d)",
                     hipGetErrorString(e), (int)e);
            set_last_error(msg);
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    return g_scratch_ptr[dev];
}

// Writes the line descriptor, the work list (one item per tile of line 0)
// and a cleared iteration state (the sweep kernels skip a state marked done).
__global__ __launch_bounds__(kBlock) void k_noalloc_setup(LineDesc L, int ntiles, LineDesc* __restrict__ line,
                                                         WorkItem* __restrict__ work, ProbState* __restrict__ ps)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < ntiles) work[t] = WorkItem{0, t};
    if (t == 0) {
        *line = L;
        ProbState z;
        memset(&z, 0, sizeof(z));
        *ps = z;
    }
}

}  // namespace
}  // namespace finom

using namespace finom;

extern "C" int finom_matvec_noalloc(const double* x_rows, int64_t n, const double* y_cols, int64_t m, double eps,
                                    const double* in, double* out, const finom_opts* opts, void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (!x_rows || !y_cols || !in || !out || n < 1 || m < 1 || !(eps > 0.0) || !std::isfinite(eps))
        return FINOM_E_ARG;
    if (o.precision != 0 && o.precision != 1) return FINOM_E_ARG;
    if (o.domain != 0 && o.domain != 1) return FINOM_E_ARG;
    if (n + m > kMaxMerged) {
        char msg[160];
        snprintf(msg, sizeof(msg), "finom_matvec_noalloc: n + m = %lld exceeds FINOM_NOALLOC_MAX_POINTS = %lld",
                 (long long)(n + m), kMaxMerged);
        set_last_error(msg);
        return FINOM_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char* base = scratch_address();
    if (!base) return FINOM_E_HIP;
    try {
        ProbState* ps = reinterpret_cast<ProbState*>(base + kOffState);
        LineDesc* dline = reinterpret_cast<LineDesc*>(base + kOffLine);
        WorkItem* work = reinterpret_cast<WorkItem*>(base + kOffWork);
        int* trs = reinterpret_cast<int*>(base + kOffTrs);
        void* agg = base + kOffAgg;
        int* zeta = reinterpret_cast<int*>(base + kOffZeta);

        // the tile shape finom_matvec takes for this size, so both give the same bits
        const int cfg = tuned_cfg(o.precision, n + m);
        const int T = kCfgs[cfg].T();
        if (T < kMinTile) throw HipError{hipErrorInvalidValue};
        enqueue_partition(x_rows, n, y_cols, m, T, zeta, trs, s);

        Sweep sw;
        sw.kind = 0;
        sw.cfg = cfg;
        sw.epi = (o.domain == 1) ? EPI_STORE_NAT : EPI_STORE_LIN;
        LineDesc L = make_line(x_rows, n, y_cols, m, zeta, trs, T, eps);
        L.gin = in;
        L.out = out;
        L.dec_part_off = -1;
        L.agg_base = 0;
        sw.lines.push_back(L);
        const int nt = L.ntiles;
        hipLaunchKernelGGL(k_noalloc_setup, dim3(blocks_for(nt)), dim3(kBlock), 0, s, L, nt, dline, work, ps);
        HIPCHK(hipGetLastError());
        sw.dev.work = work;
        sw.dev.nwork = nt;
        sw.dev.max_tiles = nt;
        sw.dev.max_dec = 0;
        sw.dev.work_multi = nt > 1 ? work : nullptr;
        sw.dev.nwork_multi = nt > 1 ? nt : 0;
        sw.dev.lines = dline;
        sw.dev.agg = agg;
        launch_sweep(o.precision, (o.domain == 1) ? IN_NAT : IN_LIN, sw, ps, nullptr, nullptr, 0, s);
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}
