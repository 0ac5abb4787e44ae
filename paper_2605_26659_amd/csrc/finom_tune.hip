// Tile-shape autotuner. For each length class of merged lines (2^9 .. 2^21
// elements) it times the update sweep of a batch of lines that fills the GPU
// (2^22 merged elements in all, distinct meshes and potentials per line) with
// every tile shape, and keeps the fastest shape for the class. The choice only
// changes how the work is tiled, never what is computed.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/finom.h"
#include "finom_host.hpp"

using namespace finom;

namespace {

// x_i = (i + 1/2)/n and y_j = (j + 1/4)/m for every line of the batch
__global__ void k_tune_meshes(double* __restrict__ X, long long n, double* __restrict__ Y, long long m,
                              long long count)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count * n) X[k] = ((double)(k % n) + 0.5) / (double)n;
    if (k < count * m) Y[k] = ((double)(k % m) + 0.25) / (double)m;
}

constexpr long long kTuneTotal = 1LL << 22;

// Seconds per launch of the update sweep over `count` lines of n + n
// elements with tile shape cfg.
double time_shape(Alloc& al, int precision, int cfg, long long n, long long count, const double* X,
                  const double* Y, const double* Gin, const double* A0, double* Out, ProbState* ps,
                  hipStream_t s)
{
    const int T = kCfgs[cfg].T();
    const size_t eb = ext_bytes(precision);
    const Part p = make_part(al, X, n, Y, n, T, s);
    Sweep sw;
    sw.kind = 0;
    sw.cfg = cfg;
    sw.epi = EPI_UPDATE;
    for (long long q = 0; q < count; ++q) {
        LineDesc L = make_line(X + q * n, n, Y + q * n, n, p.zeta, p.trs, T, 1e-2);
        L.gin = Gin + q * n;
        L.out = Out + q * n;
        L.a0 = A0 + q * n;
        L.dec_part_off = -1;
        sw.lines.push_back(L);
    }
    const int mt = sw.multi_tiles();
    if (mt > 0) {
        // as in the iteration: aggregates come from the previous epilogue
        sw.agg_from_prev = true;
        sw.agg_buf = al.dev<char>((size_t)mt * 2 * eb);
        sw.agg_next = al.dev<char>((size_t)mt * 2 * eb);
    }
    upload_sweep(al, sw, eb);
    if (mt > 0) launch_aggregate(precision, IN_LOG2, sw, ps, s);
    for (int w = 0; w < 3; ++w) launch_sweep(precision, IN_LOG2, sw, ps, nullptr, nullptr, 0, s);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int reps = 10;
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_sweep(precision, IN_LOG2, sw, ps, nullptr, nullptr, 0, s);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ms * 1e-3 / reps;
}

bool read_cache(const char* path, int precision)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char head[64] = {0};
    bool ok = fgets(head, sizeof(head), f) && strncmp(head, "finom-tune 1", 12) == 0;
    int cfg[kTuneClasses] = {0};
    unsigned got = 0;
    int p, c, v;
    while (ok && fscanf(f, "%d %d %d", &p, &c, &v) == 3) {
        if (p != precision) continue;
        if (c < 0 || c >= kTuneClasses || v < 0 || v >= kNumCfg) {
            ok = false;
            break;
        }
        cfg[c] = v;
        got |= 1u << c;
    }
    fclose(f);
    if (!ok || got != (1u << kTuneClasses) - 1) return false;
    for (int k = 0; k < kTuneClasses; ++k) set_tuned_cfg(precision, k, cfg[k]);
    return true;
}

void write_cache(const char* path)
{
    // keep the other precision's entries if the file already holds them
    int old[2][kTuneClasses];
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < kTuneClasses; ++c) old[p][c] = get_tuned_cfg(p, c);
    FILE* f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "finom-tune 1\n");
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < kTuneClasses; ++c)
            if (old[p][c] >= 0) fprintf(f, "%d %d %d\n", p, c, old[p][c]);
    fclose(f);
}

}  // namespace

extern "C" {

int finom_autotune(int32_t precision, const char* cache_path, void* stream)
{
    if (precision != 0 && precision != 1) return FINOM_E_ARG;
    if (cache_path && *cache_path && read_cache(cache_path, precision)) return FINOM_OK;
    hipStream_t s = (hipStream_t)stream;
    try {
        Alloc al(stream);
        const long long cap_n = kTuneTotal / 2;
        double* X = al.dev<double>(cap_n);
        double* Y = al.dev<double>(cap_n);
        double* Gin = al.dev<double>(cap_n);
        double* A0 = al.dev<double>(cap_n);
        double* Out = al.dev<double>(cap_n);
        ProbState* ps = al.dev<ProbState>(1);
        HIPCHK(hipMemsetAsync(Gin, 0, sizeof(double) * cap_n, s));
        HIPCHK(hipMemsetAsync(A0, 0, sizeof(double) * cap_n, s));
        HIPCHK(hipMemsetAsync(ps, 0, sizeof(ProbState), s));
        int best[kTuneClasses];
        for (int c = 0; c < kTuneClasses; ++c) {
            const long long L = 512LL << c;       // merged elements per line
            const long long n = L / 2;            // n = m
            const long long count = std::max(1LL, kTuneTotal / L);
            hipLaunchKernelGGL(k_tune_meshes, dim3(blocks_for(count * n)), dim3(kBlock), 0, s, X, n, Y, n, count);
            HIPCHK(hipGetLastError());
            double tbest = 0.0;
            best[c] = 0;
            for (int cfg = 0; cfg < kNumCfg; ++cfg) {
                const double t = time_shape(al, precision, cfg, n, count, X, Y, Gin, A0, Out, ps, s);
                if (cfg == 0 || t < tbest) {
                    tbest = t;
                    best[c] = cfg;
                }
            }
        }
        al.uploaded();
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < kTuneClasses; ++c) set_tuned_cfg(precision, c, best[c]);
        if (cache_path && *cache_path) write_cache(cache_path);
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

int finom_tile_config(int32_t precision, int64_t merged)
{
    if (precision != 0 && precision != 1) return FINOM_E_ARG;
    return tuned_cfg(precision, merged);
}

}  // extern "C"
