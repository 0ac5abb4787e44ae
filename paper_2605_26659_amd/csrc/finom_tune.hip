// Tile-shape autotuner. For each length class of merged lines (2^9 .. 2^21
// elements) it times a batch of lines that fills the GPU (2^22 merged elements
// in all, distinct meshes per line) with every tile shape, and keeps the
// fastest shape for the class. A class runs where its problems will run: the
// streaming sweeps (one iteration's two sweeps over all lines), or, in FP32
// where some shape lets a line of the class run on the resident solver, the
// resident batch grid (a fixed number of iterations of every line as one batch,
// its grid timed by HIP events), among the shapes that keep it there. The
// choice only changes how the work is tiled, never what is computed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

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

__global__ void k_tune_fill(double* __restrict__ a, long long n, double v)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = v;
}

constexpr long long kTuneTotal = 1LL << 22;

__global__ void k_tune_fill_ext(Ext<float>* __restrict__ a, long long n, float m, int e)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = Ext<float>{m, e};
}

// 2^{c kappa} (called with 2 kappa: B of the fast sweeps)
__global__ void k_tune_exp(const double* __restrict__ c, long long n, double kappa, Ext<float>* __restrict__ E)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) E[i] = split_exp2(c[i] * kappa);
}

struct TuneArrays {
    double *X, *Y, *F, *G0, *G1, *LU, *LV, *V;
    double* M;   // masses of the resident timings
    Ext<float>*EX, *EY;
    ProbState* ps;
};

// Seconds per Sinkhorn iteration (the checking K^T phi sweep and the K psi
// sweep with its stop decision, tile aggregates passed between them) over
// `count` lines of n + n elements with tile shape cfg. FP32 runs the fast
// sweeps (eps = 1 keeps every tile inside their range), FP64 the general ones.
double time_pair(Alloc& al, int precision, int cfg, long long n, long long count, const TuneArrays& A,
                 hipStream_t s)
{
    const int T = kCfgs[cfg].T();
    const size_t eb = ext_bytes(precision);
    const bool fast = precision == 1;
    const double eps = fast ? 1.0 : 1e-2;
    const Part pk = make_part(al, A.X, n, A.Y, n, T, s);
    const Part pkt = make_part_transposed(al, pk, s);
    Sweep kt, kk;
    kt.cfg = kk.cfg = cfg;
    kt.epi = EPI_UPDATE_CHECK;
    kk.epi = EPI_UPDATE;
    kt.fast = kk.fast = fast;
    for (long long q = 0; q < count; ++q) {
        const long long o = q * n;
        LineDesc a = make_line(A.Y + o, n, A.X + o, n, pkt.zeta, pkt.trs, T, eps);
        a.gin = A.F + o;
        a.out = A.G1 + o;
        a.a0 = A.LV + o;
        a.a1 = A.V + o;
        a.a2 = A.G0 + o;
        a.dec_part_off = -1;
        LineDesc c = make_line(A.X + o, n, A.Y + o, n, pk.zeta, pk.trs, T, eps);
        c.gin = A.G1 + o;
        c.out = A.F + o;
        c.a0 = A.LU + o;
        if (fast) {
            a.er = A.EY + o;
            a.ec = A.EX + o;
            c.er = A.EX + o;
            c.ec = A.EY + o;
        }
        kt.lines.push_back(a);
        kk.lines.push_back(c);
    }
    assign_parts(kt, 0);
    for (size_t q = 0; q < kk.lines.size(); ++q) {
        kk.lines[q].dec_part_off = kt.lines[q].part_base;
        kk.lines[q].dec_nparts = kt.lines[q].ntiles;
        kk.lines[q].writes_state = 1;
    }
    const int mt = kt.multi_tiles();
    if (mt > 0) {
        void* agg_kt = al.dev<char>((size_t)mt * 2 * eb);
        void* agg_k = al.dev<char>((size_t)mt * 2 * eb);
        kt.agg_from_prev = kk.agg_from_prev = true;
        kt.agg_buf = agg_kt;
        kt.agg_next = agg_k;
        kk.agg_buf = agg_k;
        kk.agg_next = agg_kt;
    }
    upload_sweep(al, kt, eb);
    upload_sweep(al, kk, eb);
    double* partial = al.dev<double>(std::max(kt.total_tiles(), 1));
    if (mt > 0) launch_aggregate(precision, IN_LOG2, kt, A.ps, s);
    auto iteration = [&](int b) {
        launch_sweep(precision, IN_LOG2, kt, A.ps, partial, nullptr, b, s);
        launch_sweep(precision, IN_LOG2, kk, A.ps, partial, partial, b, s);
    };
    for (int w = 0; w < 2; ++w) iteration(w & 1);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // best of three timings of 8 iterations each
    const int reps = 8;
    float best = 0.f;
    for (int trial = 0; trial < 3; ++trial) {
        HIPCHK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) iteration(r & 1);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (trial == 0 || ms < best) best = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best * 1e-3 / reps;
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
        if (c < 0 || c >= kTuneClasses || v < 0 || v >= kNumTunedCfg) {
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

// Iterations of each resident timing; even, so both sweeps of an iteration
// and the loop head are timed alike for every shape.
constexpr long long kTuneResidentIters = 64;

// Seconds of the resident batch grid that runs kTuneResidentIters iterations
// (tol 0) of `count` FP32 problems of n + n points, uniform masses `mass`, with
// tile shape cfg for their size class cls: the best of two timed calls after
// one warm-up. Every member of such a batch reports the grid's time.
double time_resident(int cls, int cfg, long long n, long long count, const TuneArrays& A, const double* mass,
                     hipStream_t s)
{
    set_tuned_cfg(1, cls, cfg);
    std::vector<finom_problem> pr((size_t)count);
    std::vector<finom_result> rs((size_t)count);
    for (long long q = 0; q < count; ++q) {
        finom_problem& p = pr[(size_t)q];
        memset(&p, 0, sizeof(p));
        p.dim = 1;
        p.n1 = p.n2 = n;   // dim 1: x = x1, y = x2
        p.x1 = A.X + q * n;
        p.x2 = A.Y + q * n;
        p.u = p.v = mass + q * n;
        p.eps = 1.0;   // every tile inside the fast sweeps' range, as in time_pair
        p.tol = 0.0;
        p.itr_max = kTuneResidentIters;
        p.f_out = A.F + q * n;
        p.g_out = A.G0 + q * n;
    }
    finom_opts o;
    memset(&o, 0, sizeof(o));
    o.precision = 1;
    o.skip_checks = 1;
    double best = 0.0;
    for (int trial = 0; trial < 3; ++trial) {
        const int rc = finom_batch(pr.data(), count, &o, rs.data(), s);
        if (rc < 0) throw StatusError{rc};
        double ms = 0.0;
        for (const finom_result& r : rs) ms = std::max(ms, r.loop_ms);
        if (trial == 1 || (trial > 1 && ms < best)) best = ms;
    }
    return best * 1e-3;
}

}  // namespace

extern "C" {

int finom_autotune(int32_t precision, const char* cache_path, void* stream)
{
    if (precision != 0 && precision != 1) return FINOM_E_ARG;
    if (cache_path && *cache_path && read_cache(cache_path, precision)) return FINOM_OK;
    hipStream_t s = (hipStream_t)stream;
    // The tuner's buffers come from a workspace of its own: the resident
    // timings call finom_batch on the same stream, and a call restarts the
    // stream's workspace from its first block.
    Arena own;
    int rc = FINOM_OK;
    try {
        Alloc al(&own, s);
        const long long cap_n = kTuneTotal / 2;
        TuneArrays A;
        double** dbl[8] = {&A.X, &A.Y, &A.F, &A.G0, &A.G1, &A.LU, &A.LV, &A.V};
        for (double** d : dbl) *d = al.dev<double>(cap_n);
        A.M = al.dev<double>(cap_n);
        A.EX = al.dev<Ext<float>>(cap_n);
        A.EY = al.dev<Ext<float>>(cap_n);
        A.ps = al.dev<ProbState>(1);
        if (precision == 1) {
            // the fast sweeps' state (U = 1) and masses (2^-21) as Ext<float>
            for (double* d : {A.F, A.G0, A.G1})
                hipLaunchKernelGGL(k_tune_fill_ext, dim3(blocks_for(cap_n)), dim3(kBlock), 0, s, (Ext<float>*)d,
                                   cap_n, 1.0f, 0);
            for (double* d : {A.LU, A.LV})
                hipLaunchKernelGGL(k_tune_fill_ext, dim3(blocks_for(cap_n)), dim3(kBlock), 0, s, (Ext<float>*)d,
                                   cap_n, 1.0f, -21);
        } else {
            for (double* d : {A.F, A.G0, A.G1, A.LU, A.LV}) HIPCHK(hipMemsetAsync(d, 0, sizeof(double) * cap_n, s));
        }
        // V: weights of the error terms; never stop (tolerance below any error)
        hipLaunchKernelGGL(k_tune_fill, dim3(blocks_for(cap_n)), dim3(kBlock), 0, s, A.V, cap_n, 1.0 / (double)cap_n);
        ProbState* hst = al.host<ProbState>(1);
        memset(hst, 0, sizeof(ProbState));
        hst->itr_max = 1LL << 60;
        hst->tol = -1.0;
        HIPCHK(hipMemcpyAsync(A.ps, hst, sizeof(ProbState), hipMemcpyHostToDevice, s));
        int best[kTuneClasses];
        for (int c = 0; c < kTuneClasses; ++c) {
            const long long L = 512LL << c;       // merged elements per line
            const long long n = L / 2;            // n = m
            const long long count = std::max(1LL, kTuneTotal / L);
            hipLaunchKernelGGL(k_tune_meshes, dim3(blocks_for(count * n)), dim3(kBlock), 0, s, A.X, n, A.Y, n, count);
            hipLaunchKernelGGL(k_tune_exp, dim3(blocks_for(count * n)), dim3(kBlock), 0, s, A.X, count * n,
                               2.0 / kLn2, A.EX);
            hipLaunchKernelGGL(k_tune_exp, dim3(blocks_for(count * n)), dim3(kBlock), 0, s, A.Y, count * n,
                               2.0 / kLn2, A.EY);
            HIPCHK(hipGetLastError());
            // FP32 problems whose tiles fit the resident solver at once run
            // there (one launch per solve): where some shape lets a line of this
            // class fit, only such shapes are candidates, so that tuning never
            // moves a problem off the resident solver
            bool allowed[kNumTunedCfg];
            bool any_resident = false;
            for (int cfg = 0; cfg < kNumTunedCfg; ++cfg) {
                allowed[cfg] = precision == 1 && fast_allowed() && resident_fits(n, n, kCfgs[cfg].T(), false);
                any_resident = any_resident || allowed[cfg];
            }
            // The resident solver sees a shape only through the tiles it cuts a
            // line into: shapes that tile the class's lines alike (the whole
            // line in one tile, or the same tile length) are timed there once.
            // Among the shapes of the fastest tiling, the streaming sweeps
            // decide, as they do for every class without a resident shape:
            // the class's lines take them on the other paths (d-dimensional
            // and general sweeps, problems beyond the resident bound).
            int tiling[kNumTunedCfg];
            int win = -1;
            if (any_resident) {
                hipLaunchKernelGGL(k_tune_fill, dim3(blocks_for(count * n)), dim3(kBlock), 0, s, A.M, count * n,
                                   1.0 / (double)n);
                double twin = 0.0;
                for (int cfg = 0; cfg < kNumTunedCfg; ++cfg) {
                    const int T = kCfgs[cfg].T();
                    tiling[cfg] = 2 * n <= T ? 0 : T;
                    if (!allowed[cfg]) continue;
                    bool seen = false;
                    for (int o = 0; o < cfg; ++o) seen = seen || (allowed[o] && tiling[o] == tiling[cfg]);
                    if (seen) continue;
                    const double t = time_resident(c, cfg, n, count, A, A.M, s);
                    if (win < 0 || t < twin) {
                        twin = t;
                        win = tiling[cfg];
                    }
                }
            }
            double tbest = 0.0;
            best[c] = -1;
            for (int cfg = 0; cfg < kNumTunedCfg; ++cfg) {
                if (any_resident && (!allowed[cfg] || tiling[cfg] != win)) continue;
                const double t = time_pair(al, precision, cfg, n, count, A, s);
                if (best[c] < 0 || t < tbest) {
                    tbest = t;
                    best[c] = cfg;
                }
            }
        }
        al.uploaded();
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < kTuneClasses; ++c) set_tuned_cfg(precision, c, best[c]);
        if (cache_path && *cache_path) write_cache(cache_path);
    } catch (...) {
        rc = map_exception();
    }
    hipStreamSynchronize(s);
    arena_free(&own);
    return rc;
}

int finom_tile_config(int32_t precision, int64_t merged)
{
    if (precision != 0 && precision != 1) return FINOM_E_ARG;
    return tuned_cfg(precision, merged);
}

}  // extern "C"
