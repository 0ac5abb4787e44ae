// Batch engine (see finom_engine.hpp) and the batched entry point.
//
// Setup runs as a handful of launches over task tables that cover every new
// problem at once (validation, log masses, initial potentials, dividing
// indices, merge-path partitions). The iteration merges the lines of all live
// problems into one sweep launch per (stage, tile shape); the stages of an
// iteration are, in order, 1D K^T phi (+ check), 1D K psi (+ stop decision),
// 2D K_x^T, K_y^T (+ check), K_x (+ stop decision), K_y. Each line carries
// its problem's state index, so every problem runs Algorithm 1 / Algorithm 2
// exactly as it would alone, with its own counter, tolerance and cap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <tuple>

#include "finom_engine.hpp"
#include "finom_resident.hpp"

namespace finom {

// ---------------------------------------------------------------------------
// task-table setup kernels: block b of a launch works on the task whose
// block range [first[t], first[t+1]) contains b
// ---------------------------------------------------------------------------
__device__ __forceinline__ int task_of(const int* __restrict__ first, int ntasks, int b)
{
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct ArrTask {
    const double* a;
    long long n;
    double* la;          // masses: log2 of each entry
    double* fill;        // optional: potential initialisation
    long long nfill;
    double fill_v;
    double kappa;        // meshes: 1 / (eps ln 2)
    int kind;            // 0 mesh, 1 mass
    int job;
    int slot;            // masses: 0 source, 1 target
    int checks;
};

// flags[job] |= 1 (mesh decreasing or non-finite), 2 (mass not > 0 or not
// finite), 4 (|coordinate| / (eps ln 2) out of range); mass partial sums.
__global__ __launch_bounds__(kBlock) void k_setup_arrays(const ArrTask* __restrict__ tasks,
                                                        const int* __restrict__ first, int ntasks,
                                                        int* __restrict__ flags, double* __restrict__ part)
{
    __shared__ double s_red[kBlock / kWave];
    const int ti = task_of(first, ntasks, blockIdx.x);
    const ArrTask t = tasks[ti];
    const int lb = blockIdx.x - first[ti];
    const long long stride = (long long)(first[ti + 1] - first[ti]) * kBlock;
    int bad = 0;
    double acc = 0.0;
    for (long long k = (long long)lb * kBlock + threadIdx.x; k < t.n; k += stride) {
        const double v = t.a[k];
        if (t.kind == 0) {
            if (t.checks) {
                if (!(fabs(v) * t.kappa < kCoordLimit)) bad |= (v == v && fabs(v) != __builtin_inf()) ? 4 : 1;
                if (k + 1 < t.n && v > t.a[k + 1]) bad |= 1;
            }
        } else {
            if (!(v > 0.0) || v == __builtin_inf()) bad |= 2;
            t.la[k] = log2(v);
            acc += v;
        }
    }
    if (t.fill)
        for (long long k = (long long)lb * kBlock + threadIdx.x; k < t.nfill; k += stride) t.fill[k] = t.fill_v;
    if (bad) atomicOr(flags + t.job, bad);
    if (t.kind == 1) {
        acc = block_sum_f64<kBlock>(acc, s_red);
        if (threadIdx.x == 0) part[blockIdx.x] = acc;
    }
}

__global__ void k_setup_sums(const ArrTask* __restrict__ tasks, const int* __restrict__ first, int ntasks,
                             const double* __restrict__ part, double* __restrict__ sums)
{
    const int ti = blockIdx.x * blockDim.x + threadIdx.x;
    if (ti >= ntasks) return;
    const ArrTask t = tasks[ti];
    if (t.kind != 1) return;
    double s = 0.0;
    for (int b = first[ti]; b < first[ti + 1]; ++b) s += part[b];
    sums[2 * t.job + t.slot] = s;
}

struct PairTask {
    const double* xr;
    const double* yc;
    long long R, C;
    int* zeta;           // rows xr over columns yc: #{j : yc_j <= xr_i}
    int* zeta_t;         // rows yc over columns xr: #{i : xr_i <= yc_j}
    int* trs;            // merge-path tile row starts of (xr, yc)
    int* trs_t;          // of the transposed pair on the same tiles
    int* trs_c;          // of (xr, yc) at the cost tile size
    int T, ntiles, Tc, ntiles_c;
};

// task 2p: zeta of pair p; task 2p + 1: zeta_t of pair p
__global__ __launch_bounds__(kBlock) void k_setup_zeta(const PairTask* __restrict__ P, const int* __restrict__ first,
                                                      int ntasks)
{
    const int ti = task_of(first, ntasks, blockIdx.x);
    const PairTask p = P[ti >> 1];
    const bool tr = (ti & 1) != 0;
    const double* rows = tr ? p.yc : p.xr;
    const double* cols = tr ? p.xr : p.yc;
    const long long nr = tr ? p.C : p.R;
    const long long nc = tr ? p.R : p.C;
    int* z = tr ? p.zeta_t : p.zeta;
    const int lb = blockIdx.x - first[ti];
    const long long stride = (long long)(first[ti + 1] - first[ti]) * kBlock;
    for (long long i = (long long)lb * kBlock + threadIdx.x; i < nr; i += stride) {
        const double x = rows[i];
        long long lo = 0, hi = nc;
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            if (cols[mid] <= x) lo = mid + 1;
            else hi = mid;
        }
        z[i] = (int)lo;
    }
}

__device__ __forceinline__ int merge_rows_before(const int* __restrict__ zeta, long long R, long long d)
{
    long long lo = 0, hi = R;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (mid + zeta[mid] < d) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo;
}

__global__ __launch_bounds__(kBlock) void k_setup_tiles(const PairTask* __restrict__ P, const int* __restrict__ first,
                                                       int ntasks)
{
    const int ti = task_of(first, ntasks, blockIdx.x);
    const PairTask p = P[ti];
    const int lb = blockIdx.x - first[ti];
    const int stride = (first[ti + 1] - first[ti]) * kBlock;
    const long long total = p.R + p.C;
    for (int t = lb * kBlock + threadIdx.x; t <= p.ntiles; t += stride) {
        const int r = (t == p.ntiles) ? (int)p.R : merge_rows_before(p.zeta, p.R, (long long)t * p.T);
        p.trs[t] = r;
        const long long d = ((long long)t * p.T < total) ? (long long)t * p.T : total;
        p.trs_t[t] = (int)(d - r);
    }
    for (int t = lb * kBlock + threadIdx.x; t <= p.ntiles_c; t += stride)
        p.trs_c[t] = (t == p.ntiles_c) ? (int)p.R : merge_rows_before(p.zeta, p.R, (long long)t * p.Tc);
}

struct StateInit {
    int slot;
    int pad;
    long long itr_max;
    double tol;
};

__global__ void k_init_states(const StateInit* __restrict__ in, int n, ProbState* __restrict__ ps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    ProbState s{};
    s.itr_max = in[k].itr_max;
    s.tol = in[k].tol;
    ps[in[k].slot] = s;
}

struct SegTask {
    int off, n;
    double* out;
};

// Sum of partial slots [off, off + n) per task (one block each), in the same
// order as the single-problem reduction.
__global__ __launch_bounds__(kBlock) void k_segment_sums(const double* __restrict__ partial,
                                                        const SegTask* __restrict__ segs)
{
    __shared__ double s_red[kBlock / kWave];
    const SegTask t = segs[blockIdx.x];
    double v = 0.0;
    for (int k = threadIdx.x; k < t.n; k += kBlock) v += partial[t.off + k];
    v = block_sum_f64<kBlock>(v, s_red);
    if (threadIdx.x == 0) *t.out = v;
}

// b = f a over n elements. mode 0: same layout; mode 1: a is a column-major
// grid of `rows` rows, b receives it row-major; mode 2: a is row-major, b
// receives it column-major.
struct ScaleTask {
    const double* a;
    double* b;
    long long n;
    double f;
    long long rows;
    int mode;
};

__global__ __launch_bounds__(kBlock) void k_scale_tasks(const ScaleTask* __restrict__ tasks,
                                                       const int* __restrict__ first, int ntasks)
{
    const int ti = task_of(first, ntasks, blockIdx.x);
    const ScaleTask t = tasks[ti];
    const int lb = blockIdx.x - first[ti];
    const long long stride = (long long)(first[ti + 1] - first[ti]) * kBlock;
    const long long cols = t.rows > 0 ? t.n / t.rows : 0;
    for (long long k = (long long)lb * kBlock + threadIdx.x; k < t.n; k += stride) {
        long long src = k;
        if (t.mode == 1) {
            const long long l = k / cols;
            src = l + (k - l * cols) * t.rows;
        } else if (t.mode == 2) {
            const long long j = k / t.rows;
            src = j + (k - j * t.rows) * cols;
        }
        t.b[k] = t.a[src] * t.f;
    }
}

// blocks given to a task of n elements (at least one, at most 1024)
static int task_blocks(long long n)
{
    const long long per = (long long)kBlock * 8;
    return (int)std::min<long long>(1024, std::max<long long>(1, (n + per - 1) / per));
}

// Copies a host vector to device memory carved from `al` (pinned staging).
template <typename T>
static T* upload_vec(Alloc& al, const std::vector<T>& v)
{
    const size_t n = std::max<size_t>(v.size(), 1);
    T* h = al.host<T>(n);
    T* d = al.dev<T>(n);
    if (!v.empty()) {
        memcpy(h, v.data(), sizeof(T) * v.size());
        HIPCHK(hipMemcpyAsync(d, h, sizeof(T) * v.size(), hipMemcpyHostToDevice, al.s));
    }
    return d;
}

static std::vector<int> prefix_blocks(const std::vector<long long>& sizes)
{
    std::vector<int> first(sizes.size() + 1, 0);
    for (size_t i = 0; i < sizes.size(); ++i) first[i + 1] = first[i] + task_blocks(sizes[i]);
    return first;
}

// ---------------------------------------------------------------------------
// jobs
// ---------------------------------------------------------------------------
JobDesc job_from_problem(const finom_problem& p)
{
    JobDesc d;
    d.dim = p.dim;
    d.n1 = p.n1;
    d.n2 = p.n2;
    d.m1 = p.dim == 2 ? p.m1 : 1;
    d.m2 = p.dim == 2 ? p.m2 : 1;
    d.x1 = p.x1;
    d.x2 = p.x2;
    d.y1 = p.dim == 2 ? p.y1 : nullptr;
    d.y2 = p.dim == 2 ? p.y2 : nullptr;
    d.u = p.u;
    d.v = p.v;
    d.eps = p.eps;
    d.tol = p.tol;
    d.itr_max = p.itr_max;
    d.f_out = p.f_out;
    d.g_out = p.g_out;
    return d;
}

int check_job_args(const JobDesc& d, int precision)
{
    if (precision != 0 && precision != 1) return FINOM_E_ARG;
    if (d.dim != 1 && d.dim != 2) return FINOM_E_ARG;
    if (!d.x1 || !d.x2 || !d.u || !d.v) return FINOM_E_ARG;
    if (!(std::isfinite(d.eps) && d.eps > 0.0)) return FINOM_E_ARG;
    if (!(d.tol >= 0.0) || !std::isfinite(d.tol) || d.itr_max < 0) return FINOM_E_ARG;
    if (d.n1 < 1 || d.n2 < 1) return FINOM_E_ARG;
    if (d.n1 + d.n2 > (long long)INT32_MAX) return FINOM_E_ARG;
    if (d.dim == 2) {
        if (!d.y1 || !d.y2 || d.m1 < 1 || d.m2 < 1) return FINOM_E_ARG;
        if (d.m1 + d.m2 > (long long)INT32_MAX) return FINOM_E_ARG;
        if (d.n1 * d.m1 > (1LL << 40) || d.n2 * d.m2 > (1LL << 40)) return FINOM_E_ARG;
    }
    return FINOM_OK;
}

JobPlan plan_job(const JobDesc& d, int precision)
{
    JobPlan p;
    p.dim = d.dim;
    const int Tc = cost_tile_size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = align_up(off, 256);
        off = o + std::max<size_t>(bytes, 1);
        return o;
    };
    p.R[0] = d.n1;
    p.C[0] = d.n2;
    if (d.dim == 1) {
        p.na = d.n1;
        p.nb = d.n2;
    } else {
        p.R[1] = d.m1;
        p.C[1] = d.m2;
        p.na = d.n1 * d.m1;
        p.nb = d.n2 * d.m2;
        p.s_len = d.n2 * d.m1;
    }
    p.o_lu = take(8 * p.na);
    p.o_lv = take(8 * p.nb);
    p.o_F = take(8 * p.na);
    p.o_G0 = take(8 * p.nb);
    p.o_G1 = take(8 * p.nb);
    if (d.dim == 2) {
        p.o_S = take(8 * p.s_len);
        p.o_lvr = take(8 * p.nb);
        p.o_vr = take(8 * p.nb);
    }
    if (d.dim == 1 && precision == 1) {
        p.o_Bx = take(sizeof(Ext<float>) * p.na);
        p.o_By = take(sizeof(Ext<float>) * p.nb);
    }
    if (d.dim == 2) {
        p.lx_shape = ext2d_shape(d.n1, d.m1, d.n2, d.m2, precision);
        if (p.lx_shape >= 0) p.o_lx = take(ext2d_bytes(d.n1, d.m1, d.n2, d.m2));
    }
    for (int a = 0; a < d.dim; ++a) {
        p.cfg[a] = d.dim == 2 ? short_line_cfg(precision, p.R[a] + p.C[a]) : tuned_cfg(precision, p.R[a] + p.C[a]);
        const int T = kCfgs[p.cfg[a]].T();
        p.ntiles[a] = ntiles_for(p.R[a], p.C[a], T);
        p.ntiles_c[a] = ntiles_for(p.R[a], p.C[a], Tc);
        p.o_zeta[a] = take(4 * p.R[a]);
        p.o_zeta_t[a] = take(4 * p.C[a]);
        p.o_trs[a] = take(4 * (size_t)(p.ntiles[a] + 1));
        p.o_trs_t[a] = take(4 * (size_t)(p.ntiles[a] + 1));
        p.o_trs_c[a] = take(4 * (size_t)(p.ntiles_c[a] + 1));
    }
    p.bytes = align_up(off, 256);
    return p;
}

void Job::bind()
{
    lu = (double*)(mem + p.o_lu);
    lv = (double*)(mem + p.o_lv);
    F = (double*)(mem + p.o_F);
    G[0] = (double*)(mem + p.o_G0);
    G[1] = (double*)(mem + p.o_G1);
    S = d.dim == 2 ? (double*)(mem + p.o_S) : nullptr;
    lvr = d.dim == 2 ? (double*)(mem + p.o_lvr) : nullptr;
    vr = d.dim == 2 ? (double*)(mem + p.o_vr) : nullptr;
    Bx = p.o_Bx ? (Ext<float>*)(mem + p.o_Bx) : nullptr;
    By = p.o_By ? (Ext<float>*)(mem + p.o_By) : nullptr;
    if (p.lx_shape >= 0) ext2d_bind(lx, mem + p.o_lx, d.n1, d.m1, d.n2, d.m2, p.lx_shape);
    const int Tc = cost_tile_size();
    for (int a = 0; a < d.dim; ++a) {
        const double* xr = a == 0 ? d.x1 : d.y1;
        const double* yc = a == 0 ? d.x2 : d.y2;
        const long long R = p.R[a], C = p.C[a];
        const int T = kCfgs[p.cfg[a]].T();
        int* zeta = (int*)(mem + p.o_zeta[a]);
        int* zeta_t = (int*)(mem + p.o_zeta_t[a]);
        pk[a] = part_view(xr, R, yc, C, zeta, (int*)(mem + p.o_trs[a]), T);
        pkt[a] = part_view(yc, C, xr, R, zeta_t, (int*)(mem + p.o_trs_t[a]), T);
        pc[a] = part_view(xr, R, yc, C, zeta, (int*)(mem + p.o_trs_c[a]), Tc);
    }
}

static long long job_tiles(const Job& j)
{
    if (j.d.dim == 1) return 2LL * j.p.ntiles[0];
    return (j.d.m1 + j.d.m2) * (long long)j.p.ntiles[0] + (j.d.n1 + j.d.n2) * (long long)j.p.ntiles[1];
}

// ---------------------------------------------------------------------------
// engine
// ---------------------------------------------------------------------------
Engine::Engine(int precision, hipStream_t stream, int capacity, bool use_graphs)
    : precision_(precision), s_(stream), cap_(std::max(capacity, 1)), use_graphs_(use_graphs)
{
    HIPCHK(hipMalloc((void**)&ps_, sizeof(ProbState) * (cap_ + 1)));
    if (hipHostMalloc((void**)&hps_, sizeof(ProbState) * (cap_ + 1), hipHostMallocDefault) != hipSuccess) {
        hipFree(ps_);
        throw std::bad_alloc();
    }
    memset(hps_, 0, sizeof(ProbState) * (cap_ + 1));
    // every state not done (a job's state is set when it starts), and the
    // cost sweeps' state (never done)
    HIPCHK(hipMemsetAsync(ps_, 0, sizeof(ProbState) * (cap_ + 1), s_));
    for (int i = 0; i < cap_; ++i) free_slots_.push(i);
    HIPCHK(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&ev0_));
    HIPCHK(hipEventCreate(&ev1_));
    HIPCHK(hipStreamCreateWithFlags(&s2_, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&ev2_));
    HIPCHK(hipEventCreate(&ev3_));
    HIPCHK(hipEventCreateWithFlags(&evu_, hipEventDisableTiming));
}

Engine::~Engine()
{
    drop_graph();
    hipStreamSynchronize(s_);
    arena_free(&ar_setup_);
    arena_free(&ar_loop_);
    arena_free(&ar_cost_);
    arena_free(&ar_res_);
    arena_free(&ar_chk_);
    if (ev0_) hipEventDestroy(ev0_);
    if (ev1_) hipEventDestroy(ev1_);
    if (s2_) {
        hipStreamSynchronize(s2_);
        hipStreamDestroy(s2_);
    }
    if (ev2_) hipEventDestroy(ev2_);
    if (ev3_) hipEventDestroy(ev3_);
    if (evu_) hipEventDestroy(evu_);
    if (cs_) hipStreamDestroy(cs_);
    hipFree(ps_);
    hipHostFree(hps_);
}

void Engine::drop_graph()
{
    if (exec_) hipGraphExecDestroy(exec_);
    if (graph_) hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
    graph_k_ = 0;
}

void Engine::setup(const std::vector<Job*>& jobs, bool checks)
{
    if (jobs.empty()) return;
    Alloc al(&ar_setup_, s_);
    const int nj = (int)jobs.size();
    std::vector<ArrTask> at;
    std::vector<long long> at_n;
    std::vector<PairTask> pt;
    std::vector<long long> z_n, t_n;
    for (int i = 0; i < nj; ++i) {
        Job* j = jobs[i];
        const JobDesc& d = j->d;
        const double kappa = 1.0 / (d.eps * kLn2);
        auto mesh = [&](const double* a, long long n) {
            if (!checks) return;
            ArrTask t;
            memset(&t, 0, sizeof(t));
            t.a = a;
            t.n = n;
            t.kind = 0;
            t.job = i;
            t.kappa = kappa;
            t.checks = checks ? 1 : 0;
            at.push_back(t);
            at_n.push_back(n);
        };
        mesh(d.x1, d.n1);
        mesh(d.x2, d.n2);
        if (d.dim == 2) {
            mesh(d.y1, d.m1);
            mesh(d.y2, d.m2);
        }
        auto mass = [&](const double* a, long long n, double* la, double* fill, int slot) {
            ArrTask t;
            memset(&t, 0, sizeof(t));
            t.a = a;
            t.n = n;
            t.la = la;
            t.fill = fill;
            t.nfill = n;
            t.fill_v = -log2((double)n);
            t.kind = 1;
            t.job = i;
            t.slot = slot;
            at.push_back(t);
            at_n.push_back(n);
        };
        mass(d.u, j->p.na, j->lu, j->F, 0);
        mass(d.v, j->p.nb, j->lv, j->G[0], 1);
        for (int a = 0; a < d.dim; ++a) {
            PairTask q;
            memset(&q, 0, sizeof(q));
            q.xr = j->pk[a].xr;
            q.yc = j->pk[a].yc;
            q.R = j->pk[a].R;
            q.C = j->pk[a].C;
            q.zeta = j->pk[a].zeta;
            q.zeta_t = j->pkt[a].zeta;
            q.trs = j->pk[a].trs;
            q.trs_t = j->pkt[a].trs;
            q.trs_c = j->pc[a].trs;
            q.T = j->pk[a].T;
            q.ntiles = j->pk[a].ntiles;
            q.Tc = j->pc[a].T;
            q.ntiles_c = j->pc[a].ntiles;
            pt.push_back(q);
            z_n.push_back(q.R);
            z_n.push_back(q.C);
            t_n.push_back(std::max(q.ntiles, q.ntiles_c) + 1);
        }
    }
    const std::vector<int> fa = prefix_blocks(at_n), fz = prefix_blocks(z_n), ft = prefix_blocks(t_n);
    const ArrTask* d_at = upload_vec(al, at);
    const int* d_fa = upload_vec(al, fa);
    const PairTask* d_pt = upload_vec(al, pt);
    const int* d_fz = upload_vec(al, fz);
    const int* d_ft = upload_vec(al, ft);
    int* flags = al.dev<int>(nj);
    double* sums = al.dev<double>(2 * (size_t)nj);
    double* part = al.dev<double>(fa.back());
    int* hflags = al.host<int>(nj);
    double* hsums = al.host<double>(2 * (size_t)nj);
    HIPCHK(hipMemsetAsync(flags, 0, sizeof(int) * nj, s_));
    const int na = (int)at.size(), npt = (int)pt.size();
    hipLaunchKernelGGL(k_setup_arrays, dim3(fa.back()), dim3(kBlock), 0, s_, d_at, d_fa, na, flags, part);
    hipLaunchKernelGGL(k_setup_sums, dim3(blocks_for(na)), dim3(kBlock), 0, s_, d_at, d_fa, na, part, sums);
    hipLaunchKernelGGL(k_setup_zeta, dim3(fz.back()), dim3(kBlock), 0, s_, d_pt, d_fz, 2 * npt);
    hipLaunchKernelGGL(k_setup_tiles, dim3(ft.back()), dim3(kBlock), 0, s_, d_pt, d_ft, npt);
    HIPCHK(hipGetLastError());
    // 2D: the target masses and their logs row-major, as psi
    std::vector<ScaleTask> tr;
    std::vector<long long> tr_n;
    for (Job* j : jobs)
        if (j->d.dim == 2) {
            tr.push_back(ScaleTask{j->lv, j->lvr, j->p.nb, 1.0, j->d.n2, 1});
            tr.push_back(ScaleTask{j->d.v, j->vr, j->p.nb, 1.0, j->d.n2, 1});
            tr_n.push_back(j->p.nb);
            tr_n.push_back(j->p.nb);
        }
    if (!tr.empty()) {
        const std::vector<int> fr = prefix_blocks(tr_n);
        const ScaleTask* d_tr = upload_vec(al, tr);
        const int* d_fr = upload_vec(al, fr);
        hipLaunchKernelGGL(k_scale_tasks, dim3(fr.back()), dim3(kBlock), 0, s_, d_tr, d_fr, (int)tr.size());
        HIPCHK(hipGetLastError());
    }
    // 2D FP32 jobs on the extended-state loop: their state and masses
    for (Job* j : jobs) {
        j->ext2d = j->p.lx_shape >= 0;
        if (j->ext2d)
            ext2d_init(j->lx, j->d.x1, j->d.x2, j->d.y1, j->d.y2, j->lu, j->lvr, 1.0 / (j->d.eps * kLn2), s_);
    }
    // fast-sweep eligibility of the 1D jobs (the static range bound of every tile)
    std::vector<BoundTask> bt;
    std::vector<long long> bt_n;
    for (int i = 0; i < nj; ++i) {
        Job* j = jobs[i];
        if (!(j->d.dim == 1 && j->Bx && fast_allowed())) continue;
        const double kappa = 1.0 / (j->d.eps * kLn2);
        for (int dir = 0; dir < 2; ++dir) {
            // dir 0: K psi, columns y with masses v; dir 1: K^T phi, columns x with masses u
            const Part& pp = dir == 0 ? j->pk[0] : j->pkt[0];
            BoundTask b;
            memset(&b, 0, sizeof(b));
            b.yc = pp.yc;
            b.lmass = dir == 0 ? j->lv : j->lu;
            b.trs = pp.trs;
            b.R = pp.R;
            b.C = pp.C;
            b.kappa = kappa;
            b.T = pp.T;
            b.ntiles = pp.ntiles;
            b.flag = i;
            bt.push_back(b);
            bt_n.push_back(pp.ntiles);
        }
    }
    int* fflags = al.dev<int>(nj);
    int* hfflags = al.host<int>(nj);
    HIPCHK(hipMemsetAsync(fflags, 0, sizeof(int) * nj, s_));
    if (!bt.empty()) {
        std::vector<int> fb(bt.size() + 1, 0);
        for (size_t q = 0; q < bt.size(); ++q) fb[q + 1] = fb[q] + (int)bt_n[q];
        const BoundTask* d_bt = upload_vec(al, bt);
        const int* d_fb = upload_vec(al, fb);
        hipLaunchKernelGGL((k_tile_bounds<kBlock>), dim3(fb.back()), dim3(kBlock), 0, s_, d_bt, d_fb, (int)bt.size(),
                           fflags);
        HIPCHK(hipGetLastError());
    }
    al.uploaded();
    for (Job* j : jobs) j->status = FINOM_OK;
    HIPCHK(hipMemcpyAsync(hfflags, fflags, sizeof(int) * nj, hipMemcpyDeviceToHost, s_));
    if (checks) {
        HIPCHK(hipMemcpyAsync(hflags, flags, sizeof(int) * nj, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(hsums, sums, sizeof(double) * 2 * nj, hipMemcpyDeviceToHost, s_));
    }
    HIPCHK(hipStreamSynchronize(s_));
    // fast jobs: B = 2^{2 c kappa}, the masses as Ext<float> over the log
    // masses (the bound has read them), the state U = w 2^{-c kappa} over the
    // log potentials
    std::vector<FastStateTask> fst;
    for (int i = 0; i < nj; ++i) {
        Job* j = jobs[i];
        j->fast = j->d.dim == 1 && j->Bx && fast_allowed() && hfflags[i] == 0;
        j->gen = !j->fast && resident_ && j->d.dim == 1 && j->Bx && fast_allowed() &&
                 resident_fits(j->p.na, j->p.nb, j->pk[0].T, true);
        if (!j->fast && !j->gen) continue;
        const double kappa = 1.0 / (j->d.eps * kLn2);
        FastStateTask t;
        memset(&t, 0, sizeof(t));
        t.mode = 0;
        t.a = 0.0;
        t.b = 2.0 * kappa;
        t.out = j->Bx; t.in = j->d.x1; t.n = j->p.na; fst.push_back(t);
        t.out = j->By; t.in = j->d.x2; t.n = j->p.nb; fst.push_back(t);
        t.b = -kappa;
        t.out = j->F; t.in = j->d.x1; t.n = j->p.na; t.a = -log2((double)j->p.na); fst.push_back(t);
        t.out = j->G[0]; t.in = j->d.x2; t.n = j->p.nb; t.a = -log2((double)j->p.nb); fst.push_back(t);
        t.mode = 1;
        t.a = t.b = 0.0;
        t.out = j->lu; t.in = j->d.u; t.n = j->p.na; fst.push_back(t);
        t.out = j->lv; t.in = j->d.v; t.n = j->p.nb; fst.push_back(t);
    }
    if (!fst.empty()) {
        enqueue_fast_state(al, fst, s_);
        al.uploaded();
    }
    if (!checks) return;
    for (int i = 0; i < nj; ++i) {
        const int f = hflags[i];
        const double su = hsums[2 * i], sv = hsums[2 * i + 1];
        int st = FINOM_OK;
        if (f & 1) st = FINOM_E_UNSORTED;
        else if (f & 2) st = FINOM_E_MASS;
        else if (!(fabs(su - sv) <= 1e-12 * std::max(fabs(su), fabs(sv)))) st = FINOM_E_MASS;
        else if (f & 4) st = FINOM_E_ARG;
        jobs[i]->status = st;
    }
}

// ---------------------------------------------------------------------------
// resident batch
// ---------------------------------------------------------------------------
static const void* resident_batch_kernel(bool gen)
{
    return gen ? (const void*)k_resident_batch<kResidentBlockGen, kResidentIptGen, kResidentWavesGen, true>
               : (const void*)k_resident_batch<kResidentBlock, kResidentIpt, kResidentWaves, false>;
}

int resident_batch_capacity(bool gen)
{
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_batch_kernel(gen), resident_block(gen), 0) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

// Waits (one lane, at most max_ticks of the 100 MHz real-time counter) until
// a persistent grid's tile counter shows that `target` blocks have taken their
// first tile; the launches behind it on the stream then find those blocks
// resident. A bound, not a condition: the next launch is correct either way.
constexpr long long kStartWaitTicks = 5000000;   // 50 ms

__global__ void k_wait_started(const int* __restrict__ counter, int target, long long max_ticks)
{
    if (threadIdx.x != 0) return;
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
           (long long)__builtin_amdgcn_s_memrealtime() - t0 < max_ticks)
        __builtin_amdgcn_s_sleep(2);
}

void Engine::solve_resident()
{
    if (precision_ != 1 || !fast_allowed() || !resident_allowed()) return;
    std::vector<Job*> rj[2];
    for (int gen = 0; gen < 2; ++gen)
        for (Job* j : pending_init_)
            if (gen ? j->gen : (j->d.dim == 1 && j->fast && resident_fits(j->p.na, j->p.nb, j->pk[0].T, false)))
                rj[gen].push_back(j);
    if (rj[0].empty() || rj[1].empty()) {
        for (int gen = 0; gen < 2; ++gen)
            if (!rj[gen].empty()) run_resident_batch(rj[gen], gen != 0);
        return;
    }
    // Both variants at once: the extended grid (cooperative, on the engine's
    // stream) and the fast grid (an ordinary launch on the second stream,
    // which ROCm runs beside a cooperative one; cooperative launches run one
    // at a time). A fast block does not fit beside an extended one, so the
    // fast grid starts once every extended block has taken its first tile
    // (k_wait_started), and its blocks take the CUs the extended blocks leave.
    // No wait can deadlock: a grid stalls only while fewer of its blocks are
    // resident than its largest problem has tiles, both grids' largest
    // problems together need far fewer CUs than the GPU has, and a grid that
    // runs frees its CUs for the other (neither waits for the other's tiles).
    Alloc al(&ar_res_, s_);
    ResidentGrid g[2];
    for (int gen = 0; gen < 2; ++gen) prepare_resident(al, rj[gen], gen != 0, false, g[gen]);
    al.uploaded();
    HIPCHK(hipEventRecord(evu_, s_));
    HIPCHK(hipStreamWaitEvent(s2_, evu_, 0));
    launch_resident(g[1], s_, ev0_, ev1_, true);
    hipLaunchKernelGGL(k_wait_started, dim3(1), dim3(kWave), 0, s2_, (const int*)g[1].b.next, g[1].grid,
                       kStartWaitTicks);
    HIPCHK(hipGetLastError());
    launch_resident(g[0], s2_, ev2_, ev3_, false);
    HIPCHK(hipMemcpyAsync(g[0].hfail, g[0].flags, sizeof(int), hipMemcpyDeviceToHost, s2_));
    HIPCHK(hipMemcpyAsync(g[1].hfail, g[1].flags, sizeof(int), hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s2_));
    read_states();
    float ms[2] = {0.f, 0.f};
    HIPCHK(hipEventElapsedTime(&ms[0], ev2_, ev3_));
    HIPCHK(hipEventElapsedTime(&ms[1], ev0_, ev1_));
    for (int gen = 0; gen < 2; ++gen) finish_resident(g[gen], ms[gen]);
}

void Engine::prepare_resident(Alloc& al, const std::vector<Job*>& jobs, bool gen, bool resume, ResidentGrid& g)
{
    std::vector<Job*>& rj = g.jobs;
    rj = jobs;
    g.gen = gen;
    // larger problems first: the tiles are handed out in this order
    std::stable_sort(rj.begin(), rj.end(), [](const Job* a, const Job* b) { return a->pk[0].ntiles > b->pk[0].ntiles; });
    if (!resume) {
        std::vector<Job*> rest;
        for (Job* j : pending_init_)
            if (std::find(rj.begin(), rj.end(), j) == rj.end()) rest.push_back(j);
        pending_init_.swap(rest);
    }
    std::vector<StateInit> ini;
    std::vector<int> first(1, 0);
    for (Job* j : rj) {
        if (!resume) ini.push_back(StateInit{j->slot, 0, j->d.itr_max, j->d.tol});
        first.push_back(first.back() + j->pk[0].ntiles);
    }
    const int total = first.back();
    unsigned long long* rec = al.dev<unsigned long long>(5 * (size_t)total);
    g.flags = al.dev<int>(2);   // fail, tile counter
    g.hfail = al.host<int>(1);
    unsigned spin = kResidentSpin;
    if (const char* e = getenv("FINOM_RESIDENT_SPIN")) spin = (unsigned)strtoul(e, nullptr, 10);
    std::vector<ResidentArgs> args(rj.size());
    for (size_t i = 0; i < rj.size(); ++i) {
        const Job* j = rj[i];
        ResidentArgs& a = args[i];
        memset(&a, 0, sizeof(a));
        a.UF = (Ext<float>*)j->F;
        a.UG = (Ext<float>*)j->G[0];
        a.Ax = (const Ext<float>*)j->lu;
        a.Ay = (const Ext<float>*)j->lv;
        a.Bx = j->Bx;
        a.By = j->By;
        a.zx = j->pk[0].zeta;
        a.zy = j->pkt[0].zeta;
        a.trs = j->pk[0].trs;
        a.n = j->p.na;
        a.m = j->p.nb;
        a.ntiles = j->pk[0].ntiles;
        a.T = j->pk[0].T;
        a.rec = rec + 5 * (size_t)first[i];
        a.fail = g.flags;
        a.spin_limit = spin;
        a.ps = ps_ + j->slot;
    }
    const StateInit* d_ini = upload_vec(al, ini);
    g.b.probs = upload_vec(al, args);
    g.b.first = upload_vec(al, first);
    g.b.nprob = (int)rj.size();
    g.b.total = total;
    g.b.next = g.flags + 1;
    g.grid = std::min(total, resident_capacity(gen));
    if (!ini.empty())
        hipLaunchKernelGGL(k_init_states, dim3(blocks_for((long long)ini.size())), dim3(kBlock), 0, s_, d_ini,
                           (int)ini.size(), ps_);
    HIPCHK(hipGetLastError());
    // records start at zero (tag 0: written 0 times)
    HIPCHK(hipMemsetAsync(rec, 0, 5 * (size_t)total * sizeof(unsigned long long), s_));
    HIPCHK(hipMemsetAsync(g.flags, 0, 2 * sizeof(int), s_));
}

void Engine::launch_resident(ResidentGrid& g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, bool coop)
{
    void* kargs[] = {&g.b};
    HIPCHK(hipEventRecord(e0, s));
    if (coop)
        HIPCHK(hipLaunchCooperativeKernel(resident_batch_kernel(g.gen), dim3(g.grid), dim3(resident_block(g.gen)),
                                          kargs, 0, s));
    else
        HIPCHK(hipLaunchKernel(resident_batch_kernel(g.gen), dim3(g.grid), dim3(resident_block(g.gen)), kargs, 0, s));
    HIPCHK(hipEventRecord(e1, s));
}

void Engine::finish_resident(const ResidentGrid& g, float ms)
{
    loop_ms_total_ += ms;
    for (Job* j : g.jobs) {
        j->resident = true;
        j->started = true;
        j->loop_ms += ms;
    }
    if (*g.hfail) {
        set_last_error("resident solver: a grid wait exceeded its bound");
        throw StatusError{FINOM_E_HIP};
    }
}

void Engine::run_resident_batch(const std::vector<Job*>& jobs, bool gen, bool resume)
{
    Alloc al(&ar_res_, s_);
    ResidentGrid g;
    prepare_resident(al, jobs, gen, resume, g);
    al.uploaded();
    launch_resident(g, s_, ev0_, ev1_, true);
    HIPCHK(hipMemcpyAsync(g.hfail, g.flags, sizeof(int), hipMemcpyDeviceToHost, s_));
    read_states();
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
    finish_resident(g, ms);
}

bool Engine::add(Job* j)
{
    if (free_slots_.empty()) return false;
    j->slot = free_slots_.top();
    free_slots_.pop();
    max_slot_ = std::max(max_slot_, j->slot);
    j->loop_ms = 0.0;
    j->started = false;
    j->shift = 0;
    j->resumes = 0;
    j->last_resume_l = -1;
    j->resume_k = 0;
    j->err64 = 0.0;
    active_.push_back(j);
    pending_init_.push_back(j);
    dirty_ = true;
    return true;
}

long long Engine::live_tiles() const
{
    long long t = 0;
    for (const Job* j : active_) t += job_tiles(*j);
    return t;
}

void Engine::maybe_compact(double keep_fraction)
{
    if (dirty_) return;
    if ((double)live_tiles() < keep_fraction * (double)listed_tiles_) dirty_ = true;
}

namespace {
// stages of one iteration, in launch order
// 2D: K^T phi along x then y, K psi along y then x (psi row-major)
enum Stage { S1_KT = 0, S1_K = 1, S2_KTX = 2, S2_KTY = 3, S2_KY = 4, S2_KX = 5, NSTAGE = 6 };
constexpr int kStageEpi[NSTAGE] = {EPI_UPDATE_CHECK, EPI_UPDATE, EPI_STORE_LOG2, EPI_UPDATE_CHECK, EPI_STORE_LOG2,
                                   EPI_UPDATE};

struct LineRange {
    int group = -1;
    size_t first = 0, count = 0;
};
}  // namespace

void Engine::rebuild()
{
    drop_graph();
    HIPCHK(hipStreamSynchronize(s_));   // nothing in flight uses the old lists
    Alloc al(&ar_loop_, s_);
    const size_t eb = ext_bytes(precision_);

    // states of the jobs that joined since the last rebuild
    if (!pending_init_.empty()) {
        std::vector<StateInit> ini;
        for (Job* j : pending_init_) {
            ini.push_back(StateInit{j->slot, 0, j->d.itr_max, j->d.tol});
            j->started = true;
        }
        const StateInit* d_ini = upload_vec(al, ini);
        hipLaunchKernelGGL(k_init_states, dim3(blocks_for((long long)ini.size())), dim3(kBlock), 0, s_, d_ini,
                           (int)ini.size(), ps_);
        HIPCHK(hipGetLastError());
        // the extended-state loop's prologue (K_x^T phi of the initial phi)
        for (Job* j : pending_init_)
            if (j->ext2d) {
                ext2d_setup(j->lx, j->pk[0], j->pkt[0], j->pk[1], j->pkt[1], j->slot);
                ext2d_prologue(j->lx, ps_, s_);
            }
        pending_init_.clear();
    }

    sweeps_.clear();
    seq_[0].clear();
    seq_[1].clear();
    dec_[0].clear();
    dec_[1].clear();
    listed_ = active_;

    // Groups: one merged sweep per (stage, tile shape, split). 2D stages are
    // split by single- / multi-tile lines: multi-tile lines run the tile
    // aggregate kernel first, which then takes their stop decision, so one
    // launch must not mix the two kinds. 1D stages pass aggregates through
    // the update epilogue; their split separates fast-sweep lines from the
    // others.
    struct Group {
        int stage, cfg, split;
        Sweep* sw[2];
    };
    std::vector<Group> groups;
    std::map<std::tuple<int, int, int>, int> gidx;
    auto group = [&](int stage, int cfg, int split = 0) -> int {
        auto key = std::make_tuple(stage, cfg, split);
        auto it = gidx.find(key);
        if (it != gidx.end()) return it->second;
        Group g{stage, cfg, split, {nullptr, nullptr}};
        for (int b = 0; b < 2; ++b) {
            sweeps_.emplace_back(new Sweep());
            g.sw[b] = sweeps_.back().get();
            g.sw[b]->kind = 0;
            g.sw[b]->cfg = cfg;
            g.sw[b]->epi = kStageEpi[stage];
            g.sw[b]->fast = (stage == S1_KT || stage == S1_K) && split == 1;
        }
        groups.push_back(g);
        gidx[key] = (int)groups.size() - 1;
        return (int)groups.size() - 1;
    };

    std::vector<LineRange> chk(listed_.size()), dcd(listed_.size());
    std::vector<Job*> lx_listed;   // the jobs on the extended-state 2D loop
    for (size_t ji = 0; ji < listed_.size(); ++ji) {
        Job* j = listed_[ji];
        const JobDesc& d = j->d;
        const double eps = d.eps;
        if (j->ext2d) {
            // its own launches (ext2d_iteration), decision included
            ext2d_setup(j->lx, j->pk[0], j->pkt[0], j->pk[1], j->pkt[1], j->slot);
            lx_listed.push_back(j);
            chk[ji] = dcd[ji] = LineRange{-1, 0, 0};
            continue;
        }
        if (d.dim == 1) {
            const long long n = d.n1, m = d.n2;
            const int fs = j->fast ? 1 : 0;
            const int gt = group(S1_KT, j->p.cfg[0], fs), gk = group(S1_K, j->p.cfg[0], fs);
            const int T = kCfgs[j->p.cfg[0]].T();
            for (int b = 0; b < 2; ++b) {
                LineDesc a = make_line(d.x2, m, d.x1, n, j->pkt[0].zeta, j->pkt[0].trs, T, eps);
                a.gin = j->F;
                a.out = j->G[1 - b];
                a.a0 = j->lv;
                a.a1 = d.v;
                a.a2 = j->G[b];
                a.prob = j->slot;
                a.dec_part_off = -1;
                LineDesc c = make_line(d.x1, n, d.x2, m, j->pk[0].zeta, j->pk[0].trs, T, eps);
                c.gin = j->G[1 - b];
                c.out = j->F;
                c.a0 = j->lu;
                c.prob = j->slot;
                c.dec_part_off = -1;
                if (j->fast) {
                    a.er = j->By;
                    a.ec = j->Bx;
                    c.er = j->Bx;
                    c.ec = j->By;
                }
                if (b == 0) {
                    chk[ji] = LineRange{gt, groups[gt].sw[0]->lines.size(), 1};
                    dcd[ji] = LineRange{gk, groups[gk].sw[0]->lines.size(), 1};
                }
                groups[gt].sw[b]->lines.push_back(a);
                groups[gk].sw[b]->lines.push_back(c);
            }
        } else {
            const long long n1 = d.n1, m1 = d.m1, n2 = d.n2, m2 = d.m2;
            const int sx = j->p.ntiles[0] > 1 ? 1 : 0, sy = j->p.ntiles[1] > 1 ? 1 : 0;
            const int gtx = group(S2_KTX, j->p.cfg[0], sx), gty = group(S2_KTY, j->p.cfg[1], sy);
            const int gy = group(S2_KY, j->p.cfg[1], sy), gx = group(S2_KX, j->p.cfg[0], sx);
            chk[ji] = LineRange{gty, groups[gty].sw[0]->lines.size(), (size_t)n2};
            dcd[ji] = LineRange{gy, groups[gy].sw[0]->lines.size(), (size_t)n2};
            for (int b = 0; b < 2; ++b) {
                add_2d_kt_x_lines(*groups[gtx].sw[b], j->pkt[0], eps, j->F, n1, j->S, m1, j->slot);
                add_2d_kt_y_lines(*groups[gty].sw[b], j->pkt[1], eps, j->S, m1, j->G[1 - b], m2, j->lvr, j->vr,
                                  j->G[b], n2, j->slot);
                add_2d_k_y_lines(*groups[gy].sw[b], j->pk[1], eps, j->G[1 - b], m2, j->S, m1, n2, j->slot);
                add_2d_k_x_lines(*groups[gx].sw[b], j->pk[0], eps, j->S, n2, j->F, n1, j->lu, m1, j->slot);
            }
        }
    }

    // launch order: by stage, then tile shape
    std::vector<int> order(groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return std::make_tuple(groups[a].stage, groups[a].cfg, groups[a].split) <
               std::make_tuple(groups[b].stage, groups[b].cfg, groups[b].split);
    });

    // partial slots of the checking sweeps (same layout for both parities)
    int nparts = 0;
    for (int b = 0; b < 2; ++b) {
        int base = 0;
        for (int gi : order)
            if (groups[gi].stage == S1_KT || groups[gi].stage == S2_KTY) base += assign_parts(*groups[gi].sw[b], base);
        nparts = base;
    }
    // stop decisions: every line of a job's deciding stage reads the job's
    // partials; the first one records the state
    for (size_t ji = 0; ji < listed_.size(); ++ji) {
        if (chk[ji].group < 0) continue;
        for (int b = 0; b < 2; ++b) {
            const Sweep& cs = *groups[chk[ji].group].sw[b];
            const int off = cs.lines[chk[ji].first].part_base;
            int np = 0;
            for (size_t q = 0; q < chk[ji].count; ++q) np += cs.lines[chk[ji].first + q].ntiles;
            Sweep& ds = *groups[dcd[ji].group].sw[b];
            for (size_t q = 0; q < dcd[ji].count; ++q) {
                LineDesc& L = ds.lines[dcd[ji].first + q];
                L.dec_part_off = off;
                L.dec_nparts = np;
                L.writes_state = (q == 0) ? 1 : 0;
            }
        }
    }
    // 1D pairs of one tile shape pass tile aggregates to each other
    for (int gi : order) {
        Group& gt = groups[gi];
        if (gt.stage != S1_KT) continue;
        Group& gk = groups[gidx[std::make_tuple((int)S1_K, gt.cfg, gt.split)]];
        const int mt = gt.sw[0]->multi_tiles();
        if (mt == 0) continue;
        void* agg_kt = al.dev<char>((size_t)mt * 2 * eb);
        void* agg_k = al.dev<char>((size_t)mt * 2 * eb);
        for (int b = 0; b < 2; ++b) {
            gt.sw[b]->agg_from_prev = true;
            gt.sw[b]->agg_buf = agg_kt;
            gt.sw[b]->agg_next = agg_k;
            gk.sw[b]->agg_from_prev = true;
            gk.sw[b]->agg_buf = agg_k;
            gk.sw[b]->agg_next = agg_kt;
        }
    }
    listed_tiles_ = 0;
    for (int gi : order) {
        for (int b = 0; b < 2; ++b) upload_sweep(al, *groups[gi].sw[b], eb);
        listed_tiles_ += groups[gi].sw[0]->total_tiles();
    }
    partial_ = al.dev<double>(std::max(nparts, 1));
    // the extended-state 2D jobs: one launch per pass for all jobs of a line
    // shape and scan
    lx_groups_.clear();
    std::map<std::pair<int, int>, std::vector<Job*>> lx_by;
    for (Job* j : lx_listed) lx_by[std::make_pair(j->lx.shape, j->lx.s64)].push_back(j);
    for (const auto& kv : lx_by) {
        Ext2DGroup g;
        g.shape = kv.first.first;
        g.s64 = kv.first.second;
        g.nprob = (int)kv.second.size();
        std::vector<PairExt> pr[4];
        std::vector<int> fy(1, 0), fx(1, 0);
        for (const Job* j : kv.second) {
            for (int b = 0; b < 2; ++b) {
                pr[b].push_back(j->lx.y[b]);
                pr[2 + b].push_back(j->lx.x[b]);
            }
            fy.push_back(fy.back() + (int)j->lx.n2);
            fx.push_back(fx.back() + (int)j->lx.m1);
        }
        for (int b = 0; b < 2; ++b) {
            g.y[b] = upload_vec(al, pr[b]);
            g.x[b] = upload_vec(al, pr[2 + b]);
        }
        g.fy = upload_vec(al, fy);
        g.fx = upload_vec(al, fx);
        g.ny = fy.back();
        g.nx = fx.back();
        lx_groups_.push_back(g);
    }
    al.uploaded();
    // aggregates of the current phi for the first K^T phi of the next round
    for (int gi : order)
        if (groups[gi].stage == S1_KT && groups[gi].sw[0]->agg_from_prev)
            launch_aggregate(precision_, IN_LOG2, *groups[gi].sw[0], ps_, s_);
    for (int b = 0; b < 2; ++b)
        for (int gi : order) {
            seq_[b].push_back(groups[gi].sw[b]);
            dec_[b].push_back(groups[gi].stage == S1_K || groups[gi].stage == S2_KY);
        }
    dirty_ = false;
    stable_ = 0;
}

void Engine::launch_iterations(int k, hipStream_t s)
{
    for (int it = 0; it < k; ++it) {
        const int b = it & 1;
        for (size_t q = 0; q < seq_[b].size(); ++q)
            launch_sweep(precision_, IN_LOG2, *seq_[b][q], ps_, partial_, dec_[b][q] ? partial_ : nullptr, b, s);
        for (const Ext2DGroup& g : lx_groups_) ext2d_group_iteration(g, b, ps_, s);
    }
}

void Engine::round(int k)
{
    k += (k & 1);   // even, so every round starts on parity 0
    if (active_.empty()) return;
    if (dirty_) rebuild();
    if (use_graphs_ && stable_ >= 1 && (!exec_ || graph_k_ != k)) {
        drop_graph();
        HIPCHK(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
        try {
            launch_iterations(k, cs_);
        } catch (...) {
            hipGraph_t g2 = nullptr;
            hipStreamEndCapture(cs_, &g2);
            if (g2) hipGraphDestroy(g2);
            throw;
        }
        HIPCHK(hipStreamEndCapture(cs_, &graph_));
        HIPCHK(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
        graph_k_ = k;
    }
    HIPCHK(hipEventRecord(ev0_, s_));
    if (exec_ && graph_k_ == k) HIPCHK(hipGraphLaunch(exec_, s_));
    else launch_iterations(k, s_);
    HIPCHK(hipEventRecord(ev1_, s_));
    read_states();
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
    loop_ms_total_ += ms;
    for (Job* j : active_) j->loop_ms += ms;
    ++stable_;
}

void Engine::read_states()
{
    if (max_slot_ >= 0)
        HIPCHK(hipMemcpyAsync(hps_, ps_, sizeof(ProbState) * (max_slot_ + 1), hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s_));
}

void Engine::confirm_stops(std::vector<Job*>& fin)
{
    std::vector<Job*> todo;
    todo.swap(fin);
    while (!todo.empty()) {
        Alloc al(&ar_chk_, s_);
        const int dummy = cap_;
        // the returned pairs in FP64 log form (jobs on the fast state: phi, the
        // checked psi and log2 v, in place)
        std::vector<int> bo(todo.size());
        std::vector<FastStateTask> ft;
        for (size_t q = 0; q < todo.size(); ++q) {
            Job* j = todo[q];
            bo[q] = j->resident ? 0 : psi_slot(hps_[j->slot].iters, j->shift);
            if (j->ext2d)
                ext2d_to_log2(j->lx, bo[q], j->F, j->G[bo[q]], j->d.x1, j->d.x2, j->d.y1, j->d.y2,
                              1.0 / (j->d.eps * kLn2), s_);
            if (!j->fast && !j->gen) continue;
            const double kappa = 1.0 / (j->d.eps * kLn2);
            FastStateTask t;
            memset(&t, 0, sizeof(t));
            t.mode = 2;
            t.b = kappa;
            t.out = j->F; t.mesh = j->d.x1; t.n = j->p.na; ft.push_back(t);
            t.out = j->G[bo[q]]; t.mesh = j->d.x2; t.n = j->p.nb; ft.push_back(t);
            memset(&t, 0, sizeof(t));
            t.mode = 3;
            t.out = j->lv; t.in = j->d.v; t.n = j->p.nb; ft.push_back(t);
        }
        enqueue_fast_state(al, ft, s_);
        // K^T phi with FP64 scans and the check: 1D lines and 2D y-lines by
        // tile shape, after the 2D x-lines; each job's partials contiguous
        std::map<int, Sweep> x2d, chk1d, chk2d;
        std::vector<SegTask> segs;
        double* err_d = al.dev<double>(todo.size());
        int P = 0;
        for (size_t q = 0; q < todo.size(); ++q) {
            Job* j = todo[q];
            const JobDesc& d = j->d;
            const int b = bo[q];
            const int base = P;
            if (d.dim == 1) {
                Sweep& sw = chk1d[j->p.cfg[0]];
                LineDesc a = make_line(d.x2, d.n2, d.x1, d.n1, j->pkt[0].zeta, j->pkt[0].trs, j->pkt[0].T, d.eps);
                a.gin = j->F; a.out = j->G[1 - b]; a.a0 = j->lv; a.a1 = d.v; a.a2 = j->G[b];
                a.prob = dummy;
                a.dec_part_off = -1;
                a.part_base = P;
                P += a.ntiles;
                sw.lines.push_back(a);
            } else {
                add_2d_kt_x_lines(x2d[j->p.cfg[0]], j->pkt[0], d.eps, j->F, d.n1, j->S, d.m1, dummy);
                Sweep& sw = chk2d[j->p.cfg[1]];
                const size_t q0 = sw.lines.size();
                add_2d_kt_y_lines(sw, j->pkt[1], d.eps, j->S, d.m1, j->G[1 - b], d.m2, j->lvr, j->vr, j->G[b], d.n2,
                                  dummy);
                for (size_t k = q0; k < sw.lines.size(); ++k) {
                    sw.lines[k].part_base = P;
                    P += sw.lines[k].ntiles;
                }
            }
            segs.push_back(SegTask{base, P - base, err_d + q});
        }
        double* partial = al.dev<double>(std::max(P, 1));
        for (auto* m : {&x2d, &chk1d, &chk2d})
            for (auto& kv : *m) {
                kv.second.cfg = kv.first;
                kv.second.epi = (m == &x2d) ? EPI_STORE_LOG2 : EPI_UPDATE_CHECK;
                upload_sweep(al, kv.second, sizeof(Ext<double>));
            }
        const SegTask* d_segs = upload_vec(al, segs);
        double* err_h = al.host<double>(todo.size());
        al.uploaded();
        for (auto& kv : x2d) launch_sweep(0, IN_LOG2, kv.second, ps_, nullptr, nullptr, 0, s_);
        for (auto* m : {&chk1d, &chk2d})
            for (auto& kv : *m) launch_sweep(0, IN_LOG2, kv.second, ps_, partial, nullptr, 0, s_);
        hipLaunchKernelGGL(k_segment_sums, dim3((unsigned)segs.size()), dim3(kBlock), 0, s_, partial, d_segs);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(err_h, err_d, sizeof(double) * todo.size(), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));

        // confirmed stops, and the jobs that resume from the same pair (back
        // in their own representation)
        std::vector<Job*> again[2];   // resident, by variant
        ft.clear();
        for (size_t q = 0; q < todo.size(); ++q) {
            Job* j = todo[q];
            const ProbState& st = hps_[j->slot];
            j->err64 = err_h[q];
            const long long l = st.iters;
            if (!(j->err64 > j->d.tol) || l >= j->d.itr_max || !std::isfinite(j->err64) || st.status ||
                !may_resume(l, j->last_resume_l)) {
                fin.push_back(j);
                continue;
            }
            if (j->fast || j->gen) {
                const double kappa = 1.0 / (j->d.eps * kLn2);
                FastStateTask t;
                memset(&t, 0, sizeof(t));
                t.mode = 4;
                t.b = kappa;
                t.out = j->F; t.mesh = j->d.x1; t.n = j->p.na; ft.push_back(t);
                t.out = j->G[bo[q]]; t.mesh = j->d.x2; t.n = j->p.nb; ft.push_back(t);
                memset(&t, 0, sizeof(t));
                t.mode = 1;
                t.out = j->lv; t.in = j->d.v; t.n = j->p.nb; ft.push_back(t);
            }
            if (bo[q] == 1) {
                HIPCHK(hipMemcpyAsync(j->G[0], j->G[1], sizeof(double) * j->p.nb, hipMemcpyDeviceToDevice, s_));
                if (j->ext2d)
                    HIPCHK(hipMemcpyAsync(j->lx.UG[0], j->lx.UG[1], sizeof(Ext<float>) * j->p.nb,
                                          hipMemcpyDeviceToDevice, s_));
            }
            j->shift = (int)(l & 1);
            j->resume_k = resume_step(j->resume_k);
            enqueue_rearm(ps_ + j->slot, l, resume_until(l, j->resume_k, j->d.itr_max), s_);
            j->last_resume_l = l;
            ++j->resumes;
            if (j->resident) again[j->gen ? 1 : 0].push_back(j);
            // streaming jobs go on in the next rounds: their lines are still
            // listed, and the aggregates of their phi are those of the last
            // update, which no later sweep has touched
        }
        enqueue_fast_state(al, ft, s_);
        al.uploaded();
        todo.clear();
        for (int gen = 0; gen < 2; ++gen)
            if (!again[gen].empty()) {
                run_resident_batch(again[gen], gen != 0, true);
                todo.insert(todo.end(), again[gen].begin(), again[gen].end());
            }
    }
}

std::vector<Job*> Engine::harvest()
{
    std::vector<Job*> fin;
    for (Job* j : active_)
        if (j->started && hps_[j->slot].done) fin.push_back(j);
    if (fin.empty()) return fin;
    if (precision_ == 1) {
        confirm_stops(fin);
        if (fin.empty()) return fin;
    }

    Alloc al(&ar_cost_, s_);
    const int dummy = cap_;
    Sweep kc, cx_m, cy_p, cx_p, cy_m;
    kc.kind = 2;
    kc.epi = EPI_COST;
    cy_p.kind = 1;
    cy_p.epi = EPI_STORE_LOG2;
    cx_m.kind = 2;
    cx_m.epi = EPI_COST;
    cy_m.kind = 2;
    cy_m.epi = EPI_STORE_LOG2;
    cx_p.kind = 1;
    cx_p.epi = EPI_COST;
    std::vector<SegTask> segs;
    std::vector<ScaleTask> sc;
    std::vector<long long> sc_n;
    // the fast sweeps' state is in log form already: only FP32 jobs run on
    // it, and the FP64 check of their stop converted the returned pair
    int P = 0;
    for (Job* j : fin) {
        const JobDesc& d = j->d;
        const ProbState& st = hps_[j->slot];
        double* Gf = j->resident ? j->G[0] : j->G[psi_slot(st.iters, j->shift)];
        const double eps = d.eps;
        const int base = P;
        if (d.dim == 1) {
            LineDesc c = make_line(d.x1, d.n1, d.x2, d.n2, j->pc[0].zeta, j->pc[0].trs, j->pc[0].T, eps);
            c.gin = Gf;
            c.a0 = j->F;
            c.prob = dummy;
            c.dec_part_off = -1;
            c.part_base = P;
            P += c.ntiles;
            kc.lines.push_back(c);
        } else {
            // <C, Gamma> = sum Phi o (M_x Psi K_y^T) + sum Phi o (K_x Psi M_y^T), M = C o K,
            // each product along y first, as in the loop
            add_2d_k_y_lines(cy_p, j->pc[1], eps, Gf, d.m2, j->S, d.m1, d.n2, dummy);
            size_t q0 = cx_m.lines.size();
            add_2d_k_x_lines(cx_m, j->pc[0], eps, j->S, d.n2, nullptr, d.n1, j->F, d.m1, dummy);
            for (size_t q = q0; q < cx_m.lines.size(); ++q) {
                cx_m.lines[q].part_base = P;
                P += cx_m.lines[q].ntiles;
            }
            add_2d_k_y_lines(cy_m, j->pc[1], eps, Gf, d.m2, j->S, d.m1, d.n2, dummy);
            q0 = cx_p.lines.size();
            add_2d_k_x_lines(cx_p, j->pc[0], eps, j->S, d.n2, nullptr, d.n1, j->F, d.m1, dummy);
            for (size_t q = q0; q < cx_p.lines.size(); ++q) {
                cx_p.lines[q].part_base = P;
                P += cx_p.lines[q].ntiles;
            }
        }
        segs.push_back(SegTask{base, P - base, &ps_[j->slot].w1});
        if (d.f_out) {
            sc.push_back(ScaleTask{j->F, d.f_out, j->p.na, eps * kLn2, 0, 0});
            sc_n.push_back(j->p.na);
        }
        if (d.g_out) {
            sc.push_back(ScaleTask{Gf, d.g_out, j->p.nb, eps * kLn2, d.dim == 2 ? d.n2 : 0, d.dim == 2 ? 2 : 0});
            sc_n.push_back(j->p.nb);
        }
    }
    double* partial = al.dev<double>(std::max(P, 1));
    Sweep* order[5] = {&kc, &cy_p, &cx_m, &cy_m, &cx_p};
    for (Sweep* c : order)
        if (!c->lines.empty()) upload_sweep(al, *c, sizeof(Ext<double>));
    const SegTask* d_segs = upload_vec(al, segs);
    const std::vector<int> fs = prefix_blocks(sc_n);
    const ScaleTask* d_sc = upload_vec(al, sc);
    const int* d_fs = upload_vec(al, fs);
    al.uploaded();
    for (Sweep* c : order)
        if (!c->lines.empty()) launch_sweep(precision_, IN_LOG2, *c, ps_, partial, nullptr, 0, s_);
    hipLaunchKernelGGL(k_segment_sums, dim3((unsigned)segs.size()), dim3(kBlock), 0, s_, partial, d_segs);
    if (!sc.empty())
        hipLaunchKernelGGL(k_scale_tasks, dim3(fs.back()), dim3(kBlock), 0, s_, d_sc, d_fs, (int)sc.size());
    HIPCHK(hipGetLastError());
    read_states();

    for (Job* j : fin) {
        const ProbState& st = hps_[j->slot];
        finom_result& r = j->res;
        memset(&r, 0, sizeof(r));
        r.w1 = st.w1;
        r.marginal_err = st.err;
        r.iters = st.iters;
        r.converged = st.converged;
        int bad = st.status;
        if (precision_ == 1) {
            r.marginal_err = j->err64;
            r.converged = (j->err64 <= j->d.tol) ? 1 : 0;
            if (!std::isfinite(j->err64)) bad = 1;
        }
        r.sweeps = j->d.dim == 1 ? 2 * st.iters + 1 + j->resumes : 4 * st.iters + 2 + 2 * j->resumes;
        r.loop_ms = j->loop_ms;
        r.resumes = j->resumes;
        r.status = bad ? FINOM_E_NUMERIC : (r.converged ? FINOM_OK : FINOM_NOT_CONVERGED);
        r.fast = j->fast ? (j->resident ? 2 : 1) : (j->gen ? 3 : (j->ext2d ? 4 : 0));
        free_slots_.push(j->slot);
        j->slot = -1;
    }
    // The caller may free the finished jobs once this returns: no list keeps
    // them. Their lines in the uploaded sweeps and the extended-state launch
    // descriptors (device copies) stay until the next rebuild and return at
    // once (their slots are done, and a slot is reused only by add(), which
    // forces that rebuild).
    auto live = [](std::vector<Job*>& v) {
        std::vector<Job*> keep;
        for (Job* j : v)
            if (j->slot >= 0) keep.push_back(j);
        v.swap(keep);
    };
    live(active_);
    live(listed_);
    max_slot_ = -1;
    for (Job* j : active_) max_slot_ = std::max(max_slot_, j->slot);
    return fin;
}

// ---------------------------------------------------------------------------
// slab
// ---------------------------------------------------------------------------
Slab::Slab(size_t bytes) : cap_(align_up(std::max<size_t>(bytes, 256), 256))
{
    HIPCHK(hipMalloc((void**)&base_, cap_));
    free_.push_back({0, cap_});
}

Slab::~Slab()
{
    if (base_) hipFree(base_);
}

char* Slab::alloc(size_t bytes)
{
    bytes = align_up(std::max<size_t>(bytes, 1), 256);
    for (size_t i = 0; i < free_.size(); ++i) {
        if (free_[i].second < bytes) continue;
        const size_t off = free_[i].first;
        free_[i].first += bytes;
        free_[i].second -= bytes;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        used_ += bytes;
        return base_ + off;
    }
    return nullptr;
}

void Slab::release(char* p, size_t bytes)
{
    bytes = align_up(std::max<size_t>(bytes, 1), 256);
    const size_t off = (size_t)(p - base_);
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
    it = free_.insert(it, {off, bytes});
    used_ -= bytes;
    // merge with the neighbours
    size_t i = (size_t)(it - free_.begin());
    if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
        free_[i].second += free_[i + 1].second;
        free_.erase(free_.begin() + i + 1);
    }
    if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
        free_[i - 1].second += free_[i].second;
        free_.erase(free_.begin() + i);
    }
}

}  // namespace finom

using namespace finom;

extern "C" {

int64_t finom_footprint(const finom_problem* p, const finom_opts* opts)
{
    if (!p) return FINOM_E_ARG;
    const int precision = opts ? opts->precision : 0;
    const JobDesc d = job_from_problem(*p);
    const int st = check_job_args(d, precision);
    if (st != FINOM_OK) return st;
    return (int64_t)plan_job(d, precision).bytes;
}

int finom_batch(const finom_problem* probs, int64_t count, const finom_opts* opts, finom_result* res,
                void* stream)
{
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (count < 0 || count > (1 << 26) || (count > 0 && (!probs || !res))) return FINOM_E_ARG;
    if (o.precision != 0 && o.precision != 1) return FINOM_E_ARG;
    if (count == 0) return FINOM_OK;
    for (int64_t i = 0; i < count; ++i) memset(res + i, 0, sizeof(finom_result));
    std::vector<Job> jobs((size_t)count);
    std::vector<Job*> valid;
    int first_err = FINOM_OK;
    size_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        Job& j = jobs[(size_t)i];
        j.d = job_from_problem(probs[i]);
        j.tag = i;
        const int st = check_job_args(j.d, o.precision);
        if (st != FINOM_OK) {
            res[i].status = st;
            if (first_err == FINOM_OK) first_err = st;
            continue;
        }
        j.p = plan_job(j.d, o.precision);
        total += j.p.bytes;
        valid.push_back(&j);
    }
    if (valid.empty()) return first_err;
    try {
        hipStream_t s = (hipStream_t)stream;
        Alloc al(stream);
        char* mem = al.dev<char>(total);
        size_t off = 0;
        for (Job* j : valid) {
            j->mem = mem + off;
            off += j->p.bytes;
            j->bind();
        }
        Engine eng(o.precision, s, (int)valid.size(), true);
        eng.enable_resident();
        eng.setup(valid, !o.skip_checks);
        for (Job* j : valid) {
            if (j->status != FINOM_OK) {
                res[j->tag].status = j->status;
                if (first_err == FINOM_OK) first_err = j->status;
                continue;
            }
            eng.add(j);
        }
        const int k = o.graph_iters > 0 ? o.graph_iters : 16;
        bool any_nc = false;
        eng.solve_resident();
        bool first = true;
        while (eng.live() > 0) {
            if (!first) eng.round(k);
            first = false;
            for (Job* j : eng.harvest()) {
                res[j->tag] = j->res;
                if (j->res.status < 0 && first_err == FINOM_OK) first_err = j->res.status;
                if (j->res.status == FINOM_NOT_CONVERGED) any_nc = true;
            }
            eng.maybe_compact(0.5);
        }
        if (first_err != FINOM_OK) return first_err;
        return any_nc ? FINOM_NOT_CONVERGED : FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

}  // extern "C"
