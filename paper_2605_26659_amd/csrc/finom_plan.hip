// Dense transport plans from potentials, and the Frobenius norm of the
// difference of two plans: Gamma = diag(phi) K diag(psi) of section 2.1, the
// matrices whose difference section 4's tables report. This runs once after
// a solve and is off the iteration's path.
//
// Entry (r, c), r a source point and c a target point:
//   Gamma_rc = exp((f_r + g_c - C_rc) / eps)
// with f = eps ln phi and g = eps ln psi. C_rc = |x_r - y_c| in 1D. On tensor
// meshes C_rc = |x1_k - x2_l| + |y1_i - y2_j| with r = k + i n1 and
// c = l + j n2, the column-major grid order of the potentials (eq. 2d-kron).
// The argument is formed in the order ((f + g) - C) / eps, with C summed as
// x part + y part, and the exponential is the device library's FP64 one.
//
// Every entry is independent, so both kernels are a plain map over
// (row group, column chunk) items: an item is kPlanRows consecutive rows and
// kPlanBlock * kPlanIpt consecutive columns. Thread t takes the columns
// t + q kPlanBlock, loads their potentials and coordinates once into
// registers and reuses them for every row of the group; the row values are
// the same for the whole block. Each store of a wave covers 64 consecutive
// doubles of a row. Export writes n*m doubles and reads O(n + m): it is bound
// by HBM writes, 8 B per entry. The difference writes nothing and evaluates
// two exponentials per entry: it is bound by FP64 arithmetic. Its sum of
// squares is reduced per block in a fixed order over a fixed grid, then the
// block partials by one block in a fixed order, so the result is the same on
// every run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/finom.h"
#include "finom_host.hpp"

namespace finom {

constexpr int kPlanBlock = 256, kPlanIpt = 8, kPlanRows = 8;
constexpr int kPlanChunk = kPlanBlock * kPlanIpt;
constexpr int kPlanDiffGrid = 2048;      // blocks of the difference kernel
constexpr long long kPlanMaxGrid = 1LL << 30;

struct PlanArgs {
    const double* xs;   // source first axis (x in 1D, x1 on tensor meshes)
    const double* ys;   // source second axis (tensor meshes)
    const double* xt;   // target first axis (y in 1D, x2)
    const double* yt;   // target second axis (y2)
    const double* fa;   // potentials of the plan (a)
    const double* ga;
    const double* fb;   // potentials of the plan (b) of a difference
    const double* gb;
    long long ns1;      // source first-axis length (rows r = k + i ns1)
    long long nt1;      // target first-axis length (columns c = l + j nt1)
    long long rows, cols, ld, chunks, items;
    double rinv_t1;     // 1 / nt1, for the first column split of a thread
    int dl, dj;         // kPlanBlock = dj nt1 + dl: a thread's step in (l, j)
    double eps;
    double* gamma;      // export: rows x ld, row-major
    double* part;       // difference: one partial sum of squares per block
};

// Column data of one thread for one chunk: for each of its columns the
// target coordinates and the potential(s). Columns past the end get cost 0
// and potential 0 and are never stored or summed.
template <bool TD, bool DIFF>
struct PlanCols {
    double cx[kPlanIpt], cy[kPlanIpt], ga[kPlanIpt], gb[kPlanIpt];
};

template <bool TD, bool DIFF>
__device__ __forceinline__ void plan_load_cols(const PlanArgs& a, long long c0, PlanCols<TD, DIFF>& cc)
{
    long long l = c0, j = 0;
    if (TD) {
        // first split by a rounded reciprocal, corrected by one step
        j = (long long)((double)c0 * a.rinv_t1);
        l = c0 - j * a.nt1;
        if (l < 0) {
            --j;
            l += a.nt1;
        } else if (l >= a.nt1) {
            ++j;
            l -= a.nt1;
        }
    }
#pragma unroll
    for (int q = 0; q < kPlanIpt; ++q) {
        const long long c = c0 + (long long)q * kPlanBlock;
        const bool in = c < a.cols;
        cc.cx[q] = in ? a.xt[l] : 0.0;
        cc.cy[q] = (TD && in) ? a.yt[j] : 0.0;
        cc.ga[q] = in ? a.ga[c] : 0.0;
        cc.gb[q] = (DIFF && in) ? a.gb[c] : 0.0;
        if (TD) {
            l += a.dl;
            j += a.dj;
            if (l >= a.nt1) {
                l -= a.nt1;
                ++j;
            }
        } else {
            l += kPlanBlock;
        }
    }
}

// Grid indices of the rows of a group: row r = k + i ns1. The first row is
// split once per item; the next rows step k with a wrap into i.
struct PlanRowIdx {
    long long k, i;
};

template <bool TD>
__device__ __forceinline__ PlanRowIdx plan_row_first(const PlanArgs& a, long long r0)
{
    if (!TD) return PlanRowIdx{r0, 0};
    const long long i = r0 / a.ns1;
    return PlanRowIdx{r0 - i * a.ns1, i};
}

template <bool TD>
__device__ __forceinline__ void plan_row_next(const PlanArgs& a, PlanRowIdx& ri)
{
    ++ri.k;
    if (TD && ri.k == a.ns1) {
        ri.k = 0;
        ++ri.i;
    }
}

// Source coordinates of a row (the same for the whole block).
template <bool TD>
__device__ __forceinline__ void plan_row(const PlanArgs& a, const PlanRowIdx& ri, double& xr, double& yr)
{
    xr = a.xs[ri.k];
    yr = TD ? a.ys[ri.i] : 0.0;
}

template <bool TD>
__device__ __forceinline__ double plan_cost(double xr, double yr, double cx, double cy)
{
    if (TD) return fabs(xr - cx) + fabs(yr - cy);
    return fabs(xr - cx);
}

template <bool TD>
__global__ __launch_bounds__(kPlanBlock) void k_plan_export(PlanArgs a)
{
    for (long long it = blockIdx.x; it < a.items; it += gridDim.x) {
        const long long rg = it / a.chunks;
        const long long c0 = (it - rg * a.chunks) * kPlanChunk + threadIdx.x;
        PlanCols<TD, false> cc;
        plan_load_cols<TD, false>(a, c0, cc);
        const long long r0 = rg * kPlanRows;
        const int nr = (int)min((long long)kPlanRows, a.rows - r0);
        PlanRowIdx ri = plan_row_first<TD>(a, r0);
        for (int rr = 0; rr < nr; ++rr, plan_row_next<TD>(a, ri)) {
            const long long r = r0 + rr;
            double xr, yr;
            plan_row<TD>(a, ri, xr, yr);
            const double fr = a.fa[r];
            double* out = a.gamma + r * a.ld;
#pragma unroll
            for (int q = 0; q < kPlanIpt; ++q) {
                const long long c = c0 + (long long)q * kPlanBlock;
                if (c < a.cols) {
                    const double arg = ((fr + cc.ga[q]) - plan_cost<TD>(xr, yr, cc.cx[q], cc.cy[q])) / a.eps;
                    __builtin_nontemporal_store(exp(arg), out + c);
                }
            }
        }
    }
}

__device__ __forceinline__ double plan_block_sum(double v, double* s_w)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kPlanBlock / 64; ++k) t += s_w[k];
    return t;
}

template <bool TD>
__global__ __launch_bounds__(kPlanBlock) void k_plan_diff(PlanArgs a)
{
    __shared__ double s_w[kPlanBlock / 64];
    double acc = 0.0;
    for (long long it = blockIdx.x; it < a.items; it += gridDim.x) {
        const long long rg = it / a.chunks;
        const long long c0 = (it - rg * a.chunks) * kPlanChunk + threadIdx.x;
        PlanCols<TD, true> cc;
        plan_load_cols<TD, true>(a, c0, cc);
        const long long r0 = rg * kPlanRows;
        const int nr = (int)min((long long)kPlanRows, a.rows - r0);
        PlanRowIdx ri = plan_row_first<TD>(a, r0);
        for (int rr = 0; rr < nr; ++rr, plan_row_next<TD>(a, ri)) {
            const long long r = r0 + rr;
            double xr, yr;
            plan_row<TD>(a, ri, xr, yr);
            const double fra = a.fa[r], frb = a.fb[r];
#pragma unroll
            for (int q = 0; q < kPlanIpt; ++q) {
                const long long c = c0 + (long long)q * kPlanBlock;
                if (c < a.cols) {
                    const double C = plan_cost<TD>(xr, yr, cc.cx[q], cc.cy[q]);
                    const double d = exp(((fra + cc.ga[q]) - C) / a.eps) - exp(((frb + cc.gb[q]) - C) / a.eps);
                    acc = fma(d, d, acc);
                }
            }
        }
    }
    const double t = plan_block_sum(acc, s_w);
    if (threadIdx.x == 0) a.part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kPlanBlock) void k_plan_diff_final(const double* __restrict__ part, int nb,
                                                                double* __restrict__ out)
{
    __shared__ double s_w[kPlanBlock / 64];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kPlanBlock) v += part[b];
    const double t = plan_block_sum(v, s_w);
    if (threadIdx.x == 0) *out = sqrt(t);
}

// Validates the sizes and fills the shape fields; the caller sets the
// pointers. Throws StatusError(FINOM_E_ARG) on a bad argument.
static void plan_shape(PlanArgs& a, long long ns1, long long ms1, long long nt1, long long mt1, double eps,
                       long long ld, bool need_ld)
{
    auto bad = [](const char* msg) {
        set_last_error(msg);
        throw StatusError{FINOM_E_ARG};
    };
    if (ns1 < 1 || ms1 < 1 || nt1 < 1 || mt1 < 1) bad("plan: every axis needs at least one point");
    if (!(eps > 0.0) || !std::isfinite(eps)) bad("plan: eps must be positive and finite");
    if (ns1 > INT64_MAX / ms1 || nt1 > INT64_MAX / mt1) bad("plan: grid size overflows");
    a.ns1 = ns1;
    a.nt1 = nt1;
    a.rows = ns1 * ms1;
    a.cols = nt1 * mt1;
    if (need_ld) {
        if (ld < a.cols) bad("plan: ld is smaller than the number of target points");
        if (a.rows > INT64_MAX / ld) bad("plan: rows * ld overflows");
    }
    a.ld = ld;
    a.chunks = (a.cols + kPlanChunk - 1) / kPlanChunk;
    const long long groups = (a.rows + kPlanRows - 1) / kPlanRows;
    if (groups > INT64_MAX / a.chunks) bad("plan: too many items");
    a.items = groups * a.chunks;
    a.rinv_t1 = 1.0 / (double)nt1;
    a.dl = (int)(kPlanBlock % nt1);
    a.dj = (int)(kPlanBlock / nt1);
    a.eps = eps;
}

static int plan_export(bool td, const double* xs, long long ns1, const double* ys, long long ms1,
                       const double* xt, long long nt1, const double* yt, long long mt1, const double* f,
                       const double* g, double eps, double* gamma, long long ld, void* stream)
{
    try {
        if (!xs || !xt || !f || !g || !gamma || (td && (!ys || !yt))) {
            set_last_error("plan: a required pointer is NULL");
            return FINOM_E_ARG;
        }
        PlanArgs a{};
        plan_shape(a, ns1, ms1, nt1, mt1, eps, ld, true);
        a.xs = xs;
        a.ys = ys;
        a.xt = xt;
        a.yt = yt;
        a.fa = f;
        a.ga = g;
        a.gamma = gamma;
        const long long grid = std::min(a.items, kPlanMaxGrid);
        hipStream_t s = (hipStream_t)stream;
        if (td) hipLaunchKernelGGL(k_plan_export<true>, dim3((unsigned)grid), dim3(kPlanBlock), 0, s, a);
        else hipLaunchKernelGGL(k_plan_export<false>, dim3((unsigned)grid), dim3(kPlanBlock), 0, s, a);
        HIPCHK(hipGetLastError());
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

static int plan_diff(bool td, const double* xs, long long ns1, const double* ys, long long ms1, const double* xt,
                     long long nt1, const double* yt, long long mt1, const double* fa, const double* ga,
                     const double* fb, const double* gb, double eps, double* out, void* stream)
{
    try {
        if (!xs || !xt || !fa || !ga || !fb || !gb || !out || (td && (!ys || !yt))) {
            set_last_error("plan difference: a required pointer is NULL");
            return FINOM_E_ARG;
        }
        PlanArgs a{};
        plan_shape(a, ns1, ms1, nt1, mt1, eps, 0, false);
        a.xs = xs;
        a.ys = ys;
        a.xt = xt;
        a.yt = yt;
        a.fa = fa;
        a.ga = ga;
        a.fb = fb;
        a.gb = gb;
        Alloc al(stream);
        const int grid = (int)std::min<long long>(a.items, kPlanDiffGrid);
        a.part = al.dev<double>(grid);
        hipStream_t s = (hipStream_t)stream;
        if (td) hipLaunchKernelGGL(k_plan_diff<true>, dim3(grid), dim3(kPlanBlock), 0, s, a);
        else hipLaunchKernelGGL(k_plan_diff<false>, dim3(grid), dim3(kPlanBlock), 0, s, a);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_plan_diff_final, dim3(1), dim3(kPlanBlock), 0, s, (const double*)a.part, grid, out);
        HIPCHK(hipGetLastError());
        al.uploaded();
        return FINOM_OK;
    } catch (...) {
        return map_exception();
    }
}

}  // namespace finom

using namespace finom;

extern "C" {

int finom_plan_1d(const double* x, int64_t n, const double* y, int64_t m, const double* f, const double* g,
                  double eps, double* gamma, int64_t ld, void* stream)
{
    return plan_export(false, x, n, nullptr, 1, y, m, nullptr, 1, f, g, eps, gamma, ld, stream);
}

int finom_plan_2d(const double* x1, int64_t n1, const double* y1, int64_t m1, const double* x2, int64_t n2,
                  const double* y2, int64_t m2, const double* f, const double* g, double eps, double* gamma,
                  int64_t ld, void* stream)
{
    return plan_export(true, x1, n1, y1, m1, x2, n2, y2, m2, f, g, eps, gamma, ld, stream);
}

int finom_plan_diff_1d(const double* x, int64_t n, const double* y, int64_t m, const double* fa,
                       const double* ga, const double* fb, const double* gb, double eps, double* out,
                       void* stream)
{
    return plan_diff(false, x, n, nullptr, 1, y, m, nullptr, 1, fa, ga, fb, gb, eps, out, stream);
}

int finom_plan_diff_2d(const double* x1, int64_t n1, const double* y1, int64_t m1, const double* x2,
                       int64_t n2, const double* y2, int64_t m2, const double* fa, const double* ga,
                       const double* fb, const double* gb, double eps, double* out, void* stream)
{
    return plan_diff(true, x1, n1, y1, m1, x2, n2, y2, m2, fa, ga, fb, gb, eps, out, stream);
}

}  // extern "C"
