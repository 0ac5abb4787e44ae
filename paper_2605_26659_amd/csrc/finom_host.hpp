// Host-side helpers: error mapping, the per-stream workspace arena, sweep
// descriptors and their upload, kernel dispatch.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/finom.h"
#include "finom_fast.hpp"
#include "finom_kernels.hpp"
#include "finom_line_ext.hpp"

namespace finom {

constexpr int kBlock = 256;     // block size of the setup / utility kernels
constexpr double kLn2 = 0.69314718055994530942;

// Scan tile shapes: threads per block x elements per thread. T = block * ipt
// merged elements per tile. The FP32 fast sweeps run every shape; the general
// sweeps run a shape as the shape `general` of the same T (they are not
// instantiated for 512 x 4). The cost sweeps (FP64 moment sums, four LDS
// arrays) always use kCostBlock x kCostIpt.
struct TileCfg {
    int block, ipt;
    int general;
    int T() const { return block * ipt; }
};
// The first kNumTunedCfg shapes are the tuner's (and FINOM_TILE_CFG's);
// kShortCfg, one wave per block, only takes general-sweep lines that fit one
// of its tiles whole (short_line_cfg).
constexpr int kNumTunedCfg = 5;
constexpr int kShortCfg = 5;
constexpr int kNumCfg = 6;
constexpr TileCfg kCfgs[kNumCfg] = {{256, 4, 0}, {256, 8, 1}, {512, 8, 2}, {128, 4, 3}, {512, 4, 1}, {64, 4, 5}};
constexpr int kCostBlock = 256, kCostIpt = 2;

struct HipError {
    hipError_t e;
};

// A failure with its own status and message (the message is already in the
// library's last-error text, set with set_last_error).
struct StatusError {
    int status;
};

void set_last_error(const char* msg);

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t _e = (x);                       \
        if (_e != hipSuccess) throw HipError{_e};  \
    } while (0)

inline unsigned blocks_for(long long n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }
inline int ntiles_for(long long R, long long C, int T) { return (int)((R + C + T - 1) / T); }
inline int cost_tile_size() { return kCostBlock * kCostIpt; }
inline size_t ext_bytes(int precision) { return precision == 1 ? sizeof(Ext<float>) : sizeof(Ext<double>); }

// Default tile shape for a 1D line of `merged` elements; the autotuner can
// override it per size class (class c holds lengths up to 2^(9 + c), the
// last class everything longer).
int default_cfg(int precision, long long merged);
int tuned_cfg(int precision, long long merged);
// Shape of the lines of a 2D or d-dimensional problem's general sweeps: a
// line of at most 256 merged points runs as one tile of the one-wave shape
// (no cross-wave steps), others take tuned_cfg. FINOM_TILE_CFG overrides both.
int short_line_cfg(int precision, long long merged);
constexpr int kTuneClasses = 13;
int tune_class(long long merged);
void set_tuned_cfg(int precision, int cls, int cfg);
int get_tuned_cfg(int precision, int cls);   // -1 when not tuned

// ---------------------------------------------------------------------------
// Workspace: per stream, a list of device blocks and pinned host blocks.
// A call carves what it needs with a bump pointer through the blocks in
// order, moving to the next block when one is full; when the last one
// overflows, another block is added. The next call on the stream starts again
// at the first block, so a call that fits the blocks the earlier calls grew
// allocates nothing, and no block is freed before the workspace is released.
// Device memory is reused in stream order; the pinned host blocks only after
// the previous call's uploads have completed (upload_done).
// ---------------------------------------------------------------------------
struct Block {
    char* p;
    size_t cap;
};

struct Arena {
    std::vector<Block> dblk, hblk;
    size_t dcur = 0, hcur = 0;     // block the next carve tries first
    size_t dused = 0, hused = 0;   // bytes used in that block
    hipEvent_t upload_done = nullptr;
};

Arena* arena_for(void* stream);
void arena_release_all();
// Frees the blocks and the event of an arena that is not in the per-stream map.
void arena_free(Arena* a);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Alloc {
    Arena* a;
    hipStream_t s;
    explicit Alloc(void* stream) : a(arena_for(stream)), s((hipStream_t)stream) { begin(); }
    Alloc(Arena* arena, hipStream_t stream) : a(arena), s(stream) { begin(); }

    void begin()
    {
        if (a->upload_done) HIPCHK(hipEventSynchronize(a->upload_done));
        else HIPCHK(hipEventCreateWithFlags(&a->upload_done, hipEventDisableTiming));
        a->dcur = a->hcur = 0;
        a->dused = 0;
        a->hused = 0;
    }
    // Block bases are at least 256-byte aligned (hipMalloc, hipHostMalloc),
    // so offsets aligned within a block are aligned addresses.
    static char* carve(std::vector<Block>& v, size_t& cur, size_t& used, size_t bytes, size_t align, bool host)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), align);
        while (cur < v.size()) {
            const size_t off = align_up(used, align);
            if (off <= v[cur].cap && bytes <= v[cur].cap - off) {
                used = off + bytes;
                return v[cur].p + off;
            }
            ++cur;
            used = 0;
        }
        const size_t cap = std::max(bytes, v.empty() ? (size_t)(host ? (1u << 20) : (16u << 20)) : v.back().cap);
        Block b{nullptr, cap};
        if (host) {
            if (hipHostMalloc((void**)&b.p, cap, hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
        } else {
            if (hipMalloc((void**)&b.p, cap) != hipSuccess) throw std::bad_alloc();
        }
        v.push_back(b);
        cur = v.size() - 1;
        used = bytes;
        return b.p;
    }
    template <typename T>
    T* dev(size_t count)
    {
        return reinterpret_cast<T*>(carve(a->dblk, a->dcur, a->dused, sizeof(T) * count, 256, false));
    }
    template <typename T>
    T* host(size_t count)
    {
        return reinterpret_cast<T*>(carve(a->hblk, a->hcur, a->hused, sizeof(T) * count, 64, true));
    }
    void uploaded() { HIPCHK(hipEventRecord(a->upload_done, s)); }
};

// ---------------------------------------------------------------------------
// Sweeps
// ---------------------------------------------------------------------------
struct SweepDev {
    const WorkItem* work = nullptr;        // all tiles
    int nwork = 0;
    int max_tiles = 0;                     // largest tile count of a line (fast sweeps: of the uncarried)
    int max_dec = 0;                       // largest number of decision partials of a line (idem)
    const int* big = nullptr;              // fast sweeps: lines whose carries k_fast_carries forms
    int nbig = 0;
    void* carries = nullptr;               // their carries, laid out as agg
    const WorkItem* work_multi = nullptr;  // tiles of lines with more than one tile
    int nwork_multi = 0;
    const LineDesc* lines = nullptr;
    void* agg = nullptr;                   // tile aggregates this sweep reads
};

// kind: 0 = scan in the call's precision (plain sums), 1 = FP64 cost tile
// (plain sums), 2 = FP64 cost tile with moment sums.
// agg_from_prev: the tile aggregates are written by the previous sweep's
// epilogue (shared partition), so no aggregate kernel runs.
// agg_next: where this sweep's epilogue writes the next sweep's aggregates.
struct Sweep {
    std::vector<LineDesc> lines;
    int kind = 0;
    int cfg = 1;
    int epi = EPI_STORE_LOG2;
    bool agg_from_prev = false;
    bool fast = false;                     // FP32 fast sweeps (lines carry er / ec)
    void* agg_next = nullptr;
    void* agg_buf = nullptr;               // preassigned aggregate buffer (optional)
    SweepDev dev;
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
    int ns() const { return kind == 2 ? 4 : 2; }
    int T() const { return kind == 0 ? kCfgs[cfg].T() : cost_tile_size(); }
};

inline LineDesc make_line(const double* xr, long long R, const double* yc, long long C,
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
    L.ntiles = ntiles_for(R, C, T);
    return L;
}

// Assigns agg slots and per-problem partial slots (tiles of problem p in this
// sweep, in line order), fills work lists and uploads from pinned memory.
void upload_sweep(Alloc& al, Sweep& sw, size_t ext_b);

void launch_sweep(int precision, int inm, const Sweep& sw, ProbState* ps, double* partial,
                  const double* dec, int parity, hipStream_t s);
// Only the tile-aggregate kernel of a sweep (initial aggregates).
void launch_aggregate(int precision, int inm, const Sweep& sw, ProbState* ps, hipStream_t s);

// ---------------------------------------------------------------------------
// Mesh-pair partition: dividing index + merge-path tile rows at tile size T
// ---------------------------------------------------------------------------
struct Part {
    const double* xr = nullptr;
    long long R = 0;
    const double* yc = nullptr;
    long long C = 0;
    int* zeta = nullptr;
    int* trs = nullptr;
    int T = 0;
    int ntiles = 0;
};

// A partition whose arrays are already allocated (filled by the batched
// setup kernels).
inline Part part_view(const double* xr, long long R, const double* yc, long long C, int* zeta, int* trs,
                      int T)
{
    Part p;
    p.xr = xr;
    p.R = R;
    p.yc = yc;
    p.C = C;
    p.zeta = zeta;
    p.trs = trs;
    p.T = T;
    p.ntiles = ntiles_for(R, C, T);
    return p;
}

Part make_part(Alloc& al, const double* xr, long long R, const double* yc, long long C, int T,
               hipStream_t s);
// The same into caller-provided arrays: zeta (R ints) and the tile row starts
// trs (ntiles_for(R, C, T) + 1 ints). Allocates nothing.
void enqueue_partition(const double* xr, long long R, const double* yc, long long C, int T, int* zeta,
                       int* trs, hipStream_t s);
// Reuses an existing dividing index with another tile size.
Part make_part_like(Alloc& al, const Part& base, int T, hipStream_t s);
// The transposed pair (rows yc, columns xr) on the SAME merged-sequence tiles
// as `base`: its tile t holds base's columns of tile t as rows.
Part make_part_transposed(Alloc& al, const Part& base, hipStream_t s);

// ---------------------------------------------------------------------------
// Validation and mass preparation
// ---------------------------------------------------------------------------
void enqueue_sorted_check(const double* a, long long n, int* dflag, hipStream_t s);
void enqueue_log2_mass(const double* a, long long n, double* la, int* dflag, hipStream_t s);
void enqueue_sum(Alloc& al, const double* a, long long n, double* dsum, hipStream_t s);
void enqueue_fill(double* a, long long n, double v, hipStream_t s);
void enqueue_scale(const double* a, double* b, long long n, double f, hipStream_t s);

int map_exception();

// Fast sweeps are used for eligible FP32 lines unless FINOM_FAST=0.
bool fast_allowed();
// The resident solver is used for eligible 1D FP32 problems unless
// FINOM_RESIDENT=0.
bool resident_allowed();
// Blocks of the resident kernels (single problem and batch; gen: the variant
// with extended-number scans) that can be resident at once on the current
// device; 0 when it cannot launch them cooperatively.
// resident_batch_capacity is the batch kernel's alone.
int resident_capacity(bool gen);
int resident_batch_capacity(bool gen);
// Whether a 1D problem of n + m points on tiles of T runs on the resident
// solver, alone or in a batch: the fast variant once its tiles pass the fast
// sweeps' bound, the gen variant otherwise.
bool resident_fits(long long n, long long m, int T, bool gen);
// Classifies the 1D pair (x: n, y: m) on partition pk (rows x) and its
// transpose pkt for the fast sweeps; fills 2^{c kappa} for both meshes when
// eligible. Synchronises the stream. Returns true when the pair is eligible.
// Conversions for the fast sweeps' state, one thread per element:
//   mode 0: out = 2^{a + b in_k} as Ext<float> (B = 2^{2 c kappa}, the initial state);
//   mode 1: out = in_k as Ext<float> (masses);
//   mode 2: out = log2(state_k) + b mesh_k as double, in place over the Ext<float> state;
//   mode 3: out = log2(in_k) as double (masses back to FP64 log masses, in place over mode 1's output);
//   mode 4: the inverse of mode 2, in place: the Ext<float> state 2^(out_k - b mesh_k).
struct FastStateTask {
    void* out;
    const double* in;
    const double* mesh;
    long long n;
    double a, b;
    int mode;
    int pad;
};
void enqueue_fast_state(Alloc& al, const std::vector<FastStateTask>& tasks, hipStream_t s);

// Static range bound of every tile of both products of a 1D problem; when
// it holds, B = 2^{2 c kappa} of both meshes into *Bx / *By and the masses u,
// v as Ext<float> over the log masses lu, lv (which the bound has read).
// With convert_always the conversions are made also when the bound fails
// (for the resident solver's extended-number variant); the return value is
// still the bound's.
bool setup_fast_1d(Alloc& al, const Part& pk, const Part& pkt, double* lu, double* lv, const double* u,
                   const double* v, double eps, Ext<float>** Bx, Ext<float>** By, hipStream_t s,
                   bool convert_always = false);

constexpr double kCoordLimit = 33554432.0;   // 2^25: bound on |coordinate| / (eps ln 2)

// ---------------------------------------------------------------------------
// FP32 mode: the stop of Algorithm 1's loop head confirmed in FP64.
// The FP32 loops decide with their own estimate of the marginal error (FP32
// sums, a few units of 2^-24 per entry of K^T phi). When one stops, the
// returned pair is checked again with FP64 scans (the general sweep with FP64
// mantissas): ||diag(psi_old) K^T phi - v||_1 in FP64. That value is the
// reported error and decides convergence; if it exceeds tol before the cap,
// the loop resumes from the same pair with a lower threshold for its estimate
// (resume_threshold) and stops again later, to be checked again.
// ---------------------------------------------------------------------------
// Where a loop whose stop the FP64 check rejected at iteration l stops next:
// it runs k more iterations with its own estimate's stop switched off and is
// checked again; k doubles from 1 at each rejection of the same solve (at most
// 64), never past the cap. The FP64 error of an FP32 pair carries the FP32
// rounding of its states (about 1e-7 on unit mass), so its decrease over one
// iteration near tol is no guide to how many more are needed; doubling reaches
// any count in a logarithmic number of checks and overshoots it at most 2x.
inline long long resume_step(long long k_prev) { return k_prev < 1 ? 1 : std::min<long long>(64, 2 * k_prev); }
inline long long resume_until(long long l, long long k, long long cap) { return std::min(cap, l + k); }
// ---------------------------------------------------------------------------
// Precision 2: the linear domain with the stored vector representation of
// section 2.2 (finom_linear.hip)
// ---------------------------------------------------------------------------
// Whether the mode's scalings fit FP64 for a mesh spanning [lo, hi].
bool linear_span_ok(double lo, double hi, double eps);
// K w for the product of partition p (rows p.xr, columns p.yc), linear.
void linear_matvec(Alloc& al, const Part& p, double eps, const double* w, double* out, int cfg, hipStream_t s);
// Algorithm 1 with the linear-domain products: phi (n), psi[2] (m) scalings;
// *ret_psi is the psi buffer of the returned pair.
int linear_loop(Alloc& al, const Part& pk, const Part& pkt, int cfg, const double* u, const double* v, double eps,
                long long itr_max, int k, double* phi, double* psi[2], ProbState* ps, ProbState* hps,
                hipStream_t s, finom_result* res, int* ret_psi);

// A rejected stop resumes only if the loop has advanced since the last resume
// (a guard: every resume runs at least one iteration).
inline bool may_resume(long long l, long long last_resume_l) { return l > last_resume_l; }
// A streaming loop resumed at a graph's first iteration (parity 0): psi of
// iteration l sits in G[(l & 1) ^ shift], shift = (l_resume & 1).
inline int psi_slot(long long l, int shift) { return (int)((l & 1) ^ shift); }
// Re-arms a stopped state for a resumed loop: not done, the estimate's stop
// off (threshold -1), stop at iteration itr_stop, iteration l in both
// counter slots (iters keeps l: the resident solver starts from it).
void enqueue_rearm(ProbState* ps, long long l, long long itr_stop, hipStream_t s);

// ---------------------------------------------------------------------------
// The 2D loop on extended-number state (FP32 mode, finom_line_ext.hpp),
// shared by sinkhorn_w1_2d and the batch engine so that a problem runs the
// same launches alone and in a batch
// ---------------------------------------------------------------------------
// Line shape for a 2D problem (-1: the general sweeps run it).
int ext2d_shape(long long n1, long long m1, long long n2, long long m2, int precision);
// Bytes of the arrays, and their carving from one block of that size.
size_t ext2d_bytes(long long n1, long long m1, long long n2, long long m2);
void ext2d_bind(Ext2D& e, char* mem, long long n1, long long m1, long long n2, long long m2, int shape);
// Launch descriptors on the four partitions (px: rows x1, columns x2; py:
// rows y1, columns y2; *_t transposed) for problem state `prob`.
void ext2d_setup(Ext2D& e, const Part& px, const Part& px_t, const Part& py, const Part& py_t, int prob);
// 2^{2 c kappa} per axis, phi = 1 / (n1 m1), psi = 1 / (n2 m2) and the masses
// from their log2 (lu column-major, lvr row-major).
// Also decides the scan (Ext2D::s64; reads the axis meshes on the host).
void ext2d_init(Ext2D& e, const double* x1, const double* x2, const double* y1, const double* y2,
                const double* lu, const double* lvr, double kappa, hipStream_t s);
void ext2d_prologue(const Ext2D& e, ProbState* ps, hipStream_t s);
void ext2d_iteration(const Ext2D& e, int parity, ProbState* ps, hipStream_t s);
// One iteration of every problem of a group: two launches in all.
void ext2d_group_iteration(const Ext2DGroup& g, int parity, ProbState* ps, hipStream_t s);
// phi and psi (buffer bo) as log2 potentials into F (column-major) and G (row-major).
void ext2d_to_log2(const Ext2D& e, int bo, double* F, double* G, const double* x1, const double* x2,
                   const double* y1, const double* y2, double kappa, hipStream_t s);

// ---------------------------------------------------------------------------
// Line builders shared by the single-problem solvers and the batch engine
// ---------------------------------------------------------------------------

// Lines of a 2D sweep along the first axis: every column j of an
// (in_rows x ncols) column-major input is one line.
inline void add_axis0_lines(Sweep& sw, const Part& p, double eps, const double* in, long long in_rows,
                            double* out, long long out_rows, long long ncols, int prob = 0)
{
    for (long long j = 0; j < ncols; ++j) {
        LineDesc L = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
        L.gin = in + j * in_rows;
        L.out = out + j * out_rows;
        L.dec_part_off = -1;
        L.prob = prob;
        sw.lines.push_back(L);
    }
}

// ---------------------------------------------------------------------------
// 2D solves keep psi (and the target-side masses the check reads) row-major,
// element (l, j) of the n2 x m2 target grid at j + l m2, while phi stays
// column-major (k + i n1). Every sweep then reads contiguous lines, and the
// only strided stream of a product is the store of its intermediate: K^T phi
// runs along x (columns of phi into the n2 x m1 intermediate, stored
// row-major) and then along y (rows of the intermediate into rows of psi);
// K psi runs along y first (rows of psi into the intermediate, stored
// column-major) and then along x (its columns into columns of phi). The
// products along the two axes commute (eq. 2d-kpsi).
// ---------------------------------------------------------------------------

// K^T phi, along x: line i (< m1) reads column i of phi (contiguous, n1
// points) and writes column i of the row-major n2 x m1 intermediate (stride m1).
inline void add_2d_kt_x_lines(Sweep& sw, const Part& p, double eps, const double* F, long long n1, double* S,
                              long long m1, int prob = 0)
{
    for (long long i = 0; i < m1; ++i) {
        LineDesc L = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
        L.gin = F + i * n1;
        L.out = S + i;
        L.ostride = m1;
        L.dec_part_off = -1;
        L.prob = prob;
        sw.lines.push_back(L);
    }
}

// K^T phi, along y: line l (< n2) reads row l of the row-major intermediate
// (contiguous, m1 points) and writes row l of psi (contiguous, m2 points); the
// epilogue operands are indexed as psi.
inline void add_2d_kt_y_lines(Sweep& sw, const Part& p, double eps, const double* S, long long m1,
                              double* G, long long m2, const double* a0, const double* a1, const double* a2,
                              long long n2, int prob = 0)
{
    for (long long l = 0; l < n2; ++l) {
        LineDesc L = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
        L.gin = S + l * m1;
        L.out = G + l * m2;
        L.a0 = a0 ? a0 + l * m2 : nullptr;
        L.a1 = a1 ? a1 + l * m2 : nullptr;
        L.a2 = a2 ? a2 + l * m2 : nullptr;
        L.dec_part_off = -1;
        L.prob = prob;
        sw.lines.push_back(L);
    }
}

// K psi, along y: line l (< n2) reads row l of psi (contiguous, m2 points)
// and writes row l of the column-major n2 x m1 intermediate (stride n2).
inline void add_2d_k_y_lines(Sweep& sw, const Part& p, double eps, const double* G, long long m2, double* S,
                             long long m1, long long n2, int prob = 0)
{
    for (long long l = 0; l < n2; ++l) {
        LineDesc L = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
        L.gin = G + l * m2;
        L.out = S + l;
        L.ostride = n2;
        L.dec_part_off = -1;
        L.prob = prob;
        sw.lines.push_back(L);
    }
}

// K psi, along x: line i (< m1) reads column i of the column-major
// intermediate (contiguous, n2 points) and writes column i of phi (contiguous,
// n1 points), or only reads phi there (a0) when out is NULL (the cost sweeps).
inline void add_2d_k_x_lines(Sweep& sw, const Part& p, double eps, const double* S, long long n2, double* F,
                             long long n1, const double* a0, long long m1, int prob = 0)
{
    for (long long i = 0; i < m1; ++i) {
        LineDesc L = make_line(p.xr, p.R, p.yc, p.C, p.zeta, p.trs, p.T, eps);
        L.gin = S + i * n2;
        L.out = F ? F + i * n1 : nullptr;
        L.a0 = a0 ? a0 + i * n1 : nullptr;
        L.dec_part_off = -1;
        L.prob = prob;
        sw.lines.push_back(L);
    }
}

// b = f a, with a's (rows x cols) column-major grid written row-major
// (to_rows) or a's row-major grid written column-major (!to_rows).
template <int = 0>
__global__ __launch_bounds__(kBlock) void k_transpose_scale(const double* __restrict__ a, double* __restrict__ b,
                                                            long long rows, long long cols, int to_rows, double f)
{
    const long long n = rows * cols;
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < n; k += (long long)gridDim.x * kBlock) {
        if (to_rows) {
            const long long l = k / cols, j = k - l * cols;   // b[j + l cols] = a[l + j rows]
            b[k] = a[l + j * rows] * f;
        } else {
            const long long j = k / rows, l = k - j * rows;   // b[l + j rows] = a[j + l cols]
            b[k] = a[j + l * cols] * f;
        }
    }
}

inline void enqueue_transpose_scale(const double* a, double* b, long long rows, long long cols, bool to_rows,
                                    double f, hipStream_t s)
{
    const long long n = rows * cols;
    const unsigned grid = (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_transpose_scale<0>, dim3(std::max(1u, grid)), dim3(kBlock), 0, s, a, b, rows, cols,
                       to_rows ? 1 : 0, f);
}

// Partial-slot layout of a checking / cost sweep: consecutive per line.
inline int assign_parts(Sweep& sw, int base)
{
    int off = base;
    for (auto& L : sw.lines) {
        L.part_base = off;
        off += L.ntiles;
    }
    return off - base;
}

}  // namespace finom
