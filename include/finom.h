/*
 * finom.h - C ABI of the MI355X (gfx950) FINOM library.
 *
 * Entropic Wasserstein-1 with L1 cost on non-uniform 1D meshes and on
 * tensor-product meshes in two or more dimensions, solved by Sinkhorn
 * iterations whose kernel-vector products K psi and K^T phi use the
 * dividing-index split of K = exp(-C/eps) into two quasi-collinear blocks and
 * their O(N) recurrences (section 2, eq. decompose to p+q, eq. p-DP,
 * eq. q-DP; section 3, eq. 2d-kron, Algorithms 1 and 2); the transport plans
 * of the results and their differences (section 4).
 *
 * Conventions for every entry point
 *  - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *    owned by the caller, float64, contiguous. The library never frees them.
 *  - Meshes must be non-decreasing (ties allowed); the library does not sort,
 *    because sorting would permute the caller's masses.
 *  - Every coordinate must satisfy |c| / (eps ln 2) < 2^25: the products are
 *    formed from 2^(+-c/(eps ln 2)) with a 32-bit binary exponent. Checked on
 *    the end points of each mesh (FINOM_E_ARG) unless skip_checks is set.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is enqueued on that stream. Entry points that return host results
 *    (finom_result, device-side validation) synchronise that stream.
 *  - Internal workspace is cached per stream and released by finom_release().
 *    Calls on the same stream from different host threads must be serialised
 *    by the caller; distinct streams are independent.
 *  - Return value: FINOM_OK (0), a positive warning (results written) or a
 *    negative error (nothing written). No exception crosses the ABI.
 *  - Potentials are returned in natural-log units: f = eps ln phi and
 *    g = eps ln psi, so Gamma_ij = exp((f_i + g_j - C_ij)/eps).
 */
#ifndef FINOM_H
#define FINOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FINOM_OK = 0,
    FINOM_NOT_CONVERGED = 1,   /* iteration cap reached before err <= tol; results valid */
    FINOM_E_ARG = -1,          /* bad argument (null pointer, size < 1, eps <= 0, ...)   */
    FINOM_E_UNSORTED = -2,     /* a mesh is decreasing somewhere or holds a NaN         */
    FINOM_E_MASS = -3,         /* a mass is <= 0 / non-finite, or sum(u) != sum(v)      */
    FINOM_E_NOMEM = -4,        /* device or pinned allocation failed                    */
    FINOM_E_HIP = -5,          /* a HIP runtime call failed                              */
    FINOM_E_ADMIT = -6,        /* serving: request larger than the HBM budget           */
    FINOM_E_NUMERIC = -7       /* non-finite marginal error during the iteration        */
} finom_status;

/* Options. A NULL pointer means all defaults (zero-initialised struct). */
typedef struct {
    int32_t precision;  /* 0 = FP64 scans, FP64 log potentials as state.
                           1 = FP32-mantissa scans. The state is FP64 log potentials on
                           the general sweeps (result fast = 0: d >= 3, 2D with an axis
                           mesh longer than 2048) and the scalings
                           U = w 2^(-c/(eps ln 2)) as FP32 mantissa + int32 exponent on
                           the fast and resident sweeps (fast = 1, 2, 3) and the 2D
                           extended-state loop (fast = 4; c is the sum of the point's
                           two coordinates).
                           The loop head's stop test uses the loop's own FP32-sum
                           estimate; every stop is then confirmed by an FP64 check of
                           the returned pair (K^T phi with FP64 scans), which is the
                           reported marginal_err and decides convergence (a rejected
                           stop resumes the loop). The cost is FP64 in both modes.
                        2 = the linear domain with the stored vector representation
                           of section 2.2 (r_i per row, each column's lower- and
                           upper-block entries), eq. p-DP / q-DP as FP64 scans of
                           affine maps: no exponential or logarithm per iteration.
                           sinkhorn_w1_1d and finom_matvec (domain 0) only; the
                           scalings must fit FP64, so sinkhorn_w1_1d refuses
                           (FINOM_E_ARG) meshes with (max - min coordinate) / eps >
                           600, and a scaling that overflows or underflows on the
                           way ends the loop with FINOM_E_NUMERIC.                   */
    int32_t domain;     /* matvec entry points only: 0 = linear (out = K in, in >= 0);
                           1 = log (in = eps ln psi, out = eps ln K psi).               */
    int32_t skip_checks;/* 1 = trust the inputs: no device-side sortedness / mass checks
                           (and no stream synchronisation for them).                    */
    int32_t graph_iters;/* solver: iterations per captured HIP graph launch; 0 = default.*/
} finom_opts;

typedef struct {
    double w1;            /* <C, Gamma> of the returned pair, FP64                       */
    double marginal_err;  /* ||diag(psi) K^T phi - v||_1 of the returned pair (loop-head
                             check of Algorithm 1), with FP64 scans in both modes        */
    int64_t iters;        /* completed iterations l                                      */
    int32_t converged;    /* marginal_err <= tol                                         */
    int32_t status;       /* the value the call returned                                 */
    double loop_ms;       /* GPU time of the iteration loop (HIP events on `stream`),
                             excluding setup and the final cost reduction             */
    int64_t sweeps;       /* half-iteration products executed in the loop: 2 l + 1     */
    int32_t fast;         /* 1D, precision 1: which loop ran. With every tile inside
                             the FP32 exponent range: 1 for the streaming FP32 fast sweeps,
                             2 for the resident solver (one cooperative launch holding the
                             state on chip; single calls and finom_batch members whose
                             tiles fit the GPU at once). Beyond that range: 3 for the
                             resident solver's extended-number variant (same condition),
                             else 0 (the streaming general sweeps). 2D, precision 1: 4 for
                             the extended-state loop (every axis mesh of at most 2048
                             points: one block per line holds the whole line, each pair
                             of products along one axis in one launch), else 0. 0 for
                             precision 0 and d >= 3 (sinkhorn_w1_nd with one or two axes
                             reports as sinkhorn_w1_1d / _2d). finom_batch members and
                             server requests report what their single calls report. */
    int32_t resumes;      /* precision 1: stops of the FP32 loop that the FP64 check of
                             the returned pair rejected (the loop then went on); 0 for
                             precision 0                                               */
} finom_result;

/*
 * K * in for the 1D kernel K_ij = exp(-|x_rows_i - y_cols_j| / eps)
 * (section 2.1) through the dividing-index split and the two recurrences
 * (eq. decompose to p+q, eq. p-DP, eq. q-DP).
 *   x_rows: n row coordinates; y_cols: m column coordinates (both ascending).
 *   in: m values (domain 0: psi >= 0; domain 1: eps ln psi, -inf allowed).
 *   out: n values (domain 0: K psi; domain 1: eps ln K psi).
 * K^T * u is the same call with (y_cols, m) as rows and (x_rows, n) as
 * columns. Errors: FINOM_E_ARG, FINOM_E_UNSORTED, FINOM_E_NOMEM, FINOM_E_HIP.
 */
int finom_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m,
                 double eps, const double* in, double* out, const finom_opts* opts,
                 void* stream);
/* (finom_matvec with opts->precision 2 evaluates the linear-domain product
 * from the stored representation; domain must be 0, else FINOM_E_ARG.
 * dense_matvec, finom_matvec_noalloc, sinkhorn_w1_2d, sinkhorn_w1_nd,
 * finom_batch and the server accept precision 0 and 1 only.) */

/*
 * The same product evaluated densely, O(n*m) kernel entries generated on the
 * fly ("standard Sinkhorn" product of section 4). Baseline; identical
 * signature and semantics to finom_matvec.
 */
int dense_matvec(const double* x_rows, int64_t n, const double* y_cols, int64_t m,
                 double eps, const double* in, double* out, const finom_opts* opts,
                 void* stream);

/*
 * The 2D dense baselines (section 4's standard Sinkhorn on tensor meshes,
 * eq. 2d-kron), log domain: out = eps ln (K e^{in/eps}) for the kernel
 * K((k,i),(l,j)) = exp(-(|x1_k - x2_l| + |y1_i - y2_j|)/eps) from the target
 * grid x2 (n2) x y2 (m2) to the source grid x1 (n1) x y1 (m1). in: n2*m2 and
 * out: n1*m1 column-major (element (l, j) at l + j*n2). K^T is the same call
 * with the grids swapped.
 *   full = 0: per axis, vec(K_x E K_y^T) as two dense FP64 matrix products on
 *     the matrix cores, every kernel entry generated as its tile is loaded;
 *     each operand is shifted by its column (row) maximum so that the linear
 *     values stay in FP64 while exp(-diam/eps) does not underflow.
 *   full = 1: the (n1 m1) x (n2 m2) product with one exponential per kernel
 *     entry and a running maximum per output (vector units).
 * Meshes need not be sorted. Asynchronous on `stream`; full = 0 uses the
 * per-stream workspace (16 (n1 + n2) m2 bytes). Errors: FINOM_E_ARG,
 * FINOM_E_NOMEM, FINOM_E_HIP.
 */
int dense_matvec_2d(const double* x1, int64_t n1, const double* y1, int64_t m1,
                    const double* x2, int64_t n2, const double* y2, int64_t m2,
                    double eps, const double* in, double* out, int32_t full, void* stream);

/* Largest n + m that finom_matvec_noalloc accepts (2^22 merged points). */
#define FINOM_NOALLOC_MAX_POINTS 4194304

/*
 * finom_matvec for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, semantics, kernels and tile shape as finom_matvec, so the
 * output is the same bit for bit. It allocates nothing (no hipMalloc,
 * hipFree or pinned host memory) and never synchronises: it only enqueues
 * kernels on `stream`. Its working arrays (dividing index, tile starts, work
 * list, descriptor, tile aggregates) live in one fixed device array of about
 * 16.4 MiB per device, which each device that runs it holds until the
 * process ends. Calls on one device share that array: calls that overlap on
 * a device (other streams, or host threads without ordering) race and give
 * wrong results; calls on one stream are ordered and safe.
 * Not checked on the device (as with opts->skip_checks = 1): the meshes
 * must be non-decreasing and within the coordinate range of the
 * conventions above; violating inputs give wrong values, never an
 * out-of-range access.
 * Errors (nothing enqueued): FINOM_E_ARG for the argument errors of
 * finom_matvec and for n + m > FINOM_NOALLOC_MAX_POINTS (finom_last_error
 * then names the limit); FINOM_E_HIP if the array's device address cannot
 * be taken or a launch fails.
 */
int finom_matvec_noalloc(const double* x_rows, int64_t n, const double* y_cols, int64_t m,
                         double eps, const double* in, double* out, const finom_opts* opts,
                         void* stream);

/*
 * Algorithm 1 (1D FINOM Sinkhorn) on meshes x (n) and y (m), masses u (n) and
 * v (m), all > 0 with sum(u) == sum(v) within 1e-12 relative.
 * Initialisation phi = 1/n, psi = 1/m. Loop while l < itr_max and
 * ||diag(psi) K^T phi - v||_1 > tol: psi = v / K^T phi, phi = u / K psi.
 * f_out (n) / g_out (m): device outputs eps ln phi / eps ln psi of the
 * returned pair (the one whose error was checked last); either may be NULL.
 * res (HOST pointer, required) receives w1 = <C, Gamma>, the error, l.
 * Returns FINOM_OK, FINOM_NOT_CONVERGED, or an error
 * (FINOM_E_ARG / _UNSORTED / _MASS / _NOMEM / _HIP / _NUMERIC).
 */
int sinkhorn_w1_1d(const double* x, int64_t n, const double* y, int64_t m,
                   const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream);

/*
 * Algorithm 2 (2D FINOM Sinkhorn) on tensor-product meshes: source grid
 * x1 (n1) x y1 (m1), target grid x2 (n2) x y2 (m2), cost |dx| + |dy|, so
 * K = K_y (x) K_x (eq. 2d-kron). u (n1*m1) and v (n2*m2) are column-major:
 * element (k, i) at k + i*n1 (the paper's grid order, section 3.1). Each
 * product is evaluated axis by axis, K^T phi = vec(K_x^T Phi K_y) and
 * K psi = vec(K_x Psi K_y^T) (eq. 2d-ktphi, eq. 2d-kpsi), with the potentials
 * absorbed as in the appendix (columns with the right absorption, rows with
 * the left one). Initialisation Phi = 1/(n1 m1), Psi = 1/(n2 m2); the loop,
 * the check and the outputs (f_out: n1*m1, g_out: n2*m2, column-major) are as
 * in sinkhorn_w1_1d. w1 = <|dx| + |dy|, Gamma> in FP64.
 */
int sinkhorn_w1_2d(const double* x1, int64_t n1, const double* y1, int64_t m1,
                   const double* x2, int64_t n2, const double* y2, int64_t m2,
                   const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream);

/* Largest number of axes sinkhorn_w1_nd accepts. */
#define FINOM_MAX_DIMS 8

/*
 * The Sinkhorn loop of Algorithms 1 and 2 on d-dimensional tensor-product
 * meshes (the remark closing section 3): the kernel factorises as
 * K = K_{d-1} (x) ... (x) K_0 for the cost sum_a |x_a - y_a|, and each product
 * is applied along one axis after another with the 1D method.
 * n_src, n_tgt: HOST arrays of d axis lengths (each >= 1); x_src, x_tgt: HOST
 * arrays of d DEVICE pointers to the non-decreasing axis coordinates.
 * u (prod n_src) and v (prod n_tgt) are column-major grids: element
 * (k_0, ..., k_{d-1}) at k_0 + n_0 (k_1 + n_1 (k_2 + ...)), axis 0 fastest;
 * f_out / g_out use the same layout. d = 1 runs sinkhorn_w1_1d and d = 2
 * sinkhorn_w1_2d (same results, bit for bit); d >= 3 runs the general sweeps
 * along every axis. Loop, check, outputs and errors as in sinkhorn_w1_2d;
 * w1 = <sum_a |x_a - y_a|, Gamma> in FP64. FINOM_E_ARG also for d < 1 or
 * d > FINOM_MAX_DIMS.
 */
int sinkhorn_w1_nd(int32_t d, const int64_t* n_src, const double* const* x_src,
                   const int64_t* n_tgt, const double* const* x_tgt,
                   const double* u, const double* v, double eps, double tol,
                   int64_t itr_max, const finom_opts* opts, double* f_out,
                   double* g_out, finom_result* res, void* stream);

/*
 * The transport plan Gamma = diag(phi) K diag(psi) (section 2.1), written
 * densely from the potentials f = eps ln phi (n) and g = eps ln psi (m) that
 * sinkhorn_w1_1d returns; these are the plans whose difference the tables of
 * section 4 report. gamma (device, caller-owned, n * ld doubles, row-major,
 * ld >= m) receives gamma[i*ld + j] = exp(((f_i + g_j) - |x_i - y_j|) / eps)
 * in FP64; the entries j >= m of a row are left untouched. x and y need not
 * be sorted. Asynchronous on `stream`; nothing is allocated.
 * Errors (nothing written): FINOM_E_ARG (NULL pointer, size < 1, ld < m,
 * eps <= 0 or not finite, n * ld overflows), FINOM_E_HIP.
 */
int finom_plan_1d(const double* x, int64_t n, const double* y, int64_t m,
                  const double* f, const double* g, double eps, double* gamma,
                  int64_t ld, void* stream);

/*
 * The same on tensor-product meshes (eq. 2d-kron): source grid x1 (n1) x
 * y1 (m1), target grid x2 (n2) x y2 (m2), potentials f (n1*m1) and g (n2*m2)
 * column-major as sinkhorn_w1_2d returns them. Row r = k + i*n1 is source
 * point (x1_k, y1_i), column c = l + j*n2 is target point (x2_l, y2_j), and
 * gamma[r*ld + c] = exp(((f_r + g_c) - (|x1_k - x2_l| + |y1_i - y2_j|)) / eps),
 * ld >= n2*m2. Errors as finom_plan_1d.
 */
int finom_plan_2d(const double* x1, int64_t n1, const double* y1, int64_t m1,
                  const double* x2, int64_t n2, const double* y2, int64_t m2,
                  const double* f, const double* g, double eps, double* gamma,
                  int64_t ld, void* stream);

/*
 * ||Gamma_a - Gamma_b||_F for two plans on the same 1D meshes, each given by
 * its potentials (fa, ga) and (fb, gb) as in finom_plan_1d: the plan
 * difference column of section 4's tables. Each entry difference is taken
 * between the two FP64 plan entries as finom_plan_1d would write them; no
 * plan is stored. out: one double in DEVICE memory, written asynchronously
 * on `stream`. The sum of squares is reduced in a fixed order, so repeated
 * calls give the same bits. Uses the per-stream workspace (16 KB).
 * Errors (nothing written): FINOM_E_ARG (NULL pointer, size < 1, eps <= 0 or
 * not finite), FINOM_E_NOMEM, FINOM_E_HIP.
 */
int finom_plan_diff_1d(const double* x, int64_t n, const double* y, int64_t m,
                       const double* fa, const double* ga, const double* fb,
                       const double* gb, double eps, double* out, void* stream);

/* The same on tensor-product meshes, with the layout of finom_plan_2d. */
int finom_plan_diff_2d(const double* x1, int64_t n1, const double* y1, int64_t m1,
                       const double* x2, int64_t n2, const double* y2, int64_t m2,
                       const double* fa, const double* ga, const double* fb,
                       const double* gb, double eps, double* out, void* stream);

/*
 * One problem of a batch or a serving request. dim = 1: Algorithm 1 on
 * x = x1 (n1 points, masses u) and y = x2 (n2 points, masses v); m1, m2, y1,
 * y2 are ignored. dim = 2: Algorithm 2 on the grids x1 (n1) x y1 (m1) and
 * x2 (n2) x y2 (m2) with column-major u, v as in sinkhorn_w1_2d. All arrays
 * are device arrays owned by the caller; f_out / g_out may be NULL.
 */
typedef struct {
    int32_t dim;
    int32_t reserved;     /* 0 */
    int64_t n1, m1, n2, m2;
    const double *x1, *y1, *x2, *y2;
    const double *u, *v;
    double eps, tol;
    int64_t itr_max;
    double *f_out, *g_out;
} finom_problem;

/*
 * Solves `count` independent problems (1D and 2D may be mixed) together: the
 * lines of all live problems share each sweep launch, every problem keeps its
 * own iteration counter, loop-head check and stop decision (the iteration of
 * Algorithm 1 / Algorithm 2 is unchanged), and stopped problems retire from
 * the launches. In precision 1, the 1D problems that fit the resident solver
 * run first on persistent grids (one per variant, the two at the same time),
 * and 2D problems on the extended-state loop each run their own line-pair
 * launches within the rounds. A problem's results equal those of
 * sinkhorn_w1_1d / sinkhorn_w1_2d on it alone.
 *   probs: HOST array of count descriptors; res: HOST array of count results
 *   (res[i].status per problem). Problems that fail validation are skipped
 *   (their status says why); the others are solved.
 * Returns FINOM_OK if every problem converged, FINOM_NOT_CONVERGED if some hit
 * their cap, else the first negative per-problem status (FINOM_E_ARG for a
 * bad count or pointer, in which case nothing runs).
 */
int finom_batch(const finom_problem* probs, int64_t count, const finom_opts* opts,
                finom_result* res, void* stream);

/* Device bytes the library holds for one problem while it is being solved
 * (the serving admission unit). Negative status for an invalid descriptor. */
int64_t finom_footprint(const finom_problem* p, const finom_opts* opts);

/*
 * Serving loop. A server owns a device memory budget, a HIP stream and a host
 * thread that admits submitted problems in arrival order while their
 * footprints fit the budget, joins them to the running batch between rounds of
 * a few iterations, and publishes each result when its problem stops.
 * The caller keeps a problem's arrays alive and unmodified until its
 * completion has been polled, and makes them ready (synchronised) before
 * submitting. Calls on one server may come from any host thread.
 */
typedef struct finom_server finom_server;

typedef struct {
    int64_t ticket;
    finom_result res;
    double latency_ms;    /* submit -> result published */
    double queue_ms;      /* submit -> joined the batch  */
} finom_completion;

typedef struct {
    int64_t submitted, admitted, completed, rejected;
    int64_t live, queued, rounds;
    double grid_pt_iters; /* sum over completed problems of grid points x iterations */
    double busy_ms;       /* GPU time of the iteration rounds                         */
    uint64_t hbm_used, hbm_budget;
} finom_server_stats;

/* opts: precision and graph_iters (iterations per round, default 8) apply. */
int finom_server_create(uint64_t hbm_budget_bytes, const finom_opts* opts, finom_server** out);
/* FINOM_E_ADMIT if the problem's footprint exceeds the whole budget,
 * FINOM_E_ARG for an invalid descriptor (nothing queued in either case). */
int finom_server_submit(finom_server* srv, const finom_problem* p, int64_t* ticket);
/* Up to max completions into out (HOST); waits up to wait_ms for the first. */
int finom_server_poll(finom_server* srv, finom_completion* out, int64_t max, int64_t* n_out,
                      int32_t wait_ms);
int finom_server_stats_get(finom_server* srv, finom_server_stats* st);
/* Stops the thread after the live problems finish; pending results are dropped. */
void finom_server_destroy(finom_server* srv);

/*
 * Tile-shape autotuner: times every tile shape on merged-line lengths of
 * 2^9 .. 2^21 elements (batches that fill the GPU) and keeps the fastest per
 * size class for all later calls in the process. A class is timed where its
 * problems run: one iteration of the streaming sweeps, or, in precision 1 where
 * some shape keeps the class's 1D problems on the resident solver, a batch of
 * them through finom_batch (64 iterations at tol 0; only such shapes compete,
 * and shapes that cut the lines into the same tiles are told apart by the
 * streaming timing). Tuning calls finom_batch internally and synchronises
 * `stream`. With cache_path,
 * results are read from that file if it exists and written to it otherwise.
 * The general sweeps of 2D and d-dimensional problems run lines of at most
 * 256 merged points as one tile of an untuned one-wave shape (64 threads x 4).
 * The environment variable FINOM_TILE_CFG (0..4) overrides every choice.
 * The 2D extended-state loop takes its own line shape (threads per line x
 * points per thread: 64x4, 256x4, 256x8 by the longest axis mesh, <= 256,
 * <= 1024, <= 2048 points); FINOM_LINE_SHAPE (0..4: 64x4, 256x4, 256x8, 128x8,
 * 64x16) picks another that holds the longest mesh.
 */
int finom_autotune(int32_t precision, const char* cache_path, void* stream);
/* The tile-shape index used for a line of `merged` = rows + columns elements. */
int finom_tile_config(int32_t precision, int64_t merged);

/* Human-readable text for a status code (static storage). */
const char* finom_strerror(int status);

/* Frees all cached device/pinned workspace (all streams). Not concurrent-safe
 * with running calls. */
void finom_release(void);

/* Detail of the last FINOM_E_HIP / FINOM_E_NOMEM raised on the calling host
 * thread (the HIP error string and code), or of finom_matvec_noalloc's size
 * refusal; empty if none. Static storage. */
const char* finom_last_error(void);

/* Library version string, e.g. "finom-gfx950 0.1". */
const char* finom_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FINOM_H */
