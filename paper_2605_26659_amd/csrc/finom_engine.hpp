// Batch engine: many independent Sinkhorn problems (1D Algorithm 1 and 2D
// Algorithm 2) iterated together. The lines of all live problems are merged
// into one sweep launch per (stage, tile shape); each problem keeps its own
// iteration state, takes its own stop decision and retires on its own. Used by
// the batched entry point and by the serving loop.
#pragma once
#include <functional>
#include <memory>
#include <queue>
#include <vector>

#include "../../include/finom.h"
#include "finom_host.hpp"
#include "finom_resident.hpp"

namespace finom {

struct JobDesc {
    int dim = 1;
    long long n1 = 0, m1 = 1, n2 = 0, m2 = 1;   // 1D: n = n1 (x = x1), m = n2 (y = x2)
    const double *x1 = nullptr, *y1 = nullptr, *x2 = nullptr, *y2 = nullptr;
    const double *u = nullptr, *v = nullptr;
    double eps = 0.0, tol = 0.0;
    long long itr_max = 0;
    double *f_out = nullptr, *g_out = nullptr;
};

JobDesc job_from_problem(const finom_problem& p);
// Host-side argument check (no device access). FINOM_OK or FINOM_E_ARG.
int check_job_args(const JobDesc& d, int precision);

// Sizes and byte offsets of the device block a job owns while it is live.
struct JobPlan {
    int dim = 1;
    int cfg[2] = {0, 0};
    long long na = 0, nb = 0, s_len = 0;
    long long R[2] = {0, 0}, C[2] = {0, 0};
    int ntiles[2] = {0, 0}, ntiles_c[2] = {0, 0};
    size_t o_lu = 0, o_lv = 0, o_F = 0, o_G0 = 0, o_G1 = 0, o_S = 0, o_Bx = 0, o_By = 0;
    size_t o_lvr = 0, o_vr = 0;   // 2D: log2 v and v row-major, as psi
    int lx_shape = -1;            // 2D FP32 on the extended-state loop: its line shape
    size_t o_lx = 0;              // and its arrays (ext2d_bind)
    size_t o_zeta[2] = {0, 0}, o_zeta_t[2] = {0, 0}, o_trs[2] = {0, 0}, o_trs_t[2] = {0, 0},
           o_trs_c[2] = {0, 0};
    size_t bytes = 0;
};

JobPlan plan_job(const JobDesc& d, int precision);

struct Job {
    JobDesc d;
    JobPlan p;
    char* mem = nullptr;     // device block of p.bytes
    int slot = -1;           // index of the iteration state
    int status = FINOM_OK;   // validation result
    long long tag = 0;       // caller's index or ticket
    double loop_ms = 0.0;    // GPU time of the rounds the job took part in
    finom_result res{};
    // views into mem. Jobs on the fast sweeps keep, in the same buffers, the
    // masses as Ext<float> in lu / lv and the state U = w 2^{-c kappa} in F / G
    // until they are harvested.
    double *lu = nullptr, *lv = nullptr, *F = nullptr, *G[2] = {nullptr, nullptr}, *S = nullptr;
    double *lvr = nullptr, *vr = nullptr;   // 2D: psi is row-major (element (l, j) at j + l m2), and so
                                            // are these copies of log2 v and v that its check reads
    Ext<float>* Bx = nullptr;   // 1D FP32: 2^{2 x kappa} and 2^{2 y kappa} for the fast sweeps
    Ext<float>* By = nullptr;
    bool fast = false;          // runs on the fast sweeps
    bool ext2d = false;         // 2D FP32 on the extended-state loop (lx; F and G hold log2 potentials only
                                // for its FP64 checks and the cost)
    Ext2D lx;
    bool gen = false;           // 1D FP32 beyond the fast bound, for the resident solver's extended-number
                                // variant (state as for the fast sweeps); only when the engine solves resident
    bool resident = false;      // solved by the resident batch kernel (final psi in G[0])
    bool started = false;       // its iteration state has been set (harvest looks at it only then)
    int shift = 0;              // streaming loop resumed after a rejected stop: psi of iteration l in
                                // G[(l & 1) ^ shift]
    int resumes = 0;            // stops the FP64 check rejected
    long long last_resume_l = -1;   // iteration of the last rejected stop
    long long resume_k = 0;         // iterations run after it
    double err64 = 0.0;         // FP32 mode: the FP64 check of the returned pair
    Part pk[2], pkt[2], pc[2];   // per axis: K, K^T, cost partition of K
    void bind();
    double points() const { return 0.5 * (double)(p.na + p.nb); }
};

// One persistent grid of the resident batch kernel, prepared for launch.
struct ResidentGrid {
    std::vector<Job*> jobs;   // in tile hand-out order
    ResidentBatch b{};
    int grid = 0;
    bool gen = false;
    int* flags = nullptr;     // device: fail flag, tile counter
    int* hfail = nullptr;     // pinned copy of the fail flag
};

class Engine {
public:
    Engine(int precision, hipStream_t stream, int capacity, bool use_graphs);
    ~Engine();
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;

    // Validates and prepares jobs whose memory is bound (dividing indices,
    // merge-path partitions, log masses, initial potentials). Sets status.
    void setup(const std::vector<Job*>& jobs, bool checks);
    // Joins a prepared job to the iteration (between rounds). False when no
    // state slot is free.
    bool add(Job* j);
    // Lets setup() prepare 1D FP32 jobs beyond the fast bound for the resident
    // solver; the caller then runs solve_resident() before any round.
    void enable_resident() { resident_ = true; }
    // Solves the 1D FP32 jobs that joined since the last round and fit the
    // resident solver, to the end of their loops, in one persistent launch per
    // variant (the two variants' grids run at the same time); they are then
    // ready for harvest. The other jobs are left to round().
    void solve_resident();
    // k iterations (k even) of every live job; then reads their states.
    void round(int k);
    // Jobs that stopped in the last round: costs, outputs, results. They
    // leave the engine.
    std::vector<Job*> harvest();
    int live() const { return (int)active_.size(); }
    long long live_tiles() const;
    long long listed_tiles() const { return listed_tiles_; }
    // Rebuilds the launch lists without the retired jobs when they hold a
    // large share of the listed work.
    void maybe_compact(double keep_fraction);
    double loop_ms_total() const { return loop_ms_total_; }

private:
    void rebuild();
    // resume: the jobs' states are already armed (a stop the FP64 check
    // rejected); otherwise they are initialised
    void run_resident_batch(const std::vector<Job*>& rj, bool gen, bool resume = false);
    // the parts of a resident batch launch: state initialisation, records and
    // arguments (on s_), the launch (cooperative or not) between two events,
    // and the jobs' bookkeeping once the grid has finished
    void prepare_resident(Alloc& al, const std::vector<Job*>& jobs, bool gen, bool resume, ResidentGrid& g);
    void launch_resident(ResidentGrid& g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, bool coop);
    void finish_resident(const ResidentGrid& g, float ms);
    // FP32 mode: the FP64 check of every stopped job's returned pair; jobs
    // that fail it before their cap resume (the resident ones are solved on
    // here, the streaming ones go on in the next rounds) and leave `fin`
    void confirm_stops(std::vector<Job*>& fin);
    void launch_iterations(int k, hipStream_t s);
    void read_states();

    int precision_;
    hipStream_t s_;
    int cap_;
    bool use_graphs_;
    bool resident_ = false;
    ProbState* ps_ = nullptr;       // cap_ + 1 states; the last is the cost sweeps' (never done)
    ProbState* hps_ = nullptr;      // pinned mirror
    std::priority_queue<int, std::vector<int>, std::greater<int>> free_slots_;   // lowest first
    int max_slot_ = -1;
    std::vector<Job*> active_;      // live jobs, in join order
    std::vector<Job*> pending_init_;   // joined since the last rebuild
    std::vector<Job*> listed_;      // jobs in the current launch lists
    std::vector<Ext2DGroup> lx_groups_;   // launches of the listed jobs on the extended-state 2D loop,
                                          // by line shape and scan
    Arena ar_setup_, ar_loop_, ar_cost_, ar_res_, ar_chk_;
    std::vector<std::unique_ptr<Sweep>> sweeps_;
    std::vector<Sweep*> seq_[2];
    std::vector<bool> dec_[2];
    double* partial_ = nullptr;
    long long listed_tiles_ = 0;
    bool dirty_ = true;
    int stable_ = 0;
    hipStream_t cs_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    int graph_k_ = 0;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    hipStream_t s2_ = nullptr;      // the second resident grid's stream
    hipEvent_t ev2_ = nullptr, ev3_ = nullptr, evu_ = nullptr;
    double loop_ms_total_ = 0.0;
    void drop_graph();
};

// First-fit sub-allocator over one device slab (the serving memory budget).
class Slab {
public:
    explicit Slab(size_t bytes);
    ~Slab();
    char* alloc(size_t bytes);        // nullptr when no free range fits
    void release(char* p, size_t bytes);
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

private:
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    std::vector<std::pair<size_t, size_t>> free_;   // (offset, size), sorted by offset
};

}  // namespace finom
