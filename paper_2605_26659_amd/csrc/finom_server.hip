// Serving loop: continuous batching of Sinkhorn problems on one GPU.
//
// A host thread owns the batch engine, a HIP stream and a device slab (the
// memory budget). Between rounds of a few iterations it admits queued
// problems in arrival order while their footprints fit the free slab space,
// prepares them in one batched setup, joins them to the running batch and
// publishes the results of the problems that stopped. Problems never move:
// their state stays resident in the slab from admission to completion.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

#include "finom_engine.hpp"

using namespace finom;

namespace {

double now_ms()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double, std::milli>(clk::now().time_since_epoch()).count();
}

struct Req {
    Job job;
    double t_submit = 0.0, t_admit = 0.0;
};

constexpr int kServerSlots = 1 << 16;

}  // namespace

struct finom_server {
    int precision = 0;
    int k = 8;
    int checks = 1;
    int device = 0;
    hipStream_t s = nullptr;
    std::unique_ptr<Slab> slab;
    std::unique_ptr<Engine> eng;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Req*> queue;
    std::deque<finom_completion> done;
    bool stop = false;
    int failed = FINOM_OK;
    long long next_ticket = 1;
    finom_server_stats st{};

    void run();
    void complete(Req* r, const finom_result& res);
};

void finom_server::complete(Req* r, const finom_result& res)
{
    finom_completion c;
    memset(&c, 0, sizeof(c));
    c.ticket = r->job.tag;
    c.res = res;
    const double t = now_ms();
    c.latency_ms = t - r->t_submit;
    c.queue_ms = (r->t_admit > 0.0 ? r->t_admit : t) - r->t_submit;
    {
        std::lock_guard<std::mutex> lk(mu);
        done.push_back(c);
        st.completed += 1;
        if (res.status >= 0) st.grid_pt_iters += r->job.points() * (double)res.iters;
    }
    cv_out.notify_all();
}

void finom_server::run()
{
    hipSetDevice(device);
    std::vector<Req*> live;
    auto fail_all = [&](int status) {
        finom_result bad;
        memset(&bad, 0, sizeof(bad));
        bad.status = status;
        for (Req* r : live) {
            complete(r, bad);
            delete r;
        }
        live.clear();
        std::deque<Req*> q;
        {
            std::lock_guard<std::mutex> lk(mu);
            q.swap(queue);
            failed = status;
        }
        for (Req* r : q) {
            complete(r, bad);
            delete r;
        }
    };
    // the results of jobs that stopped: their memory back to the slab, their
    // completions to the caller
    auto publish = [&](const std::vector<Job*>& fin) {
        for (Job* j : fin) {
            Req* r = nullptr;
            for (size_t i = 0; i < live.size(); ++i)
                if (&live[i]->job == j) {
                    r = live[i];
                    live[i] = live.back();
                    live.pop_back();
                    break;
                }
            slab->release(j->mem, j->p.bytes);
            if (r) {
                complete(r, j->res);
                delete r;
            }
        }
    };
    try {
        for (;;) {
            std::vector<Req*> admit;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop) {
                    for (Req* r : queue) delete r;
                    queue.clear();
                    if (live.empty()) break;
                }
                if (live.empty() && queue.empty()) {
                    cv_in.wait_for(lk, std::chrono::milliseconds(20));
                    continue;
                }
                while (!queue.empty()) {
                    Req* r = queue.front();
                    char* m = slab->alloc(r->job.p.bytes);
                    if (!m) break;   // in arrival order: wait for memory
                    r->job.mem = m;
                    queue.pop_front();
                    admit.push_back(r);
                }
                st.queued = (int64_t)queue.size();
            }
            if (!admit.empty()) {
                std::vector<Job*> js;
                for (Req* r : admit) {
                    r->job.bind();
                    js.push_back(&r->job);
                }
                eng->setup(js, checks != 0);
                const double t = now_ms();
                for (Req* r : admit) {
                    r->t_admit = t;
                    if (r->job.status == FINOM_OK && eng->add(&r->job)) {
                        live.push_back(r);
                        continue;
                    }
                    finom_result bad;
                    memset(&bad, 0, sizeof(bad));
                    bad.status = r->job.status != FINOM_OK ? r->job.status : FINOM_E_ADMIT;
                    slab->release(r->job.mem, r->job.p.bytes);
                    complete(r, bad);
                    delete r;
                }
                std::lock_guard<std::mutex> lk(mu);
                st.admitted += (int64_t)admit.size();
            }
            // 1D FP32 requests that fit the resident solver are solved at once,
            // as a single call would solve them; the others join the rounds
            if (!admit.empty()) {
                eng->solve_resident();
                publish(eng->harvest());
            }
            if (eng->live() == 0) continue;
            eng->round(k);
            publish(eng->harvest());
            eng->maybe_compact(0.75);
            std::lock_guard<std::mutex> lk(mu);
            st.rounds += 1;
            st.live = eng->live();
            st.busy_ms = eng->loop_ms_total();
            st.hbm_used = slab->used();
        }
    } catch (...) {
        fail_all(map_exception());
    }
}


extern "C" {

int finom_server_create(uint64_t hbm_budget_bytes, const finom_opts* opts, finom_server** out)
{
    if (!out) return FINOM_E_ARG;
    *out = nullptr;
    finom_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision != 0 && o.precision != 1) return FINOM_E_ARG;
    if (hbm_budget_bytes < 4096) return FINOM_E_ARG;
    finom_server* srv = new (std::nothrow) finom_server();
    if (!srv) return FINOM_E_NOMEM;
    try {
        srv->precision = o.precision;
        srv->k = o.graph_iters > 0 ? o.graph_iters : 8;
        srv->checks = o.skip_checks ? 0 : 1;
        HIPCHK(hipGetDevice(&srv->device));
        HIPCHK(hipStreamCreateWithFlags(&srv->s, hipStreamNonBlocking));
        srv->slab.reset(new Slab((size_t)hbm_budget_bytes));
        srv->eng.reset(new Engine(o.precision, srv->s, kServerSlots, false));
        srv->eng->enable_resident();
        srv->st.hbm_budget = srv->slab->capacity();
        srv->th = std::thread([srv] { srv->run(); });
    } catch (...) {
        const int st = map_exception();
        srv->eng.reset();
        srv->slab.reset();
        if (srv->s) hipStreamDestroy(srv->s);
        delete srv;
        return st;
    }
    *out = srv;
    return FINOM_OK;
}

int finom_server_submit(finom_server* srv, const finom_problem* p, int64_t* ticket)
{
    if (!srv || !p) return FINOM_E_ARG;
    Req* r = new (std::nothrow) Req();
    if (!r) return FINOM_E_NOMEM;
    r->job.d = job_from_problem(*p);
    int st = check_job_args(r->job.d, srv->precision);
    if (st == FINOM_OK) {
        r->job.p = plan_job(r->job.d, srv->precision);
        if (r->job.p.bytes > srv->slab->capacity()) st = FINOM_E_ADMIT;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (st != FINOM_OK || srv->stop || srv->failed != FINOM_OK) {
        if (st == FINOM_E_ADMIT) srv->st.rejected += 1;
        delete r;
        return st != FINOM_OK ? st : (srv->failed != FINOM_OK ? srv->failed : FINOM_E_ARG);
    }
    r->job.tag = srv->next_ticket++;
    r->t_submit = now_ms();
    if (ticket) *ticket = r->job.tag;
    srv->queue.push_back(r);
    srv->st.submitted += 1;
    srv->st.queued = (int64_t)srv->queue.size();
    srv->cv_in.notify_one();
    return FINOM_OK;
}

int finom_server_poll(finom_server* srv, finom_completion* out, int64_t max, int64_t* n_out, int32_t wait_ms)
{
    if (!srv || !n_out || max < 0 || (max > 0 && !out)) return FINOM_E_ARG;
    *n_out = 0;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ms > 0)
        srv->cv_out.wait_for(lk, std::chrono::milliseconds(wait_ms), [srv] { return !srv->done.empty(); });
    int64_t n = 0;
    while (n < max && !srv->done.empty()) {
        out[n++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = n;
    return FINOM_OK;
}

int finom_server_stats_get(finom_server* srv, finom_server_stats* st)
{
    if (!srv || !st) return FINOM_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->st;
    st->queued = (int64_t)srv->queue.size();
    return srv->failed;
}

void finom_server_destroy(finom_server* srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_in.notify_all();
    if (srv->th.joinable()) srv->th.join();
    srv->eng.reset();
    srv->slab.reset();
    if (srv->s) hipStreamDestroy(srv->s);
    delete srv;
}

}  // extern "C"
