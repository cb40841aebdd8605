// Request server: continuous batching of factor+solve and solve-only
// requests over resident sparsity patterns on one device.
//
// Every pattern (a symbolic handle) keeps a pool of numeric factors, each
// with its own stream.  A factor+solve request takes an idle factor of its
// pattern (or a new one, if the predicted bytes fit the budget after
// evicting idle factors of other patterns, least recently used first),
// refactors it with the request's values and solves on that factor's stream;
// once it completes without a failed pivot, the factor becomes the
// pattern's current factor, which solve-only requests use (queued on its
// stream, so they never race for its work vectors).  Up to max_inflight
// requests are on the device at once, on different streams, so their
// kernels overlap; requests that arrive meanwhile wait in a queue and are
// admitted, in arrival order where they fit, as slots and memory free up.
// Completion is signalled from the stream by a host function, so the
// scheduler thread never blocks on the device.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/spchol.h"
#include "runtime.hpp"

namespace spc {
int32_t numeric_create(spc_symbolic* sym, spc_numeric** out);
int64_t numeric_bytes(const spc_symbolic* sym);
}  // namespace spc

using namespace spc;

namespace {

typedef std::chrono::steady_clock Clock;

struct Fact {
    spc_numeric* num = nullptr;
    hipStream_t st = nullptr;
    int32_t* hstatus = nullptr;  // pinned copy of the factor's status word
    int32_t pattern = -1;
    int refs = 0;                // admitted requests that use it
    bool current = false;        // the pattern's current factor
    uint64_t last_use = 0;
    int64_t bytes = 0;
};

struct Pattern {
    spc_symbolic* sym = nullptr;
    int64_t bytes = 0;           // predicted device bytes of one factor with its work
    int64_t plan_bytes = 0;      // the symbolic handle's device plan, made with the first
                                 // factor and kept until the handle is freed
    bool plan_charged = false;   // plan_bytes counted in the server's bytes
    Fact* current = nullptr;
    std::vector<Fact*> pool;
};

struct Req {
    int64_t ticket = 0;
    spc_request r{};
    Clock::time_point t_submit, t_admit, t_done;
    Fact* f = nullptr;
    int32_t status = 0;
    bool admitted = false;
    bool done = false;                   // retired: the waiter may read it
    std::atomic<bool> dev_done{false};   // set by the stream's host function
    struct spc_server* srv = nullptr;
    hipEvent_t ready = nullptr;          // recorded on the caller's stream at submission
};

}  // namespace

struct spc_server {
    spc_server_options opt{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;       // scheduler: new work or completions
    std::condition_variable done_cv;  // waiters
    std::vector<Pattern> patterns;
    std::deque<Req*> queue;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    std::vector<Req*> running;        // admitted and launched
    std::vector<Req*> finished;       // completed, not yet retired
    int64_t next_ticket = 1;
    int inflight = 0;
    int64_t bytes = 0;
    uint64_t clock = 0;
    spc_server_stats stats{};
    bool stop = false;
    std::thread worker;
};

namespace {

// Host function at the end of a request's stream work.  It takes no lock
// and makes no HIP call: it stamps the time, raises the request's flag and
// wakes the scheduler (which also polls, so a missed wake-up costs at most
// one poll interval).
void on_done(void* p) {
    Req* q = (Req*)p;
    // once dev_done is set the scheduler may retire the request and a waiter
    // may free it: take the server pointer first and touch q no more after
    spc_server* srv = q->srv;
    q->t_done = Clock::now();
    q->dev_done.store(true, std::memory_order_release);
    srv->cv.notify_all();
}

void destroy_fact(spc_server* s, Fact* f) {
    if (f->st) (void)hipStreamSynchronize(f->st);
    spc_numeric_free(f->num);
    if (f->st) (void)hipStreamDestroy(f->st);
    if (f->hstatus) (void)hipHostFree(f->hstatus);
    s->bytes -= f->bytes;
    delete f;
}

// Frees idle factors (no admitted request uses them), least recently used
// first, until `need` more bytes fit.  Called with mu held; an idle factor's
// stream has finished, so the frees do not wait on the device.
bool make_room(spc_server* s, int64_t need) {
    while (s->bytes + need > s->opt.mem_budget_bytes) {
        Fact* victim = nullptr;
        for (Pattern& p : s->patterns)
            for (Fact* f : p.pool)
                if (f->refs == 0 && (!victim || f->last_use < victim->last_use)) victim = f;
        if (!victim) return false;
        Pattern& p = s->patterns[victim->pattern];
        for (size_t i = 0; i < p.pool.size(); ++i)
            if (p.pool[i] == victim) {
                p.pool.erase(p.pool.begin() + (long)i);
                break;
            }
        if (p.current == victim) p.current = nullptr;
        destroy_fact(s, victim);
        s->stats.evictions++;
    }
    return true;
}

int32_t new_fact(spc_server* s, int32_t pat, Fact** out) {
    Pattern& p = s->patterns[pat];
    Fact* f = new Fact();
    f->pattern = pat;
    f->bytes = p.bytes;
    int32_t st = numeric_create(p.sym, &f->num);
    if (st == OK) st = ensure_solve_work(f->num, s->opt.max_nrhs);
    if (st == OK && hipStreamCreateWithFlags(&f->st, hipStreamNonBlocking) != hipSuccess)
        st = ERR_HIP;
    if (st == OK && hipHostMalloc(&f->hstatus, 2 * sizeof(int32_t), hipHostMallocDefault) !=
                        hipSuccess)
        st = ERR_OOM;
    if (st != OK) {
        if (f->num) spc_numeric_free(f->num);
        if (f->st) (void)hipStreamDestroy(f->st);
        if (f->hstatus) (void)hipHostFree(f->hstatus);
        delete f;
        return st;
    }
    s->bytes += f->bytes;
    if (!p.plan_charged) {
        s->bytes += p.plan_bytes;
        p.plan_charged = true;
    }
    p.pool.push_back(f);
    *out = f;
    return OK;
}

// Enqueues an admitted request on its factor's stream.  Called without mu.
int32_t launch(Req* q) {
    Fact* f = q->f;
    spc_numeric* num = f->num;
    const spc_request& r = q->r;
    int32_t st = OK;
    // the caller's work on values, b and x (up to submission) comes first
    if (q->ready && hipStreamWaitEvent(f->st, q->ready, 0) != hipSuccess) st = ERR_HIP;
    if (st == OK && r.kind == 0) {
        st = run_factor(num, r.values, f->st);
        if (st == OK &&
            hipMemcpyAsync(f->hstatus, num->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost,
                           f->st) != hipSuccess)
            st = ERR_HIP;
    }
    if (st == OK) st = run_solve(num, r.nrhs, r.b, r.ldb, r.x, r.ldx, f->st);
    if (st == OK && hipLaunchHostFunc(f->st, on_done, q) != hipSuccess) st = ERR_HIP;
    return st;
}

// Admission pass over the queue in arrival order.  Called with mu held;
// returns the requests to launch.
void admit(spc_server* s, std::vector<Req*>& go) {
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (s->inflight >= s->opt.max_inflight) break;
        Req* q = *it;
        Pattern& p = s->patterns[q->r.pattern];
        Fact* f = nullptr;
        if (q->r.kind == 1) {
            if (!p.current) {
                // a factor request of this pattern ahead in the queue or in flight may provide it
                bool pending = false;
                for (Req* o : s->queue)
                    if (o == q) break;
                    else if (o->r.pattern == q->r.pattern && o->r.kind == 0) pending = true;
                for (Fact* g : p.pool) pending |= g->refs > 0;
                if (pending) {
                    ++it;
                    continue;
                }
                q->status = ERR_NOT_FACTORED;
                q->t_done = Clock::now();
                s->finished.push_back(q);
                it = s->queue.erase(it);
                continue;
            }
            f = p.current;
        } else {
            for (Fact* g : p.pool)
                if (g->refs == 0 && !g->current) f = g;
            if (!f) {
                const int64_t need = p.bytes + (p.plan_charged ? 0 : p.plan_bytes);
                if (p.bytes + p.plan_bytes > s->opt.mem_budget_bytes) {
                    q->status = ERR_OOM;
                    q->t_done = Clock::now();
                    s->finished.push_back(q);
                    s->stats.rejected++;
                    it = s->queue.erase(it);
                    continue;
                }
                if (!make_room(s, need) || new_fact(s, q->r.pattern, &f) != OK) {
                    if (s->inflight == 0) {  // nothing will free memory: give up on it
                        q->status = ERR_OOM;
                        q->t_done = Clock::now();
                        s->finished.push_back(q);
                        s->stats.rejected++;
                        it = s->queue.erase(it);
                    } else {
                        ++it;  // wait for memory to free up
                    }
                    continue;
                }
            }
        }
        f->refs++;
        f->last_use = ++s->clock;
        q->f = f;
        q->admitted = true;
        q->t_admit = Clock::now();
        s->inflight++;
        if (s->inflight > s->stats.peak_inflight) s->stats.peak_inflight = s->inflight;
        if (s->bytes > s->stats.peak_bytes) s->stats.peak_bytes = s->bytes;
        go.push_back(q);
        it = s->queue.erase(it);
    }
}

// Retires completed requests.  Called with mu held.
void retire(spc_server* s) {
    for (size_t i = 0; i < s->running.size();) {
        Req* q = s->running[i];
        if (q->dev_done.load(std::memory_order_acquire)) {
            s->finished.push_back(q);
            s->running[i] = s->running.back();
            s->running.pop_back();
        } else {
            ++i;
        }
    }
    for (Req* q : s->finished) {
        if (q->ready) {  // its wait is behind it on the stream (or never enqueued)
            (void)hipEventDestroy(q->ready);
            q->ready = nullptr;
        }
        if (q->f) {
            Fact* f = q->f;
            if (q->r.kind == 0) {
                const int32_t v = f->hstatus[0];
                if (q->status == OK) q->status = (v == INT32_MAX) ? 0 : v;
                if (q->status == OK) {
                    Pattern& p = s->patterns[f->pattern];
                    if (p.current) p.current->current = false;
                    p.current = f;
                    f->current = true;
                }
            }
            f->refs--;
            s->inflight--;
        }
        q->done = true;
        s->stats.completed++;
    }
    s->finished.clear();
    s->done_cv.notify_all();
}

void worker_main(spc_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        retire(s);
        std::vector<Req*> go;
        admit(s, go);
        retire(s);  // requests admission completed at once (errors)
        if (!go.empty()) {
            lock.unlock();
            std::vector<std::pair<Req*, int32_t>> failed;
            for (Req* q : go) {
                const int32_t st = launch(q);
                if (st != OK) failed.push_back({q, st});
            }
            for (auto& e : failed)  // part of the work may be on its stream
                (void)hipStreamSynchronize(e.first->f->st);
            lock.lock();
            for (Req* q : go) {
                bool bad = false;
                for (auto& e : failed)
                    if (e.first == q) {
                        q->status = e.second;
                        q->t_done = Clock::now();
                        s->finished.push_back(q);
                        bad = true;
                    }
                if (!bad) s->running.push_back(q);
            }
            continue;
        }
        if (s->stop && s->queue.empty() && s->inflight == 0) break;
        s->cv.wait_for(lock, std::chrono::milliseconds(2));
    }
}

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

extern "C" {

void spc_server_default_options(spc_server_options* opt) {
    if (!opt) return;
    opt->max_inflight = 8;
    opt->max_nrhs = 64;
    opt->mem_budget_bytes = 0;
}

spc_status spc_server_create(const spc_server_options* opt, spc_server** out) {
    if (!out) return SPC_ERR_ARG;
    *out = nullptr;
    spc_server_options o;
    spc_server_default_options(&o);
    if (opt) o = *opt;
    if (o.max_inflight < 1 || o.max_inflight > 64 || o.max_nrhs < 1 || o.mem_budget_bytes < 0)
        return SPC_ERR_ARG;
    spc_server* s = new (std::nothrow) spc_server();
    if (!s) return SPC_ERR_OOM;
    // hipFree(nullptr) creates the device context if nothing has yet
    if (hipGetDevice(&s->device) != hipSuccess || hipSetDevice(s->device) != hipSuccess ||
        hipFree(nullptr) != hipSuccess) {
        delete s;
        return SPC_ERR_HIP;
    }
    if (o.mem_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return SPC_ERR_HIP;
        }
        o.mem_budget_bytes = (int64_t)(0.8 * (double)free_b);
    }
    s->opt = o;
    s->stats.budget_bytes = o.mem_budget_bytes;
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        delete s;
        return SPC_ERR_OOM;
    }
    *out = s;
    return SPC_OK;
}

spc_status spc_server_add_pattern(spc_server* s, spc_symbolic* sym, int32_t* pattern) {
    if (!s || !sym || !pattern) return SPC_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    Pattern p;
    p.sym = sym;
    const Symbolic& S = sym->S;
    const size_t elem = S.opt.precision == 1 ? sizeof(float) : sizeof(double);
    p.bytes = numeric_bytes(sym) +
              (int64_t)elem * solve_work_elems_per_rhs(S) * (int64_t)s->opt.max_nrhs +
              4 * (tail_state_words(S) + split_state_words(S));
    p.plan_bytes = (int64_t)sym->plan_bytes_estimate;
    {
        // the pattern's device plan is made now, on the server's device, so
        // that its first request does not wait for it
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(s->device) != hipSuccess)
            return SPC_ERR_HIP;
        DevicePlan* plan = nullptr;
        const int32_t st = get_plan(sym, &plan);
        (void)hipSetDevice(cur);
        if (st != OK) return st;
    }
    {
        // the server keeps the handle referenced until spc_server_destroy
        std::lock_guard<std::mutex> sl(sym->mu);
        sym->refs++;
    }
    s->patterns.push_back(p);
    *pattern = (int32_t)s->patterns.size() - 1;
    return SPC_OK;
}

spc_status spc_server_submit(spc_server* s, const spc_request* r, int64_t* ticket) {
    if (!s || !r || !ticket) return SPC_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    if (r->pattern < 0 || r->pattern >= (int32_t)s->patterns.size()) return SPC_ERR_ARG;
    if (r->kind != 0 && r->kind != 1) return SPC_ERR_ARG;
    const int64_t n = s->patterns[r->pattern].sym->S.n;
    const int64_t nnz = s->patterns[r->pattern].sym->S.nnz_a;
    if (r->nrhs < 0 || r->nrhs > s->opt.max_nrhs) return SPC_ERR_ARG;
    if (r->kind == 0 && nnz > 0 && !r->values) return SPC_ERR_ARG;
    if (r->nrhs > 0 && n > 0 && (!r->b || !r->x || r->ldb < n || r->ldx < n)) return SPC_ERR_ARG;
    std::unique_ptr<Req> q(new (std::nothrow) Req());
    if (!q) return SPC_ERR_OOM;
    // order the request after the caller's stream work up to this call
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) {
        q->ready = nullptr;
        return SPC_ERR_HIP;
    }
    if (hipEventRecord(q->ready, (hipStream_t)r->stream) != hipSuccess) {
        (void)hipEventDestroy(q->ready);
        return SPC_ERR_HIP;
    }
    q->ticket = s->next_ticket++;
    q->r = *r;
    q->srv = s;
    q->t_submit = Clock::now();
    *ticket = q->ticket;
    s->queue.push_back(q.get());
    s->reqs[q->ticket] = std::move(q);
    s->stats.submitted++;
    s->cv.notify_all();
    return SPC_OK;
}

spc_status spc_server_wait(spc_server* s, int64_t ticket, spc_request_result* out) {
    if (!s) return SPC_ERR_ARG;
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SPC_ERR_ARG;
    Req* q = it->second.get();
    s->done_cv.wait(lock, [q] { return q->done; });
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->status = q->status;
        out->queue_ms = q->admitted ? ms_between(q->t_submit, q->t_admit) : 0.0;
        out->latency_ms = ms_between(q->t_submit, q->t_done);
    }
    s->reqs.erase(it);
    return SPC_OK;
}

spc_status spc_server_stats_get(spc_server* s, spc_server_stats* out) {
    if (!s || !out) return SPC_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    out->bytes_in_use = s->bytes;
    out->resident_factors = 0;
    for (const Pattern& p : s->patterns) out->resident_factors += (int32_t)p.pool.size();
    return SPC_OK;
}

spc_status spc_server_destroy(spc_server* s) {
    if (!s) return SPC_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (Pattern& p : s->patterns) {
        for (Fact* f : p.pool) destroy_fact(s, f);
        std::lock_guard<std::mutex> sl(p.sym->mu);
        p.sym->refs--;
    }
    delete s;
    return SPC_OK;
}

}  // extern "C"
