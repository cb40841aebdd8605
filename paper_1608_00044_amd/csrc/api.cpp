// C ABI of the supernodal Cholesky library (declared in include/spchol.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/spchol.h"
#include "runtime.hpp"

namespace spc {
int32_t configure_kernels();
}

using namespace spc;

namespace {

size_t real_size(int32_t prec) { return prec == 1 ? sizeof(float) : sizeof(double); }

// Device bytes of one numeric factor: supernode blocks and diagonal-block
// inverses in the factor's type, the FP64 copy of A kept for refinement
// (full CSR: 8-byte value, 4-byte column and 8-byte source index per entry,
// plus row pointers), task-queue counters, status words.
int64_t factor_bytes(const spc_symbolic* sym, int32_t prec) {
    const Symbolic& S = sym->S;
    const int64_t nnzf = 2 * S.nnz_a;  // bound: diagonal entries appear once
    int64_t b = (int64_t)((S.arena + inverse_blocks_elems(S)) * real_size(prec));
    b += nnzf * 20 + (S.n + 1) * 8;
    if (S.opt.sched == 2) b += 4 * (3 * S.nsup + 4);
    if (S.opt.deterministic) b += sym->det_scratch * real_size(prec);
    return b + 512;
}

// Frees whatever the numeric object holds (any member may still be null).
void release_numeric(spc_numeric* num) {
    if (num->fb) spc_numeric_free(num->fb);
    (void)hipFree(num->fb_values);
    (void)hipFree(num->arena);
    (void)hipFree(num->status_dev);
    (void)hipFree(num->dinv);
    (void)hipFree(num->sched_state);
    (void)hipFree(num->det_scratch);
    (void)hipFree(num->task_log);
    drop_solve_graphs(num);
    if (num->factor_exec) (void)hipGraphExecDestroy(num->factor_exec);
    if (num->factor_graph) (void)hipGraphDestroy(num->factor_graph);
    if (num->capture) (void)hipStreamDestroy(num->capture);
    (void)hipFree(num->work);
    free_refine(num);
    for (hipEvent_t e : num->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : num->sync_ev) (void)hipEventDestroy(e);
    if (num->bulk) {
        (void)hipStreamSynchronize(num->bulk);
        (void)hipStreamDestroy(num->bulk);
    }
}

template <class Run>
spc_status analyze_checked(const spc_options* opt, spc_symbolic** out, Run run) {
    if (!out) return SPC_ERR_ARG;
    *out = nullptr;
    spc_options o;
    spc_default_options(&o);
    if (opt) o = *opt;
    if (o.sn_cap < 1 || o.sn_cap > kMaxWidth) return SPC_ERR_ARG;
    if (o.sched < 0 || o.sched > 2) return SPC_ERR_ARG;
    if (o.spin_limit < 0) return SPC_ERR_ARG;
    if (!(o.amalg_ratio >= 0.0 && o.amalg_ratio <= 1.0)) return SPC_ERR_ARG;
    if (o.mem_budget_bytes < 0) return SPC_ERR_ARG;
    if (o.precision != 0 && o.precision != 1) return SPC_ERR_ARG;
    if (o.threads < 0) return SPC_ERR_ARG;
    if (o.small_w < -1 || o.small_w > kSmallW || o.small_r < 0 || o.small_r > kSmallR)
        return SPC_ERR_ARG;
    if (o.deterministic != 0 && o.deterministic != 1) return SPC_ERR_ARG;
    if (o.deterministic && o.sched == 2) return SPC_ERR_ARG;  // the queue's order is dynamic
    if (o.workers < 0) return SPC_ERR_ARG;
    if (o.solve_tail != 0 && o.solve_tail != 1) return SPC_ERR_ARG;
    if (o.upd_chunk != 0 && o.upd_chunk != 8 && o.upd_chunk != 16 && o.upd_chunk != 32)
        return SPC_ERR_ARG;
    spc_symbolic* h = new (std::nothrow) spc_symbolic();
    if (!h) return SPC_ERR_OOM;
    Options so;
    so.sn_cap = o.sn_cap;
    so.amalg_ratio = o.amalg_ratio;
    so.sched = o.sched;
    so.spin_limit = o.spin_limit;
    so.debug_flags = o.debug_flags;
    so.precision = o.precision;
    so.small_w = o.small_w == 0 ? kSmallW : (o.small_w < 0 ? 0 : o.small_w);
    so.small_r = o.small_r == 0 ? kSmallR : o.small_r;
    so.deterministic = o.deterministic;
    so.workers = o.workers;
    so.solve_tail = o.solve_tail;
    so.upd_chunk = o.upd_chunk == 0 ? 16 : o.upd_chunk;
    int32_t st;
    try {
        st = run(so, o.threads, &h->S);
        if (st == OK) h->plan_bytes_estimate = plan_bytes(h->S, &h->det_scratch);
    } catch (const std::bad_alloc&) {
        st = SPC_ERR_OOM;
    }
    if (st != OK) {
        delete h;
        return st;
    }
    h->budget = o.mem_budget_bytes;
    *out = h;
    return SPC_OK;
}

}  // namespace

extern "C" {

void spc_default_options(spc_options* opt) {
    if (!opt) return;
    opt->sn_cap = 150;
    opt->sched = 0;
    opt->amalg_ratio = 0.0;
    opt->mem_budget_bytes = 0;
    opt->spin_limit = 0;
    opt->debug_flags = 0;
    opt->precision = 0;
    opt->threads = 0;
    opt->small_w = 0;
    opt->small_r = 0;
    opt->deterministic = 1;
    opt->workers = 0;
    opt->solve_tail = 0;
    opt->upd_chunk = 0;
}

const char* spc_status_string(spc_status st) {
    if (st > 0) return "factorization stopped: a pivot was not positive";
    switch (st) {
        case SPC_OK: return "success";
        case SPC_ERR_ARG: return "invalid argument";
        case SPC_ERR_PATTERN: return "malformed lower-triangular CSC pattern";
        case SPC_ERR_OOM: return "out of memory or over the memory budget";
        case SPC_ERR_HIP: return "HIP runtime error";
        case SPC_ERR_NOT_FACTORED: return "no completed factorization";
        case SPC_ERR_NOT_CONVERGED: return "iterative refinement did not converge";
        case SPC_ERR_TIMEOUT: return "device wait exceeded its bound";
        case SPC_ERR_BUSY: return "symbolic handle is still referenced";
        case SPC_ERR_TOO_LARGE: return "the solve's work does not fit the static scratch";
        default: return "unknown status";
    }
}

spc_status spc_analyze(int64_t n, const int64_t* colptr, const int32_t* rowind,
                       const int32_t* perm, const spc_options* opt, spc_symbolic** out) {
    return analyze_checked(opt, out, [&](const Options& so, int, Symbolic* S) {
        return analyze(n, colptr, rowind, perm, so, S);
    });
}

spc_status spc_analyze_batch(int32_t count, const int64_t* n, const int64_t* const* colptr,
                             const int32_t* const* rowind, const int32_t* const* perm,
                             const spc_options* opt, spc_symbolic** out) {
    if (!out) return SPC_ERR_ARG;
    *out = nullptr;
    if (count < 0 || (count > 0 && (!n || !colptr || !rowind))) return SPC_ERR_ARG;
    int64_t rows = 0;
    for (int32_t k = 0; k < count; ++k) {
        if (n[k] < 0 || n[k] > INT32_MAX - 1 - rows) return SPC_ERR_ARG;
        rows += n[k];
    }
    return analyze_checked(opt, out, [&](const Options& so, int threads, Symbolic* S) {
        if (threads == 0) {
            const unsigned hw = std::thread::hardware_concurrency();
            threads = (int)std::min<unsigned>(16, std::max(1u, hw));
        }
        return analyze_batch(count, n, colptr, rowind, perm, so, threads, S);
    });
}

spc_status spc_symbolic_info_get(const spc_symbolic* sym, spc_symbolic_info* info) {
    if (!sym || !info) return SPC_ERR_ARG;
    const Symbolic& S = sym->S;
    std::memset(info, 0, sizeof(*info));
    info->n = S.n;
    info->nnz_a = S.nnz_a;
    info->nnz_l = S.nnz_l;
    info->nnz_stored = S.nnz_stored;
    info->nsup = S.nsup;
    info->nlevels = (int64_t)S.level_ptr.size() - 1;
    info->npairs = (int64_t)S.pairs.size();
    info->nrel = (int64_t)S.rel.size();
    info->factor_bytes = factor_bytes(sym, S.opt.precision);
    info->plan_bytes = (int64_t)sym->plan_bytes_estimate;
    info->flops = S.flops;
    info->flops_stored = S.flops_stored;
    info->max_width = S.max_w;
    info->max_below = S.max_r;
    info->nbatch = (int64_t)S.batch_ptr.size() - 1;
    info->solve_bytes_per_rhs = solve_work_elems_per_rhs(S) * (int64_t)real_size(S.opt.precision);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1, l0 = tail_start(S);
    info->tail_levels = nl > l0 ? nl - l0 : 0;
    info->tail_supernodes = nl > l0 ? S.level_ptr[nl] - S.level_ptr[l0] : 0;
    return SPC_OK;
}

spc_status spc_symbolic_export(const spc_symbolic* sym, int32_t* parent, int32_t* colcount,
                               int32_t* sn_ptr, int32_t* sn_parent) {
    if (!sym) return SPC_ERR_ARG;
    const Symbolic& S = sym->S;
    if (parent && S.n) std::memcpy(parent, S.parent.data(), sizeof(int32_t) * S.n);
    if (colcount && S.n) std::memcpy(colcount, S.colcount.data(), sizeof(int32_t) * S.n);
    if (sn_ptr) std::memcpy(sn_ptr, S.sn_ptr.data(), sizeof(int32_t) * (S.nsup + 1));
    if (sn_parent && S.nsup) std::memcpy(sn_parent, S.sn_parent.data(), sizeof(int32_t) * S.nsup);
    return SPC_OK;
}

spc_status spc_symbolic_export_rows(const spc_symbolic* sym, int64_t* rowptr, int32_t* rows) {
    if (!sym) return SPC_ERR_ARG;
    const Symbolic& S = sym->S;
    if (rowptr) std::memcpy(rowptr, S.rowptr.data(), sizeof(int64_t) * (S.nsup + 1));
    if (rows && !S.rows.empty()) std::memcpy(rows, S.rows.data(), sizeof(int32_t) * S.rows.size());
    return SPC_OK;
}

spc_status spc_symbolic_export_pairs(const spc_symbolic* sym, int32_t* src, int32_t* tgt,
                                     int32_t* seg, int64_t* rel_off, int32_t* rel) {
    if (!sym) return SPC_ERR_ARG;
    const Symbolic& S = sym->S;
    for (size_t p = 0; p < S.pairs.size(); ++p) {
        if (src) src[p] = S.pairs[p].src;
        if (tgt) tgt[p] = S.pairs[p].tgt;
        if (seg) { seg[2 * p] = S.pairs[p].seg_begin; seg[2 * p + 1] = S.pairs[p].seg_end; }
        if (rel_off) rel_off[p] = S.pairs[p].rel_off;
    }
    if (rel && !S.rel.empty()) std::memcpy(rel, S.rel.data(), sizeof(int32_t) * S.rel.size());
    return SPC_OK;
}

spc_status spc_symbolic_export_tasks(const spc_symbolic* sym, int32_t workers, int64_t* ntasks,
                                     int32_t* tasks, int32_t* cnt0) {
    if (!sym || !ntasks || workers <= 0) return SPC_ERR_ARG;
    std::vector<Task> order;
    std::vector<int32_t> c0, rb_base;
    const int32_t st = build_task_order(sym->S, workers, order, c0, rb_base);
    if (st != OK) return st;
    *ntasks = (int64_t)order.size();
    if (tasks)
        for (size_t i = 0; i < order.size(); ++i) {
            tasks[4 * i] = order[i].kind;
            tasks[4 * i + 1] = order[i].s;
            tasks[4 * i + 2] = order[i].a;
            tasks[4 * i + 3] = order[i].b;
        }
    if (cnt0 && !c0.empty()) std::memcpy(cnt0, c0.data(), sizeof(int32_t) * c0.size());
    return SPC_OK;
}

spc_status spc_symbolic_free(spc_symbolic* sym) {
    if (!sym) return SPC_OK;
    {
        std::lock_guard<std::mutex> lock(sym->mu);
        if (sym->refs > 0) return SPC_ERR_BUSY;
    }
    for (DevicePlan* p : sym->plans) free_plan(p);
    delete sym;
    return SPC_OK;
}

// A numeric object of sym whose factor has type prec (0 FP64, 1 FP32).
static spc_status alloc_numeric(spc_symbolic* sym, int32_t prec, spc_numeric** out) {
    int32_t st = configure_kernels();
    if (st != OK) return st;
    const Symbolic& S = sym->S;
    if (sym->budget > 0 &&
        factor_bytes(sym, prec) + (int64_t)sym->plan_bytes_estimate > sym->budget)
        return SPC_ERR_OOM;
    DevicePlan* plan = nullptr;
    st = get_plan(sym, &plan);
    if (st != OK) return st;
    spc_numeric* num = new (std::nothrow) spc_numeric();
    if (!num) return SPC_ERR_OOM;
    num->sym = sym;
    num->plan = plan;
    num->device = plan->device;
    num->prec = prec;
    // the lookahead's second stream reorders contributions: the deterministic
    // order runs level by level on one stream
    num->sched = (S.opt.sched == 1 && S.opt.deterministic) ? 0 : S.opt.sched;
    const size_t rs = real_size(prec);
    bool ok = hipMalloc(&num->arena, rs * (size_t)(S.arena > 0 ? S.arena : 1)) == hipSuccess &&
              hipMalloc(&num->status_dev, 256) == hipSuccess &&
              hipMalloc(&num->dinv, rs * (size_t)(plan->inv_elems > 0 ? plan->inv_elems : 1)) ==
                  hipSuccess;
    if (ok && num->sched == 2) {
        const size_t ints = 2 * (size_t)S.nsup + (size_t)plan->nrowblk + 4;
        ok = hipMalloc(&num->sched_state, ints * sizeof(int32_t)) == hipSuccess;
        num->spin_limit = S.opt.spin_limit > 0 ? S.opt.spin_limit : (int64_t)10000000;
        if (ok && (S.opt.debug_flags & 2))
            ok = hipMalloc(&num->task_log, 2 * sizeof(int32_t) *
                                               (size_t)std::max<int64_t>(plan->ntasks, 1)) ==
                 hipSuccess;
    }
    if (ok && S.opt.deterministic && num->sched != 2) {
        num->det = true;
        ok = hipMalloc(&num->det_scratch, rs * (size_t)std::max<int64_t>(plan->det_scratch, 1)) ==
             hipSuccess;
    }
    if (!ok) {
        release_numeric(num);
        delete num;
        return SPC_ERR_OOM;
    }
    if (num->sched == 1 &&
        hipStreamCreateWithFlags(&num->bulk, hipStreamNonBlocking) != hipSuccess) {
        release_numeric(num);
        delete num;
        return SPC_ERR_HIP;
    }
    {
        std::lock_guard<std::mutex> lock(sym->mu);
        sym->refs++;
    }
    *out = num;
    return SPC_OK;
}

// Factorization plus the FP64 copy of A that refinement reads.
static spc_status factor_and_keep(spc_numeric* num, const double* values_dev, hipStream_t st) {
    spc_status r = run_factor(num, values_dev, st);
    if (r != SPC_OK) return r;
    return load_refine_matrix(num, values_dev, st);
}

spc_status spc_factor(const spc_symbolic* csym, const double* values_dev, void* stream,
                      spc_numeric** out) {
    if (!csym || !out) return SPC_ERR_ARG;
    *out = nullptr;
    spc_symbolic* sym = const_cast<spc_symbolic*>(csym);
    if (sym->S.nnz_a > 0 && !values_dev) return SPC_ERR_ARG;
    spc_numeric* num = nullptr;
    spc_status st = alloc_numeric(sym, sym->S.opt.precision, &num);
    if (st != SPC_OK) return st;
    st = factor_and_keep(num, values_dev, (hipStream_t)stream);
    if (st != SPC_OK) {
        spc_numeric_free(num);
        return st;
    }
    *out = num;
    return SPC_OK;
}

spc_status spc_refactor(spc_numeric* num, const double* values_dev, void* stream) {
    if (!num) return SPC_ERR_ARG;
    if (num->sym->S.nnz_a > 0 && !values_dev) return SPC_ERR_ARG;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SPC_ERR_HIP;
    if (cur != num->device) return SPC_ERR_ARG;
    num->host_status = 0;
    return factor_and_keep(num, values_dev, (hipStream_t)stream);
}

spc_status spc_numeric_status(spc_numeric* num) {
    if (!num) return SPC_ERR_ARG;
    if (!num->factored) return SPC_ERR_NOT_FACTORED;
    if (hipStreamSynchronize(num->stream) != hipSuccess) return SPC_ERR_HIP;
    int32_t v = 0;
    if (hipMemcpy(&v, num->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return SPC_ERR_HIP;
    num->host_status = (v == INT32_MAX) ? 0 : v;
    if (num->sched_state) {
        const Symbolic& S = num->sym->S;
        int32_t err = 0;
        const size_t at = 2 * (size_t)S.nsup + (size_t)num->plan->nrowblk + 2;
        if (hipMemcpy(&err, num->sched_state + at, sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return SPC_ERR_HIP;
        if (err) num->host_status = SPC_ERR_TIMEOUT;
    }
    num->status_known = true;
    return num->host_status;
}

spc_status spc_solve(spc_numeric* num, int32_t nrhs, const double* b_dev, int64_t ldb,
                     double* x_dev, int64_t ldx, void* stream) {
    if (!num || nrhs < 0) return SPC_ERR_ARG;
    const int64_t n = num->sym->S.n;
    if (nrhs > 0 && n > 0 && (!b_dev || !x_dev || ldb < n || ldx < n)) return SPC_ERR_ARG;
    if (b_dev == x_dev && ldb != ldx) return SPC_ERR_ARG;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SPC_ERR_HIP;
    if (cur != num->device) return SPC_ERR_ARG;
    spc_status st = num->status_known ? num->host_status : spc_numeric_status(num);
    if (st != SPC_OK) return st;
    return run_solve(num, nrhs, b_dev, ldb, x_dev, ldx, (hipStream_t)stream);
}

spc_status spc_solve_refine(spc_numeric* num, int32_t nrhs, const double* b_dev, int64_t ldb,
                            double* x_dev, int64_t ldx, double tol, int32_t max_iter,
                            void* stream, int32_t* iters, double* berr) {
    if (!num || nrhs < 0 || max_iter < 0 || !(tol >= 0.0)) return SPC_ERR_ARG;
    const int64_t n = num->sym->S.n;
    if (nrhs > 0 && n > 0 && (!b_dev || !x_dev || ldb < n || ldx < n || b_dev == x_dev))
        return SPC_ERR_ARG;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SPC_ERR_HIP;
    if (cur != num->device) return SPC_ERR_ARG;
    spc_status st = num->status_known ? num->host_status : spc_numeric_status(num);
    if (st != SPC_OK) return st;
    return run_refine(num, nrhs, b_dev, ldb, x_dev, ldx, tol, max_iter, (hipStream_t)stream,
                      iters, berr);
}

spc_status spc_numeric_info_get(spc_numeric* num, spc_numeric_info* out) {
    if (!num || !out) return SPC_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    out->precision = num->prec;
    out->sched = num->sched;
    out->factor_bytes = factor_bytes(num->sym, num->prec);
    out->refine_fallbacks = num->refine_fallbacks;
    if (num->factored) {
        if (hipStreamSynchronize(num->stream) != hipSuccess) return SPC_ERR_HIP;
        int32_t v[2] = {0, 0};
        if (hipMemcpy(v, num->status_dev, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
            return SPC_ERR_HIP;
        out->fp64_blocks = v[1];
    }
    return SPC_OK;
}

spc_status spc_factor_export(spc_numeric* num, int64_t* Sp, int32_t* Si, double* Sx) {
    if (!num) return SPC_ERR_ARG;
    const Symbolic& S = num->sym->S;
    if (Sp || Si) {
        int64_t q = 0;
        if (Sp) Sp[0] = 0;
        for (int64_t s = 0; s < S.nsup; ++s) {
            const int32_t w = S.width(s), m = S.nrows(s);
            const int32_t* R = S.rows.data() + S.rowptr[s];
            for (int32_t c = 0; c < w; ++c) {
                for (int32_t i = c; i < m; ++i) {
                    if (Si) Si[q] = R[i];
                    ++q;
                }
                if (Sp) Sp[S.sn_ptr[s] + c + 1] = q;
            }
        }
    }
    if (Sx) {
        if (!num->factored) return SPC_ERR_NOT_FACTORED;
        if (hipStreamSynchronize(num->stream) != hipSuccess) return SPC_ERR_HIP;
        std::vector<double> h((size_t)(S.arena > 0 ? S.arena : 1));
        if (S.arena > 0 && num->prec == 1) {
            std::vector<float> hf((size_t)S.arena);
            if (hipMemcpy(hf.data(), num->arena, sizeof(float) * S.arena,
                          hipMemcpyDeviceToHost) != hipSuccess)
                return SPC_ERR_HIP;
            for (int64_t k = 0; k < S.arena; ++k) h[(size_t)k] = (double)hf[(size_t)k];
        } else if (S.arena > 0 &&
                   hipMemcpy(h.data(), num->arena, sizeof(double) * S.arena,
                             hipMemcpyDeviceToHost) != hipSuccess) {
            return SPC_ERR_HIP;
        }
        int64_t q = 0;
        for (int64_t s = 0; s < S.nsup; ++s) {
            const int32_t w = S.width(s), m = S.nrows(s), ld = S.ld[s];
            const double* B = h.data() + S.off[s];
            for (int32_t c = 0; c < w; ++c)
                for (int32_t i = c; i < m; ++i) Sx[q++] = B[i + (int64_t)c * ld];
        }
    }
    return SPC_OK;
}

spc_status spc_numeric_task_log(spc_numeric* num, int64_t* ntasks, int32_t* tasks,
                                int32_t* stamps) {
    if (!num || !ntasks) return SPC_ERR_ARG;
    if (!num->task_log) return SPC_ERR_ARG;
    const std::vector<Task>& T = num->plan->host_tasks;
    *ntasks = (int64_t)T.size();
    if (tasks)
        for (size_t i = 0; i < T.size(); ++i) {
            tasks[4 * i] = T[i].kind;
            tasks[4 * i + 1] = T[i].s;
            tasks[4 * i + 2] = T[i].a;
            tasks[4 * i + 3] = T[i].b;
        }
    if (stamps) {
        if (!num->factored) return SPC_ERR_NOT_FACTORED;
        if (hipStreamSynchronize(num->stream) != hipSuccess) return SPC_ERR_HIP;
        if (!T.empty() && hipMemcpy(stamps, num->task_log, 2 * sizeof(int32_t) * T.size(),
                                    hipMemcpyDeviceToHost) != hipSuccess)
            return SPC_ERR_HIP;
    }
    return SPC_OK;
}

spc_status spc_numeric_set_timing(spc_numeric* num, int32_t enable) {
    if (!num) return SPC_ERR_ARG;
    num->timing = enable != 0;
    return SPC_OK;
}

spc_status spc_numeric_get_timing(spc_numeric* num, spc_kernel_times* out) {
    if (!num || !out) return SPC_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    if (num->marks.empty()) return num->timing ? SPC_OK : SPC_ERR_ARG;
    if (hipStreamSynchronize(num->stream) != hipSuccess) return SPC_ERR_HIP;
    for (const auto& m : num->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, num->events[m.a], num->events[m.b]) != hipSuccess)
            return SPC_ERR_HIP;
        if (m.cls >= 0 && m.cls < 6) {
            out->ms[m.cls] += ms;
            out->launches[m.cls] += 1;
        }
    }
    float tot = 0.f;
    for (const auto& m : num->marks) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, num->events[num->marks.front().a], num->events[m.b]) !=
            hipSuccess)
            return SPC_ERR_HIP;
        tot = t > tot ? t : tot;
    }
    out->total_ms = tot;
    return SPC_OK;
}

void spc_numeric_free(spc_numeric* num) {
    if (!num) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(num->device);
    if (num->stream) (void)hipStreamSynchronize(num->stream);
    else (void)hipDeviceSynchronize();
    release_numeric(num);
    (void)hipSetDevice(cur);
    {
        std::lock_guard<std::mutex> lock(num->sym->mu);
        num->sym->refs--;
    }
    delete num;
}

}  // extern "C"

namespace spc {
// Numeric object of sym without a factorization (the request server's pool).
int32_t numeric_create(spc_symbolic* sym, spc_numeric** out) {
    return alloc_numeric(sym, sym->S.opt.precision, out);
}
int32_t numeric_create_prec(spc_symbolic* sym, int32_t prec, spc_numeric** out) {
    return alloc_numeric(sym, prec, out);
}
int64_t numeric_bytes(const spc_symbolic* sym) { return factor_bytes(sym, sym->S.opt.precision); }
}  // namespace spc
