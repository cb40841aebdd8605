// Task order for the device task-queue schedule.
//
// The factorization is a DAG of the paper's tasks (Section III-A): F(s)
// factors supernode s (diagonal block), T(s, b) solves row block b of its
// panel (both are the F task of the paper, split for parallelism), U(s, i, j)
// computes one 64 x 64 tile of its update and scatter-adds it into the target
// supernodes (the U and A tasks).  Edges: F(s) -> T(s, b); T(s, i), T(s, j)
// -> U(s, i, j); U(s, i, j) -> F(t) for every target t of the tile's columns.
// F(t) may run once every tile that scatters into t is done (the paper's
// incoming-dependency counter, Section IV).
//
// The device workers take tasks in one fixed order by an atomic ticket and
// wait inside a task for its inputs.  Any topological order is deadlock free:
// the lowest unfinished ticket always has its inputs done.  The order chosen
// here is the start order of a list-scheduling simulation with `workers`
// identical workers, ready tasks picked by largest bottom level (longest
// remaining path, with per-task cost estimates), so the critical path runs
// first and the bulk work fills in around it.
#include <algorithm>
#include <cmath>
#include <queue>
#include <utility>

#include "runtime.hpp"

namespace spc {

int32_t build_task_order(const Symbolic& S, int workers, std::vector<Task>& order,
                         std::vector<int32_t>& cnt0, std::vector<int32_t>& rb_base) {
    const int64_t ns = S.nsup;
    std::vector<int32_t> nb((size_t)ns);
    std::vector<int64_t> tile_base((size_t)ns + 1, 0);
    rb_base.assign((size_t)ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
        nb[s] = (S.nbelow(s) + kTile - 1) / kTile;
        if (nb[s] > INT16_MAX) return ERR_ARG;  // block indices are stored in 16 bits
        rb_base[s + 1] = rb_base[s] + nb[s];
        tile_base[s + 1] = tile_base[s] + (int64_t)nb[s] * (nb[s] + 1) / 2;
    }
    const int64_t nrb = rb_base[ns], ntile = tile_base[ns];
    const int64_t N = ns + nrb + ntile;
    if (N >= INT32_MAX) return ERR_ARG;
    // distinct targets of every column block of every source
    std::vector<int64_t> cb_ptr((size_t)nrb + 1, 0);
    std::vector<int32_t> cb_tgt;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t r = S.nbelow(s);
        for (int32_t bj = 0; bj < nb[s]; ++bj) {
            const int32_t c0 = bj * kTile, c1 = std::min(r, c0 + kTile);
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                const Pair& pr = S.pairs[p];
                if (pr.seg_end > c0 && pr.seg_begin < c1) cb_tgt.push_back(pr.tgt);
            }
            cb_ptr[rb_base[s] + bj + 1] = (int64_t)cb_tgt.size();
        }
    }
    // F counters: tiles (s, i, j) touching t = (i >= j) rows of blocks j
    cnt0.assign((size_t)ns, 0);
    for (int64_t s = 0; s < ns; ++s)
        for (int32_t bj = 0; bj < nb[s]; ++bj) {
            const int32_t ntiles_col = nb[s] - bj;  // tiles (i, bj) with i >= bj
            for (int64_t q = cb_ptr[rb_base[s] + bj]; q < cb_ptr[rb_base[s] + bj + 1]; ++q)
                cnt0[cb_tgt[q]] += ntiles_col;
        }
    // costs (rough microseconds on one workgroup) and bottom levels
    auto cost_f = [&](int64_t s) { return 3.0 + 0.45 * S.width(s); };
    auto cost_t = [&](int64_t s) { return 2.0 + 0.1 * S.width(s); };
    auto cost_u = [&](int64_t s) { return 1.0 + 0.065 * S.width(s); };
    std::vector<float> bl((size_t)N, 0.f);
    std::vector<double> mcol;
    for (int64_t s = ns - 1; s >= 0; --s) {
        mcol.assign((size_t)nb[s], 0.0);
        for (int32_t bj = 0; bj < nb[s]; ++bj) {
            double m = 0.0;
            for (int64_t q = cb_ptr[rb_base[s] + bj]; q < cb_ptr[rb_base[s] + bj + 1]; ++q)
                m = std::max(m, (double)bl[cb_tgt[q]]);
            mcol[bj] = cost_u(s) + m;
        }
        for (int32_t i = 0; i < nb[s]; ++i)
            for (int32_t j = 0; j <= i; ++j)
                bl[ns + nrb + tile_base[s] + (int64_t)i * (i + 1) / 2 + j] = (float)mcol[j];
        double bf = 0.0, run = 0.0;
        for (int32_t b = 0; b < nb[s]; ++b) {
            run = std::max(run, mcol[b]);  // tiles (b, j <= b) and (i > b, b)
            const double bt = cost_t(s) + run;
            bl[ns + rb_base[s] + b] = (float)bt;
            bf = std::max(bf, bt);
        }
        bl[s] = (float)(cost_f(s) + bf);
    }
    // list-scheduling simulation
    std::vector<int32_t> indeg((size_t)N);
    for (int64_t s = 0; s < ns; ++s) {
        indeg[s] = cnt0[s];
        for (int32_t b = 0; b < nb[s]; ++b) indeg[ns + rb_base[s] + b] = 1;
        for (int32_t i = 0; i < nb[s]; ++i)
            for (int32_t j = 0; j <= i; ++j)
                indeg[ns + nrb + tile_base[s] + (int64_t)i * (i + 1) / 2 + j] = (i == j) ? 1 : 2;
    }
    // task id -> (kind, s, a, b)
    std::vector<int32_t> owner_rb((size_t)nrb), owner_tile;
    for (int64_t s = 0; s < ns; ++s)
        for (int32_t b = 0; b < nb[s]; ++b) owner_rb[rb_base[s] + b] = (int32_t)s;
    auto decode = [&](int64_t id, Task& t) {
        if (id < ns) { t = Task{(int32_t)id, 0, 0, kTaskF}; return; }
        if (id < ns + nrb) {
            const int64_t g = id - ns;
            const int32_t s = owner_rb[g];
            t = Task{s, (int16_t)(g - rb_base[s]), 0, kTaskT};
            return;
        }
        const int64_t g = id - ns - nrb;
        const int64_t s = std::upper_bound(tile_base.begin(), tile_base.end(), g) - tile_base.begin() - 1;
        const int64_t k = g - tile_base[s];
        int32_t i = (int32_t)((std::sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
        while ((int64_t)i * (i + 1) / 2 > k) --i;
        while ((int64_t)(i + 1) * (i + 2) / 2 <= k) ++i;
        const int32_t j = (int32_t)(k - (int64_t)i * (i + 1) / 2);
        t = Task{(int32_t)s, (int16_t)i, (int16_t)j, kTaskU};
    };
    auto cost_of = [&](const Task& t) {
        return t.kind == kTaskF ? cost_f(t.s) : (t.kind == kTaskT ? cost_t(t.s) : cost_u(t.s));
    };
    typedef std::pair<float, int32_t> RItem;  // (bottom level, -id) max-heap
    std::priority_queue<RItem> ready;
    typedef std::pair<double, int32_t> EItem;  // (finish time, id) min-heap
    std::priority_queue<EItem, std::vector<EItem>, std::greater<EItem>> running;
    for (int64_t s = 0; s < ns; ++s)
        if (indeg[s] == 0) ready.push(RItem(bl[s], (int32_t)-s));
    order.clear();
    order.reserve((size_t)N);
    double now = 0.0;
    int free_workers = std::max(1, workers);
    std::vector<int32_t> succ;
    while ((int64_t)order.size() < N) {
        while (free_workers > 0 && !ready.empty()) {
            const int32_t id = -ready.top().second;
            ready.pop();
            Task t;
            decode(id, t);
            order.push_back(t);
            running.push(EItem(now + cost_of(t), id));
            --free_workers;
        }
        if (running.empty()) return ERR_PATTERN;  // a cycle cannot happen in a valid plan
        now = running.top().first;
        while (!running.empty() && running.top().first <= now) {
            const int32_t id = running.top().second;
            running.pop();
            ++free_workers;
            Task t;
            decode(id, t);
            succ.clear();
            if (t.kind == kTaskF) {
                for (int32_t b = 0; b < nb[t.s]; ++b) succ.push_back((int32_t)(ns + rb_base[t.s] + b));
            } else if (t.kind == kTaskT) {
                const int32_t b = t.a, s = t.s;
                for (int32_t j = 0; j <= b; ++j)
                    succ.push_back((int32_t)(ns + nrb + tile_base[s] + (int64_t)b * (b + 1) / 2 + j));
                for (int32_t i = b + 1; i < nb[s]; ++i)
                    succ.push_back((int32_t)(ns + nrb + tile_base[s] + (int64_t)i * (i + 1) / 2 + b));
            } else {
                const int64_t cb = rb_base[t.s] + t.b;
                for (int64_t q = cb_ptr[cb]; q < cb_ptr[cb + 1]; ++q) succ.push_back(cb_tgt[q]);
            }
            for (int32_t v : succ)
                if (--indeg[v] == 0) ready.push(RItem(bl[v], -v));
        }
    }
    return OK;
}

}  // namespace spc
