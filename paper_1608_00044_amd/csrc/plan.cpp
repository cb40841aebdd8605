// Upload of the symbolic analysis to HBM: one allocation holding the
// supernode table, row lists, slot map, update pairs, relative indices and
// the per-level work lists the kernels walk.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "runtime.hpp"

namespace spc {

namespace {

struct Layout {
    size_t total = 0;
    template <class T>
    size_t add(size_t count) {
        size_t at = (total + 255) & ~size_t(255);
        total = at + count * sizeof(T);
        return at;
    }
};

struct PlanOffsets {
    size_t sn_first, sn_w, sn_ld, sn_off, inv_off, rowptr, rows, rowpair, slot, perm, pair_tgt,
        pair_seg, pair_rel, pair_excl, rel, level_sn, rowblk, tiles, tasks, cnt0, rb_base;
    size_t pair_src, pair_end, pair_thr, small_scr, app_t, app_p0, app_pairs;
    size_t rc_ptr, rc_slot, pb_off;
    size_t total;
};

// A pair is exclusive when no other source of its level updates its target.
std::vector<uint8_t> exclusive_pairs(const Symbolic& S) {
    const size_t np = S.pairs.size();
    std::vector<uint8_t> ex(np, 0);
    std::vector<int32_t> cnt((size_t)S.nsup, 0), stamp((size_t)S.nsup, -1);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    for (int32_t l = 0; l < nl; ++l) {
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                const int32_t t = S.pairs[p].tgt;
                if (stamp[t] != l) { stamp[t] = l; cnt[t] = 0; }
                cnt[t]++;
            }
        }
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p)
                ex[p] = cnt[S.pairs[p].tgt] == 1;
        }
    }
    return ex;
}

// Fixed contribution order for targets shared inside a level (the paper's
// aggregation of updates, Section III-B, in the order of non-decreasing
// (target, source) of Section III-D): within a level the small sources'
// contributions to a shared target come first, in increasing source order,
// added by one wave per target from a scratch copy of each source's update
// block; then the large sources' tiles, in increasing source order, each
// tile waiting until the target has received every tile of the sources
// before its own (a count of finished (tile, target) scatters, cumulative
// over the levels: pair_thr).
struct DetData {
    std::vector<int32_t> pair_src, pair_end, pair_thr, app_t, app_pairs;
    std::vector<int64_t> small_scr, app_p0;
    std::vector<uint8_t> level_ordered;
    std::vector<int64_t> app_ptr;
    int64_t scratch = 0;
    bool overflow = false;  // a count past the 32-bit thresholds
};

DetData build_det(const Symbolic& S, const std::vector<uint8_t>& ex) {
    DetData d;
    const size_t np = S.pairs.size();
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    d.pair_src.resize(np);
    d.pair_end.resize(np);
    d.pair_thr.assign(np, 0);
    for (size_t p = 0; p < np; ++p) {
        d.pair_src[p] = S.pairs[p].src;
        d.pair_end[p] = S.pairs[p].seg_end;
    }
    d.small_scr.assign((size_t)S.nsup, -1);
    d.level_ordered.assign((size_t)nl, 0);
    d.app_ptr.assign((size_t)nl + 1, 0);
    d.app_p0.push_back(0);
    std::vector<int64_t> acc((size_t)S.nsup, 0);  // finished (tile, target) scatters so far
    std::vector<std::vector<int32_t>> lists((size_t)S.nsup);
    std::vector<int32_t> touched;
    for (int32_t l = 0; l < nl; ++l) {
        int64_t scr = 0;
        touched.clear();
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            if (!is_small(S, s)) continue;
            bool shared = false;
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                if (ex[p]) continue;
                shared = true;
                const int32_t t = S.pairs[p].tgt;
                if (lists[t].empty()) touched.push_back(t);
                lists[t].push_back((int32_t)p);
            }
            if (shared) {
                const int64_t r = S.nbelow(s);
                d.small_scr[s] = scr;
                scr += r * (r + 1) / 2;
            }
        }
        d.scratch = std::max(d.scratch, scr);
        std::sort(touched.begin(), touched.end());
        for (int32_t t : touched) {
            d.app_t.push_back(t);
            for (int32_t p : lists[t]) d.app_pairs.push_back(p);
            d.app_p0.push_back((int64_t)d.app_pairs.size());
            lists[t].clear();
        }
        d.app_ptr[l + 1] = (int64_t)d.app_t.size();
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            if (is_small(S, s)) continue;
            const int32_t r = S.nbelow(s), nb = (r + kTile - 1) / kTile;
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                if (ex[p]) continue;
                const Pair& pr = S.pairs[p];
                d.level_ordered[l] = 1;
                d.overflow |= acc[pr.tgt] > INT32_MAX - (int64_t)nb * (nb + 1);
                d.pair_thr[p] = (int32_t)acc[pr.tgt];
                int64_t tiles = 0;  // tiles (i, j), i >= j, whose column block j meets the pair
                for (int32_t bj = pr.seg_begin / kTile; bj <= (pr.seg_end - 1) / kTile; ++bj)
                    tiles += nb - bj;
                acc[pr.tgt] += tiles;
            }
        }
    }
    return d;
}

void count_work(const Symbolic& S, std::vector<int64_t>& rb_ptr, std::vector<int64_t>& tl_ptr) {
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    rb_ptr.assign((size_t)nl + 1, 0);
    tl_ptr.assign((size_t)nl + 1, 0);
    for (int32_t l = 0; l < nl; ++l) {
        int64_t rb = 0, tl = 0;
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            if (is_small(S, S.level_sn[q])) continue;  // one wave does all of its work
            const int64_t r = S.nbelow(S.level_sn[q]);
            const int64_t nb = (r + kTile - 1) / kTile;
            rb += nb;
            tl += nb * (nb + 1) / 2;
        }
        rb_ptr[l + 1] = rb_ptr[l] + rb;
        tl_ptr[l + 1] = tl_ptr[l] + tl;
    }
}

PlanOffsets plan_layout(const Symbolic& S, const std::vector<int64_t>& rb_ptr,
                        const std::vector<int64_t>& tl_ptr) {
    Layout L;
    PlanOffsets o;
    const size_t ns = (size_t)S.nsup;
    o.sn_first = L.add<int32_t>(ns);
    o.sn_w = L.add<int32_t>(ns);
    o.sn_ld = L.add<int32_t>(ns);
    o.sn_off = L.add<int64_t>(ns);
    o.inv_off = L.add<int64_t>(ns);
    o.rowptr = L.add<int64_t>(ns + 1);
    o.rows = L.add<int32_t>(S.rows.size());
    o.rowpair = L.add<int32_t>(S.rows.size());
    o.slot = L.add<int64_t>(S.slot.size());
    o.perm = L.add<int32_t>(S.perm.size());
    o.pair_tgt = L.add<int32_t>(S.pairs.size());
    o.pair_seg = L.add<int32_t>(S.pairs.size());
    o.pair_rel = L.add<int64_t>(S.pairs.size());
    o.pair_excl = L.add<uint8_t>(S.pairs.size());
    o.rel = L.add<int32_t>(S.rel.size());
    o.level_sn = L.add<int32_t>(S.level_sn.size());
    o.rowblk = L.add<RowBlock>((size_t)rb_ptr.back());
    o.tiles = L.add<UpdTile>((size_t)tl_ptr.back());
    o.rc_ptr = L.add<int64_t>((size_t)S.n + 1);
    o.rc_slot = L.add<int32_t>(S.rows.size() - (size_t)S.n);  // every below-diagonal row
    o.pb_off = L.add<int64_t>(ns);
    o.tasks = o.cnt0 = o.rb_base = 0;
    o.pair_src = o.pair_end = o.pair_thr = o.small_scr = o.app_t = o.app_p0 = o.app_pairs = 0;
    o.total = L.total;
    return o;
}

void det_layout(PlanOffsets& o, const DetData& d) {
    Layout L;
    L.total = o.total;
    o.pair_src = L.add<int32_t>(d.pair_src.size());
    o.pair_end = L.add<int32_t>(d.pair_end.size());
    o.pair_thr = L.add<int32_t>(d.pair_thr.size());
    o.small_scr = L.add<int64_t>(d.small_scr.size());
    o.app_t = L.add<int32_t>(d.app_t.size());
    o.app_p0 = L.add<int64_t>(d.app_p0.size());
    o.app_pairs = L.add<int32_t>(d.app_pairs.size());
    o.total = L.total;
}

}  // namespace

int64_t inverse_blocks_elems(const Symbolic& S) {
    int64_t t = 0;
    for (int64_t s = 0; s < S.nsup; ++s) t += diag_region_elems(S.width(s));
    return t;
}

size_t plan_bytes(const Symbolic& S, int64_t* det_scratch) {
    std::vector<int64_t> a, b;
    count_work(S, a, b);
    PlanOffsets o = plan_layout(S, a, b);
    if (det_scratch) *det_scratch = 0;
    if (S.opt.deterministic) {
        const DetData d = build_det(S, exclusive_pairs(S));
        det_layout(o, d);
        if (det_scratch) *det_scratch = d.scratch;
    }
    return o.total;
}

int32_t get_plan(spc_symbolic* sym, DevicePlan** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ERR_HIP;
    std::lock_guard<std::mutex> lock(sym->mu);
    for (DevicePlan* p : sym->plans)
        if (p->device == dev) { *out = p; return OK; }
    const Symbolic& S = sym->S;
    if (S.max_r >= 32767 * kTile) return ERR_ARG;  // tile coordinates are 16-bit
    if (S.rows.size() >= (size_t)INT32_MAX) return ERR_ARG;  // contribution slots are 32-bit
    DevicePlan* P = new DevicePlan();
    P->device = dev;
    count_work(S, P->rowblk_ptr, P->tile_ptr);
    PlanOffsets o = plan_layout(S, P->rowblk_ptr, P->tile_ptr);
    const std::vector<uint8_t> ex = exclusive_pairs(S);
    DetData det;
    if (S.opt.deterministic) {
        det = build_det(S, ex);
        if (det.overflow) { delete P; return ERR_ARG; }
        det_layout(o, det);
        P->level_ordered = det.level_ordered;
        P->app_ptr = det.app_ptr;
        P->det_scratch = det.scratch;
    }
    // task-queue schedule: task order, dependency counts, row-block bases
    std::vector<Task> tasks;
    std::vector<int32_t> cnt0, rb_base;
    if (S.opt.sched == 2) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
        int32_t st = build_task_order(S, ncu, tasks, cnt0, rb_base);
        if (st != OK) { delete P; return st; }
        if ((S.opt.debug_flags & 1) && S.nsup > 0) cnt0[S.nsup - 1] += 1;
        Layout L2;
        L2.total = o.total;
        o.tasks = L2.add<Task>(tasks.size());
        o.cnt0 = L2.add<int32_t>(cnt0.size());
        o.rb_base = L2.add<int32_t>(rb_base.size());
        o.total = L2.total;
        P->ntasks = (int64_t)tasks.size();
        if (S.opt.debug_flags & 2) P->host_tasks = tasks;
        P->nrowblk = rb_base.empty() ? 0 : rb_base.back();
    }
    std::vector<char> h(o.total ? o.total : 1, 0);
    auto put = [&](size_t at, const void* src, size_t bytes) {
        if (bytes) std::memcpy(h.data() + at, src, bytes);
    };
    const size_t ns = (size_t)S.nsup;
    std::vector<int32_t> w(ns), first(ns);
    std::vector<int64_t> inv(ns);
    int64_t io = 0;
    for (size_t s = 0; s < ns; ++s) {
        first[s] = S.sn_ptr[s];
        w[s] = S.width((int64_t)s);
        inv[s] = io;
        io += diag_region_elems(w[s]);
    }
    P->inv_elems = io;
    put(o.sn_first, first.data(), ns * 4);
    put(o.sn_w, w.data(), ns * 4);
    put(o.sn_ld, S.ld.data(), ns * 4);
    put(o.sn_off, S.off.data(), ns * 8);
    put(o.inv_off, inv.data(), ns * 8);
    put(o.rowptr, S.rowptr.data(), (ns + 1) * 8);
    put(o.rows, S.rows.data(), S.rows.size() * 4);
    {
        std::vector<int32_t> rp(S.rows.size(), -1);
        for (size_t p = 0; p < S.pairs.size(); ++p) {
            const Pair& pr = S.pairs[p];
            const int64_t base = S.rowptr[pr.src] + S.width(pr.src);
            for (int32_t i = pr.seg_begin; i < pr.seg_end; ++i) rp[base + i] = (int32_t)p;
        }
        put(o.rowpair, rp.data(), rp.size() * 4);
    }
    put(o.slot, S.slot.data(), S.slot.size() * 8);
    put(o.perm, S.perm.data(), S.perm.size() * 4);
    {
        const size_t np = S.pairs.size();
        std::vector<int32_t> tg(np), sg(np);
        std::vector<int64_t> ro(np);
        for (size_t p = 0; p < np; ++p) {
            tg[p] = S.pairs[p].tgt;
            sg[p] = S.pairs[p].seg_begin;
            ro[p] = S.pairs[p].rel_off;
        }
        put(o.pair_tgt, tg.data(), np * 4);
        put(o.pair_seg, sg.data(), np * 4);
        put(o.pair_rel, ro.data(), np * 8);
        put(o.pair_excl, ex.data(), np);
    }
    if (S.opt.deterministic) {
        put(o.pair_src, det.pair_src.data(), det.pair_src.size() * 4);
        put(o.pair_end, det.pair_end.data(), det.pair_end.size() * 4);
        put(o.pair_thr, det.pair_thr.data(), det.pair_thr.size() * 4);
        put(o.small_scr, det.small_scr.data(), det.small_scr.size() * 8);
        put(o.app_t, det.app_t.data(), det.app_t.size() * 4);
        put(o.app_p0, det.app_p0.data(), det.app_p0.size() * 8);
        put(o.app_pairs, det.app_pairs.data(), det.app_pairs.size() * 4);
    }
    put(o.rel, S.rel.data(), S.rel.size() * 4);
    {
        // per level: the large supernodes first (in the analysis' order), then the small
        const int32_t nl = (int32_t)S.level_ptr.size() - 1;
        std::vector<int32_t> ls;
        ls.reserve(S.level_sn.size());
        P->level_nbig.assign((size_t)nl, 0);
        P->small_maxw.assign((size_t)nl, 0);
        P->small_maxr.assign((size_t)nl, 0);
        P->small_maxm.assign((size_t)nl, 0);
        for (int32_t l = 0; l < nl; ++l) {
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                const int32_t s = S.level_sn[q];
                if (!is_small(S, s)) continue;
                P->small_maxw[l] = std::max<int32_t>(P->small_maxw[l], S.width(s));
                P->small_maxr[l] = std::max<int32_t>(P->small_maxr[l], (int32_t)S.nbelow(s));
                P->small_maxm[l] = std::max<int32_t>(P->small_maxm[l], (int32_t)S.nrows(s));
            }
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q)
                if (!is_small(S, S.level_sn[q])) ls.push_back(S.level_sn[q]);
            P->level_nbig[l] = (int32_t)(ls.size() - S.level_ptr[l]);
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q)
                if (is_small(S, S.level_sn[q])) ls.push_back(S.level_sn[q]);
        }
        put(o.level_sn, ls.data(), ls.size() * 4);
    }
    {
        const int32_t nl = (int32_t)S.level_ptr.size() - 1;
        std::vector<RowBlock> rb((size_t)P->rowblk_ptr.back());
        std::vector<UpdTile> tl((size_t)P->tile_ptr.back());
        P->level_maxw.assign((size_t)nl, 0);
        P->tile_crit.assign((size_t)nl, 0);
        size_t a = 0, b = 0;
        std::vector<UpdTile> bulk;
        std::vector<uint8_t> colcrit;
        for (int32_t l = 0; l < nl; ++l) {
            // tiles of this level whose columns reach a supernode of level l + 1
            // (needed before that level can be factored) come first, the
            // rest ("bulk") after them
            bulk.clear();
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                const int32_t s = S.level_sn[q];
                if (is_small(S, s)) continue;
                P->level_maxw[l] = std::max(P->level_maxw[l], S.width(s));
                const int32_t r = S.nbelow(s);
                const int32_t nb = (r + kTile - 1) / kTile;
                for (int32_t i = 0; i < nb; ++i) rb[a++] = RowBlock{s, i};
                colcrit.assign((size_t)nb, 0);
                for (int64_t pp = S.pair_ptr[s]; pp < S.pair_ptr[s + 1]; ++pp)
                    if (S.level[S.pairs[pp].tgt] == l + 1)
                        for (int32_t c = S.pairs[pp].seg_begin; c < S.pairs[pp].seg_end; ++c)
                            colcrit[c / kTile] = 1;
                // deterministic order: every source's tiles together, sources
                // in increasing order (a tile waits only on earlier tiles)
                for (int32_t i = 0; i < nb; ++i)
                    for (int32_t j = 0; j <= i; ++j) {
                        const UpdTile t{s, (int16_t)i, (int16_t)j};
                        if (colcrit[j] || S.opt.deterministic) tl[b++] = t;
                        else bulk.push_back(t);
                    }
            }
            P->tile_crit[l] = (int64_t)b - P->tile_ptr[l];
            for (const UpdTile& t : bulk) tl[b++] = t;
        }
        put(o.rowblk, rb.data(), rb.size() * sizeof(RowBlock));
        put(o.tiles, tl.data(), tl.size() * sizeof(UpdTile));
    }
    {
        // forward-solve contributions: one slot per below-diagonal row of every
        // supernode (its position in rows); row j pulls the slots that hold
        // row j, sources in increasing order
        std::vector<int64_t> rcp((size_t)S.n + 1, 0);
        for (int64_t s = 0; s < S.nsup; ++s)
            for (int64_t q = S.rowptr[s] + S.width(s); q < S.rowptr[s + 1]; ++q)
                rcp[(size_t)S.rows[q] + 1]++;
        for (int64_t j = 0; j < S.n; ++j) rcp[j + 1] += rcp[j];
        std::vector<int32_t> rcs((size_t)std::max<int64_t>(rcp[S.n], 1));
        std::vector<int64_t> at(rcp.begin(), rcp.end() - 1);
        for (int64_t s = 0; s < S.nsup; ++s)
            for (int64_t q = S.rowptr[s] + S.width(s); q < S.rowptr[s + 1]; ++q)
                rcs[at[S.rows[q]]++] = (int32_t)q;
        put(o.rc_ptr, rcp.data(), rcp.size() * 8);
        put(o.rc_slot, rcs.data(), (size_t)rcp[S.n] * 4);
        // backward partial sums of the large supernodes' row blocks
        std::vector<int64_t> pbo((size_t)S.nsup, 0);
        int64_t tot = 0;
        for (int64_t s = 0; s < S.nsup; ++s) {
            pbo[s] = tot;
            if (!is_small(S, s)) tot += (int64_t)((S.nbelow(s) + kTile - 1) / kTile) * S.width(s);
        }
        put(o.pb_off, pbo.data(), pbo.size() * 8);
        P->nslots = (int64_t)S.rows.size();
        P->pb_total = tot;
    }
    if (!tasks.empty()) put(o.tasks, tasks.data(), tasks.size() * sizeof(Task));
    if (!cnt0.empty()) put(o.cnt0, cnt0.data(), cnt0.size() * 4);
    if (!rb_base.empty()) put(o.rb_base, rb_base.data(), rb_base.size() * 4);
    P->max_w = S.max_w;
    void* d = nullptr;
    if (hipMalloc(&d, o.total ? o.total : 256) != hipSuccess) { delete P; return ERR_OOM; }
    if (hipMemcpy(d, h.data(), o.total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        delete P;
        return ERR_HIP;
    }
    char* base = (char*)d;
    P->block = d;
    P->bytes = o.total;
    P->sn_first = (int32_t*)(base + o.sn_first);
    P->sn_w = (int32_t*)(base + o.sn_w);
    P->sn_ld = (int32_t*)(base + o.sn_ld);
    P->sn_off = (int64_t*)(base + o.sn_off);
    P->inv_off = (int64_t*)(base + o.inv_off);
    P->rowptr = (int64_t*)(base + o.rowptr);
    P->rows = (int32_t*)(base + o.rows);
    P->rowpair = (int32_t*)(base + o.rowpair);
    P->slot = (int64_t*)(base + o.slot);
    P->perm = (int32_t*)(base + o.perm);
    P->pair_tgt = (int32_t*)(base + o.pair_tgt);
    P->pair_seg = (int32_t*)(base + o.pair_seg);
    P->pair_rel = (int64_t*)(base + o.pair_rel);
    P->pair_excl = (uint8_t*)(base + o.pair_excl);
    P->rel = (int32_t*)(base + o.rel);
    P->level_sn = (int32_t*)(base + o.level_sn);
    P->rowblk = (RowBlock*)(base + o.rowblk);
    P->tiles = (UpdTile*)(base + o.tiles);
    P->rc_ptr = (int64_t*)(base + o.rc_ptr);
    P->rc_slot = (int32_t*)(base + o.rc_slot);
    P->pb_off = (int64_t*)(base + o.pb_off);
    if (S.opt.deterministic) {
        P->pair_src = (int32_t*)(base + o.pair_src);
        P->pair_end = (int32_t*)(base + o.pair_end);
        P->pair_thr = (int32_t*)(base + o.pair_thr);
        P->small_scr = (int64_t*)(base + o.small_scr);
        P->app_t = (int32_t*)(base + o.app_t);
        P->app_p0 = (int64_t*)(base + o.app_p0);
        P->app_pairs = (int32_t*)(base + o.app_pairs);
    }
    if (S.opt.sched == 2) {
        P->tasks = (Task*)(base + o.tasks);
        P->cnt0 = (int32_t*)(base + o.cnt0);
        P->rb_base = (int32_t*)(base + o.rb_base);
    }
    sym->plans.push_back(P);
    *out = P;
    return OK;
}

void free_plan(DevicePlan* p) {
    if (!p) return;
    if (p->block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        (void)hipFree(p->block);
        (void)hipSetDevice(cur);
    }
    delete p;
}

KArgs kargs(const DevicePlan* P) {
    KArgs a;
    a.sn_first = P->sn_first;
    a.sn_w = P->sn_w;
    a.sn_ld = P->sn_ld;
    a.sn_off = P->sn_off;
    a.inv_off = P->inv_off;
    a.rowptr = P->rowptr;
    a.rows = P->rows;
    a.rowpair = P->rowpair;
    a.pair_tgt = P->pair_tgt;
    a.pair_seg = P->pair_seg;
    a.pair_rel = P->pair_rel;
    a.rel = P->rel;
    return a;
}

}  // namespace spc
