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
        pair_seg, pair_rel, pair_excl, rel, level_sn, small_rec, big_sn, rowblk, tiles, tasks,
        cnt0, rb_base;
    size_t pair_src, pair_end, scr_off, app_t, app_rb, app_p0, app_ent;
    size_t slot_shared, red_row, red_ptr, red_slot, colblk, fwdblk, sspart, pb_off;
    size_t tail_tasks, tail_segs;
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
// (target, source) of Section III-D).  A pair whose target no other source
// of the level touches adds its entries directly.  The other ("shared")
// contributions of a level take one of two forms:
//   apply: the sources write them to a per-level scratch (each source's
//          lower r x r update block, packed by columns) and one wave per
//          (shared target, block of 64 of its rows) adds them, pair by pair
//          in increasing source order, one lane per target row (so every
//          target entry is added by one lane, in program order) (always for
//          the small supernodes' lane-group kernel);
//   rounds: the large sources are coloured first-fit (round(s) = the first
//          round none of the level's earlier sources sharing a target with s
//          took), each round is one launch in which every target has one
//          writer (plain read-modify-writes), and a target meets its sources
//          round by round.
// A level's large sources take the cheaper form by a cost estimate: a round
// launch about 25 us; the scratch 16 bytes per entry at 4 TB/s plus about
// 2 us per pair of its longest per-target chain; and the scratch at most
// 2^25 entries.
struct DetData {
    std::vector<int32_t> pair_src, pair_end, app_t, app_rb;
    std::vector<AppEnt> app_ent;
    std::vector<int64_t> scr_off, app_p0;   // scr_off: per supernode, -1 = none
    std::vector<int32_t> round;             // per supernode (large sources)
    std::vector<int32_t> level_rounds;      // rounds of every level (apply form: 1)
    std::vector<uint8_t> level_apply;       // large sources in the apply form
    std::vector<int64_t> app_ptr;
    int64_t scratch = 0;
};

DetData build_det(const Symbolic& S, const std::vector<uint8_t>& ex) {
    DetData d;
    const size_t np = S.pairs.size();
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    d.pair_src.resize(np);
    d.pair_end.resize(np);
    for (size_t p = 0; p < np; ++p) {
        d.pair_src[p] = S.pairs[p].src;
        d.pair_end[p] = S.pairs[p].seg_end;
    }
    d.scr_off.assign((size_t)S.nsup, -1);
    d.round.assign((size_t)S.nsup, 0);
    d.level_rounds.assign((size_t)nl, 1);
    d.level_apply.assign((size_t)nl, 0);
    d.app_ptr.assign((size_t)nl + 1, 0);
    d.app_p0.push_back(0);
    std::vector<std::vector<int32_t>> lists((size_t)S.nsup), used((size_t)S.nsup);
    std::vector<int32_t> touched;
    std::vector<uint8_t> busy;
    std::vector<std::vector<AppEnt>> blocks;
    auto has_shared = [&](int32_t s) {
        for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p)
            if (!ex[p]) return true;
        return false;
    };
    for (int32_t l = 0; l < nl; ++l) {
        // first-fit rounds of the large sources, and the apply form's size
        int32_t rounds = 1, longest = 0;
        int64_t big_scr = 0;
        touched.clear();
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            if (is_small(S, s) || !has_shared(s)) continue;
            busy.assign((size_t)rounds + 1, 0);
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p)
                if (!ex[p])
                    for (int32_t u : used[S.pairs[p].tgt]) busy[u] = 1;
            int32_t rs = 0;
            while (busy[rs]) ++rs;
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                if (ex[p]) continue;
                const int32_t t = S.pairs[p].tgt;
                if (used[t].empty()) touched.push_back(t);
                used[t].push_back(rs);
                longest = std::max(longest, (int32_t)used[t].size());
            }
            d.round[s] = rs;
            rounds = std::max(rounds, rs + 1);
            const int64_t r = S.nbelow(s);
            big_scr += r * (r + 1) / 2;
        }
        for (int32_t t : touched) used[t].clear();
        const double round_us = 25.0 * (rounds - 1);
        const double apply_us = 16.0 * (double)big_scr / 4e6 + 2.0 * longest;
        const bool apply = rounds > 1 && big_scr <= ((int64_t)1 << 25) && apply_us < round_us;
        d.level_apply[l] = apply;
        d.level_rounds[l] = apply ? 1 : rounds;
        // scratch blocks and apply lists: the small sources, and the large
        // ones in the apply form, in increasing source order
        int64_t scr = 0;
        touched.clear();
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            const bool small = is_small(S, s);
            if (!small && apply) d.round[s] = 0;
            if ((!small && !apply) || !has_shared(s)) continue;
            for (int64_t p = S.pair_ptr[s]; p < S.pair_ptr[s + 1]; ++p) {
                if (ex[p]) continue;
                const int32_t t = S.pairs[p].tgt;
                if (lists[t].empty()) touched.push_back(t);
                lists[t].push_back((int32_t)p);
            }
            const int64_t r = S.nbelow(s);
            d.scr_off[s] = scr;
            scr += r * (r + 1) / 2;
        }
        d.scratch = std::max(d.scratch, scr);
        std::sort(touched.begin(), touched.end());
        for (int32_t t : touched) {
            // split every pair's rows by the 64-row block of the target row they
            // land in (relative indices increase with the row), then one item
            // per block with its (pair, rows) entries in source order
            const int32_t nblk = (S.nrows(t) + kTile - 1) / kTile;
            blocks.assign((size_t)nblk, {});
            for (int32_t p : lists[t]) {
                const Pair& pr = S.pairs[p];
                const int32_t r = S.nbelow(pr.src);
                int32_t i = pr.seg_begin;
                while (i < r) {
                    const int32_t blk = S.rel[pr.rel_off + (i - pr.seg_begin)] / kTile;
                    int32_t e = i + 1;
                    while (e < r && S.rel[pr.rel_off + (e - pr.seg_begin)] / kTile == blk) ++e;
                    blocks[blk].push_back(AppEnt{p, i, e, 0});
                    i = e;
                }
            }
            for (int32_t blk = 0; blk < nblk; ++blk) {
                if (blocks[blk].empty()) continue;
                d.app_t.push_back(t);
                d.app_rb.push_back(blk);
                for (const AppEnt& en : blocks[blk]) d.app_ent.push_back(en);
                d.app_p0.push_back((int64_t)d.app_ent.size());
            }
            lists[t].clear();
        }
        d.app_ptr[l + 1] = (int64_t)d.app_t.size();
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
    o.small_rec = L.add<SmallRec>(S.level_sn.size());
    o.big_sn = L.add<int32_t>(S.level_sn.size());
    o.rowblk = L.add<RowBlock>((size_t)rb_ptr.back());
    o.tiles = L.add<UpdTile>((size_t)tl_ptr.back());
    o.slot_shared = L.add<uint8_t>(S.rows.size());
    o.red_row = o.red_ptr = o.red_slot = 0;  // sized by solve_layout
    o.colblk = o.fwdblk = o.sspart = o.tail_tasks = o.tail_segs = 0;
    o.pb_off = L.add<int64_t>(ns);
    o.tasks = o.cnt0 = o.rb_base = 0;
    o.pair_src = o.pair_end = o.scr_off = o.app_t = o.app_rb = o.app_p0 = o.app_ent = 0;
    o.total = L.total;
    return o;
}

// Forward solve: every below-diagonal row of a source has a contribution
// slot (its place in rows).  A row that only one source of a level touches
// is updated by that source directly; a row that several share ("shared"
// slots) is reduced after the level, sources in increasing order, by one
// thread per row.  Backward solve: the large supernodes' column groups.
struct SolveData {
    std::vector<uint8_t> shared;       // per slot
    std::vector<int32_t> red_row;      // reduce items: target row
    std::vector<int64_t> red_ptr;      // its slots red_slot[red_ptr[k] .. red_ptr[k + 1])
    std::vector<int32_t> red_slot;
    std::vector<int64_t> red_level_ptr;  // per level: its items
    std::vector<ColBlk> colblk;        // (s, column group, row chunk) of the large supernodes
    std::vector<int64_t> colblk_ptr;   // per level
    std::vector<RowBlock> fwdblk;      // (s, 64-row block) of the large supernodes
    std::vector<int64_t> fwdblk_ptr;   // per level
    std::vector<RowBlock> sspart;      // (s, 16-row part of the diagonal block), large ones
    std::vector<int64_t> sspart_ptr;   // per level
    std::vector<int64_t> pb_off;       // per supernode
    int64_t pb_total = 0;
    int32_t tail_l0 = 0, ntail = 0;
    std::vector<TailTask> tail;        // the tail's tasks in ticket order
    std::vector<TailSeg> segs;
};

// The tail's tasks (levels [l0, levels) of the supernodal etree, every
// supernode there large), in a topological ticket order: per level from the
// leaves, the F tasks, then the R blocks; then per level from the root, the
// C blocks, then the B tasks.  A forward row block's rows are split into
// segments by target; a target receives its rows' updates source after
// source in that ticket order, so each segment's rank is the number of the
// target's rows that earlier blocks update.  A backward row block lists the
// supernodes its rows belong to (it waits for each one's solution).
void build_tail(const Symbolic& S, int32_t l0, SolveData& d) {
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    d.tail_l0 = l0;
    if (l0 >= nl) return;
    std::vector<int32_t> tix((size_t)S.nsup, -1);
    int32_t nt = 0;
    for (int32_t q = S.level_ptr[l0]; q < S.level_ptr[nl]; ++q) tix[S.level_sn[q]] = nt++;
    d.ntail = nt;
    std::vector<int32_t> need((size_t)nt, 0), acc((size_t)nt, 0);
    for (int32_t q = S.level_ptr[l0]; q < S.level_ptr[nl]; ++q) {
        const int32_t s = S.level_sn[q];
        for (int64_t k = S.rowptr[s] + S.width(s); k < S.rowptr[s + 1]; ++k)
            need[tix[S.col_owner[S.rows[k]]]]++;
    }
    auto blocks = [&](int32_t s) { return (S.nbelow(s) + kTile - 1) / kTile; };
    for (int32_t l = l0; l < nl; ++l) {
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            d.tail.push_back(TailTask{s, tix[s], kTailF, 0, need[tix[s]], 0});
        }
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            const int32_t r = S.nbelow(s);
            for (int32_t rb = 0; rb < blocks(s); ++rb) {
                const int64_t base = S.rowptr[s] + S.width(s) + (int64_t)rb * kTile;
                const int32_t m = std::min(kTile, r - rb * kTile);
                const int32_t g0 = (int32_t)d.segs.size();
                for (int32_t i = 0; i < m;) {
                    const int32_t t = S.col_owner[S.rows[base + i]];
                    int32_t j = i + 1;
                    while (j < m && S.col_owner[S.rows[base + j]] == t) ++j;
                    const int32_t u = tix[t];
                    d.segs.push_back(TailSeg{u, i, j, acc[u]});
                    acc[u] += j - i;
                    i = j;
                }
                d.tail.push_back(
                    TailTask{s, tix[s], kTailR, (int16_t)rb, g0, (int32_t)d.segs.size()});
            }
        }
    }
    for (int32_t l = nl - 1; l >= l0; --l) {
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            const int32_t r = S.nbelow(s);
            for (int32_t rb = 0; rb < blocks(s); ++rb) {
                const int64_t base = S.rowptr[s] + S.width(s) + (int64_t)rb * kTile;
                const int32_t m = std::min(kTile, r - rb * kTile);
                const int32_t g0 = (int32_t)d.segs.size();
                for (int32_t i = 0; i < m;) {
                    const int32_t t = S.col_owner[S.rows[base + i]];
                    int32_t j = i + 1;
                    while (j < m && S.col_owner[S.rows[base + j]] == t) ++j;
                    d.segs.push_back(TailSeg{tix[t], i, j, 0});
                    i = j;
                }
                d.tail.push_back(
                    TailTask{s, tix[s], kTailC, (int16_t)rb, g0, (int32_t)d.segs.size()});
            }
        }
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            d.tail.push_back(TailTask{s, tix[s], kTailB, 0, blocks(s), 0});
        }
    }
}

SolveData build_solve(const Symbolic& S) {
    SolveData d;
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    d.shared.assign(S.rows.size(), 0);
    d.red_level_ptr.assign((size_t)nl + 1, 0);
    d.colblk_ptr.assign((size_t)nl + 1, 0);
    d.fwdblk_ptr.assign((size_t)nl + 1, 0);
    d.sspart_ptr.assign((size_t)nl + 1, 0);
    d.red_ptr.push_back(0);
    d.pb_off.assign((size_t)S.nsup, 0);
    std::vector<int32_t> cnt((size_t)S.n, 0), stamp((size_t)S.n, -1);
    std::vector<int32_t> rows_touched;
    const int32_t l0 = tail_start(S);
    for (int32_t l = 0; l < nl; ++l) {
        if (l >= l0) {
            // the tail: no level kernels; 64-row partial sums for its C blocks
            d.red_level_ptr[l + 1] = d.red_level_ptr[l];
            d.colblk_ptr[l + 1] = (int64_t)d.colblk.size();
            d.fwdblk_ptr[l + 1] = (int64_t)d.fwdblk.size();
            d.sspart_ptr[l + 1] = (int64_t)d.sspart.size();
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                const int32_t s = S.level_sn[q];
                d.pb_off[s] = d.pb_total;
                d.pb_total += (int64_t)((S.nbelow(s) + kTile - 1) / kTile) * S.width(s);
            }
            continue;
        }
        rows_touched.clear();
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            for (int64_t k = S.rowptr[s] + S.width(s); k < S.rowptr[s + 1]; ++k) {
                const int32_t row = S.rows[k];
                if (stamp[row] != l) { stamp[row] = l; cnt[row] = 0; rows_touched.push_back(row); }
                cnt[row]++;
            }
        }
        std::sort(rows_touched.begin(), rows_touched.end());
        // the level's shared rows become reduce items (cnt turns into the
        // negated item index + 1); their slots, sources in increasing order
        const int64_t items0 = (int64_t)d.red_row.size();
        for (int32_t row : rows_touched)
            if (cnt[row] > 1) {
                d.red_row.push_back(row);
                cnt[row] = -(int32_t)(d.red_row.size() - items0);
            }
        const int64_t nitems = (int64_t)d.red_row.size() - items0;
        std::vector<std::vector<int32_t>> sl((size_t)nitems);
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            for (int64_t k = S.rowptr[s] + S.width(s); k < S.rowptr[s + 1]; ++k) {
                const int32_t row = S.rows[k];
                if (cnt[row] < 0) {
                    d.shared[k] = 1;
                    sl[(size_t)(-cnt[row] - 1)].push_back((int32_t)k);
                }
            }
        }
        for (auto& v : sl) {
            for (int32_t k : v) d.red_slot.push_back(k);
            d.red_ptr.push_back((int64_t)d.red_slot.size());
        }
        d.red_level_ptr[l + 1] = (int64_t)d.red_row.size();
        // every large supernode gets at least one forward workgroup: its
        // diagonal block is solved there even with no rows below
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int32_t s = S.level_sn[q];
            if (is_small(S, s)) continue;
            const int32_t nb = std::max<int32_t>(1, (S.nbelow(s) + kTile - 1) / kTile);
            for (int32_t rb = 0; rb < nb; ++rb) d.fwdblk.push_back(RowBlock{s, rb});
            for (int32_t pt = 0; pt * kPartRows < S.width(s); ++pt)
                d.sspart.push_back(RowBlock{s, pt});
            if (S.nbelow(s) == 0) continue;
            const int32_t ng = (S.width(s) + kColGroup - 1) / kColGroup;
            const int32_t nh = (S.nbelow(s) + kRowChunk - 1) / kRowChunk;
            for (int32_t h = 0; h < nh; ++h)
                for (int32_t g = 0; g < ng; ++g)
                    d.colblk.push_back(ColBlk{s, (int16_t)g, (int16_t)h});
            d.pb_off[s] = d.pb_total;
            d.pb_total += (int64_t)nh * S.width(s);
        }
        d.colblk_ptr[l + 1] = (int64_t)d.colblk.size();
        d.fwdblk_ptr[l + 1] = (int64_t)d.fwdblk.size();
        d.sspart_ptr[l + 1] = (int64_t)d.sspart.size();
    }
    build_tail(S, l0, d);
    return d;
}

void solve_layout(PlanOffsets& o, const SolveData& d) {
    Layout L;
    L.total = o.total;
    o.red_row = L.add<int32_t>(d.red_row.size());
    o.red_ptr = L.add<int64_t>(d.red_ptr.size());
    o.red_slot = L.add<int32_t>(d.red_slot.size());
    o.colblk = L.add<ColBlk>(d.colblk.size());
    o.fwdblk = L.add<RowBlock>(d.fwdblk.size());
    o.sspart = L.add<RowBlock>(d.sspart.size());
    o.tail_tasks = L.add<TailTask>(d.tail.size());
    o.tail_segs = L.add<TailSeg>(d.segs.size());
    o.total = L.total;
}

void det_layout(PlanOffsets& o, const DetData& d) {
    Layout L;
    L.total = o.total;
    o.pair_src = L.add<int32_t>(d.pair_src.size());
    o.pair_end = L.add<int32_t>(d.pair_end.size());
    o.scr_off = L.add<int64_t>(d.scr_off.size());
    o.app_t = L.add<int32_t>(d.app_t.size());
    o.app_p0 = L.add<int64_t>(d.app_p0.size());
    o.app_rb = L.add<int32_t>(d.app_rb.size());
    o.app_ent = L.add<AppEnt>(d.app_ent.size());
    o.total = L.total;
}

}  // namespace

int32_t tail_start(const Symbolic& S) {
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    // the tail's forward updates are atomic adds: only in the atomic order
    if (S.opt.solve_tail != 1 || S.opt.deterministic || nl < 2) return std::max(nl, 0);
    int32_t l = nl;
    while (l > 0) {
        const int32_t q0 = S.level_ptr[l - 1], q1 = S.level_ptr[l];
        if (q1 - q0 > kTailMaxLevelSn) break;
        bool small = false;
        for (int32_t q = q0; q < q1 && !small; ++q) small = is_small(S, S.level_sn[q]);
        if (small) break;
        --l;
    }
    return nl - l >= 2 ? l : nl;  // a tail of one level saves nothing
}

int64_t solve_pb_elems(const Symbolic& S) {
    const int32_t l0 = tail_start(S);
    int64_t pb = 0;
    for (int64_t s = 0; s < S.nsup; ++s) {
        const int32_t r = S.nbelow(s);
        if (S.level[s] >= l0) pb += (int64_t)((r + kTile - 1) / kTile) * S.width(s);
        else if (!is_small(S, s) && r > 0) pb += (int64_t)((r + kRowChunk - 1) / kRowChunk) * S.width(s);
    }
    return pb;
}

int64_t tail_state_words(const Symbolic& S) {
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    const int32_t l0 = tail_start(S);
    if (l0 >= nl) return 0;
    return 4 * (int64_t)(S.level_ptr[nl] - S.level_ptr[l0]) + 4;
}

int64_t split_state_words(const Symbolic& S) { return 2 * S.nsup + 3; }

int64_t inverse_blocks_elems(const Symbolic& S) {
    int64_t t = 0;
    for (int64_t s = 0; s < S.nsup; ++s) t += diag_region_elems(S.width(s));
    return t;
}

size_t plan_bytes(const Symbolic& S, int64_t* det_scratch) {
    std::vector<int64_t> a, b;
    count_work(S, a, b);
    PlanOffsets o = plan_layout(S, a, b);
    solve_layout(o, build_solve(S));
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
    const SolveData sd = build_solve(S);
    solve_layout(o, sd);
    const std::vector<uint8_t> ex = exclusive_pairs(S);
    DetData det;
    if (S.opt.deterministic) {
        det = build_det(S, ex);
        det_layout(o, det);
        P->app_ptr = det.app_ptr;
        P->level_apply = det.level_apply;
        P->det_scratch = det.scratch;
    }
    // task-queue schedule: task order, dependency counts, row-block bases
    std::vector<Task> tasks;
    std::vector<int32_t> cnt0, rb_base;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            ncu > 0)
            P->ncu = ncu;
    }
    if (S.opt.sched == 2) {
        int32_t st = build_task_order(S, P->ncu, tasks, cnt0, rb_base);
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
        put(o.scr_off, det.scr_off.data(), det.scr_off.size() * 8);
        put(o.app_t, det.app_t.data(), det.app_t.size() * 4);
        put(o.app_p0, det.app_p0.data(), det.app_p0.size() * 8);
        put(o.app_rb, det.app_rb.data(), det.app_rb.size() * 4);
        put(o.app_ent, det.app_ent.data(), det.app_ent.size() * sizeof(AppEnt));
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
        std::vector<SmallRec> rec(ls.size());
        for (size_t q = 0; q < ls.size(); ++q) {
            const int32_t s = ls[q];
            rec[q] = SmallRec{S.off[s], inv[s], S.rowptr[s], w[s], S.ld[s], first[s],
                              (int32_t)S.nbelow(s)};
        }
        put(o.small_rec, rec.data(), rec.size() * sizeof(SmallRec));
        std::vector<int32_t> big;
        for (int32_t l = 0; l < nl; ++l)
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l] + P->level_nbig[l]; ++q) {
                big.push_back(ls[q]);
                P->big_maxw = std::max<int32_t>(P->big_maxw, S.width(ls[q]));
            }
        P->nbig = (int64_t)big.size();
        if (!big.empty()) put(o.big_sn, big.data(), big.size() * 4);
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
        if (S.opt.deterministic) P->round_ptr.assign((size_t)nl, {});
        for (int32_t l = 0; l < nl; ++l) {
            if (S.opt.deterministic) {
                // rounds one after another, sources in increasing order in each
                const int32_t R = std::max(1, det.level_rounds[l]);
                std::vector<int64_t>& rp = P->round_ptr[l];
                rp.assign((size_t)R + 1, (int64_t)b);
                for (int32_t rr = 0; rr < R; ++rr) {
                    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                        const int32_t s = S.level_sn[q];
                        if (is_small(S, s) || det.round[s] != rr) continue;
                        const int32_t nb = (S.nbelow(s) + kTile - 1) / kTile;
                        for (int32_t i = 0; i < nb; ++i)
                            for (int32_t j = 0; j <= i; ++j)
                                tl[b++] = UpdTile{s, (int16_t)i, (int16_t)j};
                    }
                    rp[rr + 1] = (int64_t)b;
                }
                for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                    const int32_t s = S.level_sn[q];
                    if (is_small(S, s)) continue;
                    P->level_maxw[l] = std::max(P->level_maxw[l], S.width(s));
                    const int32_t nb = (S.nbelow(s) + kTile - 1) / kTile;
                    for (int32_t i = 0; i < nb; ++i) rb[a++] = RowBlock{s, i};
                }
                P->tile_crit[l] = (int64_t)b - P->tile_ptr[l];
                continue;
            }
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
                for (int32_t i = 0; i < nb; ++i)
                    for (int32_t j = 0; j <= i; ++j) {
                        const UpdTile t{s, (int16_t)i, (int16_t)j};
                        if (colcrit[j]) tl[b++] = t;
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
        put(o.slot_shared, sd.shared.data(), sd.shared.size());
        put(o.red_row, sd.red_row.data(), sd.red_row.size() * 4);
        put(o.red_ptr, sd.red_ptr.data(), sd.red_ptr.size() * 8);
        put(o.red_slot, sd.red_slot.data(), sd.red_slot.size() * 4);
        put(o.colblk, sd.colblk.data(), sd.colblk.size() * sizeof(ColBlk));
        put(o.fwdblk, sd.fwdblk.data(), sd.fwdblk.size() * sizeof(RowBlock));
        put(o.sspart, sd.sspart.data(), sd.sspart.size() * sizeof(RowBlock));
        put(o.pb_off, sd.pb_off.data(), sd.pb_off.size() * 8);
        P->nslots = (int64_t)S.rows.size();
        P->pb_total = sd.pb_total;
        P->red_level_ptr = sd.red_level_ptr;
        P->colblk_ptr = sd.colblk_ptr;
        P->fwdblk_ptr = sd.fwdblk_ptr;
        P->sspart_ptr = sd.sspart_ptr;
        put(o.tail_tasks, sd.tail.data(), sd.tail.size() * sizeof(TailTask));
        put(o.tail_segs, sd.segs.data(), sd.segs.size() * sizeof(TailSeg));
        P->tail_l0 = sd.tail_l0;
        P->ntail = sd.ntail;
        P->ntail_tasks = (int64_t)sd.tail.size();
        while (P->ntail_fwd < P->ntail_tasks &&
               (sd.tail[P->ntail_fwd].kind == kTailF || sd.tail[P->ntail_fwd].kind == kTailR))
            ++P->ntail_fwd;
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
    P->small_rec = (SmallRec*)(base + o.small_rec);
    P->big_sn = (int32_t*)(base + o.big_sn);
    P->rowblk = (RowBlock*)(base + o.rowblk);
    P->tiles = (UpdTile*)(base + o.tiles);
    P->slot_shared = (uint8_t*)(base + o.slot_shared);
    P->red_row = (int32_t*)(base + o.red_row);
    P->red_ptr = (int64_t*)(base + o.red_ptr);
    P->red_slot = (int32_t*)(base + o.red_slot);
    P->colblk = (ColBlk*)(base + o.colblk);
    P->fwdblk = (RowBlock*)(base + o.fwdblk);
    P->sspart = (RowBlock*)(base + o.sspart);
    P->pb_off = (int64_t*)(base + o.pb_off);
    P->tail_tasks = (TailTask*)(base + o.tail_tasks);
    P->tail_segs = (TailSeg*)(base + o.tail_segs);
    if (S.opt.deterministic) {
        P->pair_src = (int32_t*)(base + o.pair_src);
        P->pair_end = (int32_t*)(base + o.pair_end);
        P->scr_off = (int64_t*)(base + o.scr_off);
        P->app_t = (int32_t*)(base + o.app_t);
        P->app_p0 = (int64_t*)(base + o.app_p0);
        P->app_rb = (int32_t*)(base + o.app_rb);
        P->app_ent = (AppEnt*)(base + o.app_ent);
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
