// Device side of the supernodal Cholesky: the plan uploaded to HBM, the
// numeric factor object, and the factor / solve drivers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "symbolic.hpp"

namespace spc {

// Tile edge of the update and panel kernels (rows of the below-diagonal panel).
constexpr int kTile = 64;
// Widest supernode the diagonal-block kernels hold in LDS (packed lower
// triangle plus inverse blocks and staged rows); the paper's cap is 150.
constexpr int kMaxWidth = 150;
// Column panel of the blocked diagonal factorization; the inverse of every
// kPanel x kPanel diagonal block is kept for the panel and triangular solves.
constexpr int kPanel = 16;
// Small supernodes (at most small_w columns and small_r rows below the
// diagonal block, analysis options bounded by kSmallW and kSmallR) are
// factored and solved by a group of lanes each; the level-set schedules use
// these kernels, the task queue does not.
constexpr int kSmallW = 16;
constexpr int kSmallR = 64;
inline bool is_small(const Symbolic& S, int64_t s) {
    return S.width(s) <= S.opt.small_w && S.nbelow(s) <= S.opt.small_r;
}
// Per-supernode region of the factor's side array (dinv), for w columns:
//   the inverses of the kPanel-column diagonal blocks, compact: every full
//   panel as kPanel x kPanel, the last partial one (jb < kPanel columns) as
//   jb x jb, each row major;
//   then, for a large supernode, L11^{-1} as a packed lower triangle by
//   columns (entry (i, j) at j (2w - j - 1) / 2 + i), which the solves apply
//   as one triangular matrix-vector product (a small supernode's solves use
//   the compact inverse, its only panel);
//   then L11^{-T} as a packed upper triangle by columns (entry (i, j), i <= j,
//   at j (j + 1) / 2 + i): the backward solve's product with consecutive
//   rows in consecutive addresses.
__host__ __device__ inline int64_t inverse_elems(int32_t w) {
    const int64_t full = w / kPanel, rem = w % kPanel;
    return full * kPanel * kPanel + rem * rem;
}
__host__ __device__ inline int64_t diag_region_elems(int32_t w) {
    return inverse_elems(w) + (int64_t)w * (w + 1);
}
// Row i and column j of entry e of a packed lower triangle of order w stored
// by columns (column j starts at j (2w - j - 1) / 2 + j): j from the root of
// j^2 - (2w + 1) j + 2e = 0 in single precision, then one correction step.
__host__ __device__ inline void tri_entry(int e, int w, int& i, int& j) {
    const float b = 2.0f * (float)w + 1.0f;
    j = (int)((b - sqrtf(b * b - 8.0f * (float)e)) * 0.5f);
    if (j < 0) j = 0;
    if (j > w - 1) j = w - 1;
    auto start = [w](int c) { return (c * (2 * w - c + 1)) >> 1; };  // index of (c, c)
    if (start(j) > e) --j;
    else if (j + 1 < w && start(j + 1) <= e) ++j;
    i = e - start(j) + j;
}
// q = e / w, r = e % w for 0 <= e < 2^24 and 0 < w, by a float reciprocal
// (invw = 1.0f / w) and one correction step; integer division by a runtime
// value costs tens of instructions on the GPU.
__host__ __device__ inline void divmod_small(int e, int w, float invw, int& q, int& r) {
    q = (int)((float)e * invw);
    r = e - q * w;
    if (r < 0) {
        --q;
        r += w;
    } else if (r >= w) {
        ++q;
        r -= w;
    }
}

// Device task-queue schedule: task kinds and the task record.
enum : int32_t { kTaskF = 0, kTaskT = 1, kTaskU = 2 };
struct Task { int32_t s; int16_t a, b; int32_t kind; };

// One update tile: rows [bi*64, bi*64+64) x columns [bj*64, bj*64+64) of the
// lower triangle of P P^T, P = the below-diagonal panel of source supernode s.
struct UpdTile { int32_t s; int16_t bi, bj; };
// One panel row block of source supernode s.
struct RowBlock { int32_t s; int32_t rb; };
// One small supernode's solve metadata in one record (the kernels read it
// with one load instead of a supernode index and then seven lookups):
// arena offset of its block, offset of its diagonal region in dinv, its
// first entry in rows, width, leading dimension, first column, rows below.
struct SmallRec { int64_t off, inv, rp; int32_t w, ld, first, r; };
// Backward solve: a workgroup takes kColGroup columns of one chunk of
// kRowChunk rows below the diagonal block.
constexpr int kColGroup = 8;
constexpr int kRowChunk = 512;
// Single-right-hand-side level solves: a large supernode's diagonal block is
// applied by parts of kPartRows rows, one workgroup each.
constexpr int kPartRows = 16;
struct ColBlk { int32_t s; int16_t g, h; };  // column group g, row chunk h of supernode s
// Deterministic order, apply pass: rows [ilo, ihi) of pair p's source that
// land in one 64-row block of the target.
struct AppEnt { int32_t p, ilo, ihi, pad; };
// Solves of the top levels of the supernodal elimination tree (the tail: the
// levels above the last one with more than kTailMaxLevelSn supernodes or a
// small one) run as one persistent launch of tasks in a fixed topological
// order (solve.hip, k_tail).  u is the supernode's index among the tail's.
enum : int16_t { kTailF = 0, kTailR = 1, kTailC = 2, kTailB = 3 };
struct TailTask {
    int32_t s, u;
    int16_t kind, rb;  // task kind, 64-row block of the supernode's rows below
    int32_t a, b;      // F: rows the tail's sources update; R, C: its segments [a, b);
                       // B: its row blocks
};
// Rows [lo, hi) of an R block that land in tail supernode u (rank: rows of u
// that earlier sources update), or of a C block that belong to u (rank 0).
struct TailSeg { int32_t u, lo, hi, rank; };
constexpr int kTailMaxLevelSn = 128;

// Device copy of the symbolic analysis, shared by every factor of it on one device.
struct DevicePlan {
    int device = -1;
    int32_t ncu = 256;  // compute units of the device
    void* block = nullptr;  // single allocation holding everything below
    size_t bytes = 0;
    int32_t* sn_first = nullptr;
    int32_t* sn_w = nullptr;
    int32_t* sn_ld = nullptr;
    int64_t* sn_off = nullptr;
    int64_t* inv_off = nullptr;  // offset of the supernode's region of dinv (inverses, packed L11)
    int64_t inv_elems = 0;
    int64_t* rowptr = nullptr;
    int32_t* rows = nullptr;
    int32_t* rowpair = nullptr;  // per entry of rows: pair index of the source row, -1 on own columns
    int64_t* slot = nullptr;
    int32_t* perm = nullptr;     // perm[new] = old
    int32_t* pair_tgt = nullptr;
    int32_t* pair_seg = nullptr;  // seg_begin
    int64_t* pair_rel = nullptr;  // rel_off
    uint8_t* pair_excl = nullptr; // 1 if no other source of the level shares the target
    int32_t* rel = nullptr;
    int32_t* level_sn = nullptr;
    SmallRec* small_rec = nullptr;  // aligned with level_sn
    int32_t* big_sn = nullptr;   // every large supernode, level by level
    int64_t nbig = 0;
    int32_t big_maxw = 0;        // widest large supernode
    RowBlock* rowblk = nullptr;
    UpdTile* tiles = nullptr;
    // device task-queue schedule (only when analyzed with sched 2)
    Task* tasks = nullptr;
    int64_t ntasks = 0;
    std::vector<Task> host_tasks;  // the task order, kept for the execution log
    int32_t* cnt0 = nullptr;     // per supernode: update tiles that scatter into it
    int32_t* rb_base = nullptr;  // per supernode: index of its first panel row block
    int64_t nrowblk = 0;
    int32_t max_w = 0;
    // deterministic scatter order (analysis option deterministic = 1)
    int32_t* pair_src = nullptr;  // source supernode of each pair
    int32_t* pair_end = nullptr;  // seg_end of each pair
    int64_t* scr_off = nullptr;   // sources in the apply form: offset of the update block
                                  // in the level's scratch (-1: none)
    int32_t* app_t = nullptr;     // apply items: target supernode of item k
    int32_t* app_rb = nullptr;    // and the 64-row block of the target it covers
    int64_t* app_p0 = nullptr;    // entries of item k: app_ent[app_p0[k] .. app_p0[k + 1])
    AppEnt* app_ent = nullptr;    // in increasing source order
    // solves: a contribution slot per entry of `rows` (each source's rows
    // below its diagonal block); rows several sources of a level share are
    // reduced after the level, sources in increasing order
    uint8_t* slot_shared = nullptr;  // per slot: its row is shared inside the level
    int32_t* red_row = nullptr;      // reduce items: row
    int64_t* red_ptr = nullptr;      // slots of item k: red_slot[red_ptr[k] .. red_ptr[k + 1])
    int32_t* red_slot = nullptr;
    ColBlk* colblk = nullptr;        // backward (column group, row chunk) blocks
    RowBlock* fwdblk = nullptr;      // forward (supernode, 64-row block) blocks
    RowBlock* sspart = nullptr;      // (supernode, 16-row part of its diagonal block)
    int64_t* pb_off = nullptr;       // per supernode: its partial sums (chunk h, column k at
                                     // pb_off + h w + k) in the backward work
    int64_t nslots = 0;              // entries of rows
    int64_t pb_total = 0;
    std::vector<int64_t> red_level_ptr, colblk_ptr, fwdblk_ptr;  // per level
    std::vector<int64_t> sspart_ptr;  // per level
    // the tail's solve tasks: levels [tail_l0, levels) (none: tail_l0 = levels)
    int32_t tail_l0 = 0;
    int32_t ntail = 0;               // supernodes in the tail
    TailTask* tail_tasks = nullptr;
    int64_t ntail_tasks = 0;
    int64_t ntail_fwd = 0;           // forward tasks come first
    TailSeg* tail_segs = nullptr;
    std::vector<std::vector<int64_t>> round_ptr;  // per level: tile ranges of its rounds
    std::vector<uint8_t> level_apply;    // per level: large sources in the apply form
    std::vector<int64_t> app_ptr;        // per level: its apply items
    int64_t det_scratch = 0;             // elements of the per-level update scratch
    // host-side launch bookkeeping per level; inside each level of level_sn
    // the large supernodes come first, then the small ones
    std::vector<int32_t> level_nbig;
    std::vector<int64_t> rowblk_ptr, tile_ptr;
    std::vector<int64_t> tile_crit;   // per level: leading tiles that feed level l + 1
    std::vector<int32_t> level_maxw;  // widest large supernode of the level
    std::vector<int32_t> small_maxw, small_maxr, small_maxm;  // widest / tallest (below, all) small
                                                              // supernode of the level
};


// Forward contribution slots: (L21 y_s)[i] of a row that several sources of
// the level share goes to cb (nslots x nrhs) at the row's slot; the others
// are subtracted from y directly.
template <class R>
struct SolveBufs {
    R* cb;
    int64_t nslots;
    const uint8_t* shared;
};

// Pointer bundle passed by value to kernels.
struct KArgs {
    const int32_t* sn_first;
    const int32_t* sn_w;
    const int32_t* sn_ld;
    const int64_t* sn_off;
    const int64_t* inv_off;
    const int64_t* rowptr;
    const int32_t* rows;
    const int32_t* rowpair;
    const int32_t* pair_tgt;
    const int32_t* pair_seg;
    const int64_t* pair_rel;
    const int32_t* rel;
};

}  // namespace spc

struct spc_symbolic {
    spc::Symbolic S;
    int refs = 0;  // live numeric factors
    std::mutex mu;
    std::vector<spc::DevicePlan*> plans;  // one per device that used it
    size_t plan_bytes_estimate = 0;
    int64_t det_scratch = 0;  // elements of a factor's update scratch (deterministic order)
    int64_t budget = 0;  // mem_budget_bytes of the options (0 = none)
};

struct spc_numeric {
    spc_symbolic* sym = nullptr;
    spc::DevicePlan* plan = nullptr;
    int device = -1;
    int32_t prec = 0;               // 0: FP64 factor; 1: FP32 factor (FP64 refinement)
    void* arena = nullptr;          // supernode blocks, double or float by prec
    void* dinv = nullptr;           // inverses of the kPanel diagonal blocks, same type
    int32_t* status_dev = nullptr;  // [0] failing column (INT32_MAX = none), [1] FP64 fallbacks
    void* work = nullptr;           // solve vectors y and t, n x work_cols each, factor type
    int32_t sched = 0;              // 0 level sets, 1 level sets with lookahead
    hipStream_t bulk = nullptr;     // second stream for the lookahead schedule
    std::vector<hipEvent_t> sync_ev; // per-level ordering events between the two streams
    hipStream_t capture = nullptr;  // stream the solve sweeps are captured on
    int32_t* sched_state = nullptr; // task-queue counters: cntF, doneF, doneT, ticket/abort/err
    bool det = false;               // deterministic contribution order
    void* det_scratch = nullptr;    // small sources' update blocks of one level (factor type)
    int32_t* task_log = nullptr;    // sched 2 with debug bit 1: start and finish stamps per task
    int64_t spin_limit = 0;
    struct SolveGraph { int32_t nrhs; hipGraph_t graph; hipGraphExec_t exec; };
    std::vector<SolveGraph> solve_graphs;
    // level-set factorization launches (after the value load), captured once
    hipGraph_t factor_graph = nullptr;
    hipGraphExec_t factor_exec = nullptr;
    int64_t work_cols = 0;
    hipStream_t stream = nullptr;
    int32_t host_status = 0;
    bool status_known = false;  // host_status holds the current factorization's status
    bool factored = false;
    // iterative refinement (FP64): symmetric matrix in full CSR form, values
    // gathered from the caller's array at every factorization
    int64_t a_nnz = 0;              // entries of the full CSR
    int64_t* a_ptr = nullptr;       // n + 1
    int32_t* a_col = nullptr;       // nnz_full
    int64_t* a_src = nullptr;       // nnz_full: input entry of each CSR entry
    double* a_val = nullptr;        // nnz_full
    double* a_norm = nullptr;       // ||A_k||_inf per matrix of the batch
    int32_t* a_seg = nullptr;       // batch matrix of every row (null for one matrix)
    int64_t nseg = 1;
    double* ir_work = nullptr;      // residuals n x ir_cols, then 4 x ir_cols norms/scales
    int64_t ir_cols = 0;
    double* ir_host = nullptr;      // pinned: backward errors of the current iterate
    // FP64 factor of the same matrix for refinement that stalls on an FP32
    // factor: made on first need from the refinement copy of A, reused until
    // the next factorization of this object
    spc_numeric* fb = nullptr;
    double* fb_values = nullptr;    // A's values in the caller's order (nnz_a)
    bool fb_current = false;
    int64_t refine_fallbacks = 0;   // refinement solves that switched to fb
    // optional per-launch event timing (class, start, stop)
    bool timing = false;
    std::vector<hipEvent_t> events;
    struct Mark { int cls; int a, b; };
    std::vector<Mark> marks;
    size_t next_event = 0;
};

namespace spc {

// Device bytes of the plan; *det_scratch (may be null) receives the elements
// of the per-level update scratch of the deterministic order.
size_t plan_bytes(const Symbolic& S, int64_t* det_scratch);
int32_t build_task_order(const Symbolic& S, int workers, std::vector<Task>& order,
                         std::vector<int32_t>& cnt0, std::vector<int32_t>& rb_base);
int64_t inverse_blocks_elems(const Symbolic& S);
KArgs kargs(const DevicePlan* P);
int32_t get_plan(spc_symbolic* sym, DevicePlan** out);
void free_plan(DevicePlan* p);
int32_t run_factor(spc_numeric* num, const double* values, hipStream_t stream);
int32_t run_solve(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                  int64_t ldx, hipStream_t stream);
// Solve sweeps on the internal vectors after they hold the permuted right-hand sides.
int32_t run_sweeps(spc_numeric* num, int32_t nrhs, hipStream_t stream);
int32_t ensure_solve_work(spc_numeric* num, int32_t nrhs);
int32_t run_refine(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                   int64_t ldx, double tol, int32_t max_iter, hipStream_t stream,
                   int32_t* iters, double* berr);
// Gathers the caller's values into the refinement copy of A (FP64).
int32_t load_refine_matrix(spc_numeric* num, const double* values, hipStream_t stream);
int32_t numeric_create_prec(spc_symbolic* sym, int32_t prec, spc_numeric** out);
void free_refine(spc_numeric* num);
void drop_solve_graphs(spc_numeric* num);
// Small-supernode kernels (one wave per supernode of list[0 .. count)).
void launch_small_factor(spc_numeric* num, const KArgs& a, const int32_t* list, int count,
                         int maxw, int maxr, int maxm, hipStream_t st);
// Deterministic order: apply items [i0, i1) of the plan (one wave per shared
// target adds the level's small sources' blocks from the scratch in order).
void launch_small_apply(spc_numeric* num, int64_t i0, int64_t i1, hipStream_t st);
// y: the solve vector; cb: the forward contribution slots (factor type).
void launch_small_solve(spc_numeric* num, const KArgs& a, const SmallRec* recs, int count,
                        int maxw, int maxm, void* y, void* cb, int64_t n, int nrhs, bool forward,
                        hipStream_t st);
// Elements of the solve work (y, contribution slots, backward partial sums)
// for nrhs right-hand sides.
int64_t solve_work_elems(const spc_numeric* num, int32_t nrhs);
int64_t solve_work_elems_per_rhs(const Symbolic& S);
// First level of the solves' tail (levels when there is none).
int32_t tail_start(const Symbolic& S);
// Backward partial sums per right-hand side: kRowChunk-row chunks of the
// large supernodes below the tail, kTile-row blocks of the tail's.
int64_t solve_pb_elems(const Symbolic& S);
// int32 words of the tail's task state (four counters per supernode, the
// ticket and the abort and error words), at the end of the solve work.
int64_t tail_state_words(const Symbolic& S);
// int32 words of the split level launches' counts (forward and backward per
// supernode, then three control words: unused, abort, error, as the tail's
// waits address them), after the tail's.
int64_t split_state_words(const Symbolic& S);

}  // namespace spc
