// Host symbolic analysis for the supernodal Cholesky factorization.
//
// Everything here is integer work on the host: input checks, the symmetric
// permutation C = lower(P A P^T), the elimination tree (Section II-B), column
// counts, the supernode partition (Section II-B) with the 150-column cap
// (Section III-B) and relaxed amalgamation, supernode row structures, the
// device storage layout, relative indices for the update scatter (the
// aggregation task A of Section III-A) and the level schedule of the
// supernodal elimination tree.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace spc {

struct Options {
    int32_t sn_cap = 150;
    double amalg_ratio = 0.0;
    int32_t sched = 0;
    int32_t debug_flags = 0;  // bit 0: withhold one dependency (exercises the watchdog)
    int64_t spin_limit = 0;   // bounded waits of the task-queue schedule; 0 = default
    int32_t precision = 0;    // 0: FP64 factor; 1: FP32 factor with FP64 refinement
    int32_t small_w = 16;     // supernodes of at most small_w columns and small_r rows
    int32_t small_r = 64;     // below run on the lane-group kernels (small_w 0: none)
    int32_t deterministic = 1; // fixed order of the contributions to every target
    int32_t workers = 0;      // sched 2: persistent workgroups (0 = full occupancy)
    int32_t solve_tail = 0;   // 1: the solves' top levels in one persistent launch; 0: off
    int32_t upd_chunk = 16;   // K columns the update tiles stage per step: 8, 16 or 32
};

// One (source, target) update pair: source supernode s sends its update block
// to target supernode t.  The target's columns meet the source's rows below
// its diagonal block in the contiguous segment [seg_begin, seg_end) of those
// rows (indices into the source's below-diagonal row list); every row from
// seg_begin to the end of that list lands in t.
struct Pair {
    int32_t src, tgt;
    int32_t seg_begin, seg_end;  // in [0, r_src]
    int64_t rel_off;             // rel[rel_off + (i - seg_begin)] for i in [seg_begin, r_src)
};

struct Symbolic {
    int64_t n = 0;
    int64_t nnz_a = 0;
    Options opt;
    // permutation and permuted lower pattern
    std::vector<int32_t> perm;     // perm[new] = old
    std::vector<int64_t> Cp;       // n+1
    std::vector<int32_t> Ci;       // nnz_a
    std::vector<int64_t> amap;     // input entry -> position in C
    // elimination tree and counts (exact structure)
    std::vector<int32_t> parent, colcount, post;
    int64_t nnz_l = 0;             // exact sum of colcounts
    double flops = 0.0;            // exact sum of colcount^2
    // supernodes (after cap split and amalgamation)
    int64_t nsup = 0;
    std::vector<int32_t> sn_ptr;    // nsup+1 first columns
    std::vector<int32_t> sn_parent; // supernodal etree, -1 = root
    std::vector<int32_t> col_owner; // column -> supernode
    std::vector<int64_t> rowptr;    // nsup+1 into rows
    std::vector<int32_t> rows;      // per supernode: its columns, then the rows below
    // storage layout: column-major (nrows x w) block, leading dimension ld
    std::vector<int64_t> off;       // element offset of each block in the arena
    std::vector<int32_t> ld;
    int64_t arena = 0;              // elements
    int64_t nnz_stored = 0;         // sum over columns of stored rows
    double flops_stored = 0.0;      // sum over columns of stored^2
    std::vector<int64_t> slot;      // input entry -> arena element
    // update pairs, grouped by source in increasing target order
    std::vector<int64_t> pair_ptr;  // nsup+1 into pairs
    std::vector<Pair> pairs;
    std::vector<int32_t> rel;       // relative row indices into the target's row list
    // level schedule of the supernodal etree (leaves = level 0)
    std::vector<int32_t> level;     // per supernode
    std::vector<int32_t> level_ptr; // nlevels+1 into level_sn
    std::vector<int32_t> level_sn;  // supernodes grouped by level, increasing index inside
    int32_t max_w = 0, max_r = 0;
    // independent matrices of a batch: matrix k holds rows and columns
    // [batch_ptr[k], batch_ptr[k + 1]) of the block-diagonal whole ({0, n} for one)
    std::vector<int64_t> batch_ptr;

    int32_t width(int64_t s) const { return sn_ptr[s + 1] - sn_ptr[s]; }
    int32_t nrows(int64_t s) const { return (int32_t)(rowptr[s + 1] - rowptr[s]); }
    int32_t nbelow(int64_t s) const { return nrows(s) - width(s); }
};

// Status codes shared with the C ABI.
enum : int32_t {
    OK = 0, ERR_ARG = -1, ERR_PATTERN = -2, ERR_OOM = -3, ERR_HIP = -4,
    ERR_NOT_FACTORED = -5, ERR_NOT_CONVERGED = -6, ERR_TIMEOUT = -7, ERR_BUSY = -8
};

int32_t validate_input(int64_t n, const int64_t* colptr, const int32_t* rowind,
                       const int32_t* perm);

// Full analysis; returns a status code and fills *out.
int32_t analyze(int64_t n, const int64_t* colptr, const int32_t* rowind, const int32_t* perm,
                const Options& opt, Symbolic* out);

// Batched analysis of `count` independent matrices: each analysed alone, up
// to `threads` host threads at a time, then joined into the analysis of their
// block-diagonal direct sum (matrix k at rows and columns [o_k, o_k + n[k])),
// identical, field by field, to analysing that matrix whole, with
// batch_ptr = {o_0, ..., o_count}.  Inputs must have passed validate_input.
int32_t analyze_batch(int32_t count, const int64_t* n, const int64_t* const* colptr,
                      const int32_t* const* rowind, const int32_t* const* perm,
                      const Options& opt, int threads, Symbolic* out);

}  // namespace spc
