/*
 * spchol -- supernodal sparse Cholesky factorization and solve on one AMD
 * Instinct MI355X (gfx950), C ABI.
 *
 * Problem (arXiv:1608.00044, Section II-A, equation (1)): A is an n x n
 * symmetric positive definite matrix; after a fill-reducing symmetric
 * permutation P (Section V, nested dissection), factor P A P^T = L L^T with L
 * lower triangular and only L stored, then solve A x = b with the two
 * triangular solves L y = P b, L^T z = y, x = P^T z (Section II-A).
 *
 * The work is split in three calls:
 *   spc_analyze  -- host-only symbolic analysis: elimination tree and column
 *                   counts (Section II-B), supernodes (Section II-B) capped at
 *                   opt.sn_cap columns (Section III-B, 150 by default),
 *                   optional relaxed amalgamation, storage layout, relative
 *                   indices for the update scatter, task schedule;
 *   spc_factor   -- device numeric factorization: per supernode the diagonal
 *                   factorization and panel solve (task F of Section III-A),
 *                   the update blocks to every later supernode it touches
 *                   (task U) and their scatter-add into the target through
 *                   relative indices (task A), run in a dependency order of
 *                   the supernodal elimination tree (Section IV);
 *   spc_solve    -- device forward and backward supernodal triangular solves.
 *
 * Conventions used by every entry point:
 *   - Matrices are the LOWER triangle of A in compressed sparse column form,
 *     0-based: colptr[n+1] (int64), rowind[nnz] (int32).  Every column holds
 *     its row indices in strictly increasing order, every row index i of
 *     column j satisfies j <= i < n.  Upper-triangle entries, duplicates and
 *     unsorted rows are rejected with SPC_ERR_PATTERN.  A missing diagonal is
 *     a structural zero: the factorization then reports that column.
 *   - perm[new] = old: (P A P^T)[i][j] = A[perm[i]][perm[j]].  NULL means the
 *     identity.  The library uses exactly this permutation (no internal
 *     reordering), so its L is comparable with any other factor of P A P^T.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are memory on
 *     the current HIP device (for example torch tensor data_ptr()); "stream"
 *     is a hipStream_t passed as void* (NULL = the default stream).
 *   - Values are IEEE binary64.  values[k] belongs to the input entry
 *     (rowind[k], column of k) of the pattern given to spc_analyze.
 *   - Status: 0 success; > 0 the 1-based column of P A P^T whose pivot was not
 *     positive (or not a number), the smallest such column; < 0 an error code
 *     below.  Invalid arguments are rejected before any device work.
 *   - Handles are not thread-safe; distinct handles may be used concurrently
 *     from different threads.
 */
#ifndef SPCHOL_H
#define SPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spc_status;

enum {
    SPC_OK = 0,
    SPC_ERR_ARG = -1,           /* bad argument (NULL, size, options)               */
    SPC_ERR_PATTERN = -2,       /* malformed lower CSC pattern                      */
    SPC_ERR_OOM = -3,           /* host or device allocation failed / over budget   */
    SPC_ERR_HIP = -4,           /* a HIP runtime call failed                        */
    SPC_ERR_NOT_FACTORED = -5,  /* solve on a factor that did not complete          */
    SPC_ERR_NOT_CONVERGED = -6, /* reserved for iterative refinement                */
    SPC_ERR_TIMEOUT = -7,       /* a device wait exceeded its bounded spin          */
    SPC_ERR_BUSY = -8,          /* symbolic handle still referenced by a factor     */
    SPC_ERR_TOO_LARGE = -9      /* the work does not fit spc_solve_noalloc's scratch */
};

typedef struct spc_options {
    int32_t sn_cap;           /* maximum supernode width, 1..150 columns; default 150 */
    int32_t sched;            /* 0 = level by level; 1 = level by level with a
                                 one-level lookahead on two streams; 2 = device task
                                 queue (dependency counters, Section IV)        */
    double amalg_ratio;       /* relaxed amalgamation zero ratio; 0 = off (default) */
    int64_t mem_budget_bytes; /* device bytes a factor may hold; 0 = no limit       */
    int64_t spin_limit;       /* bound on every device wait, in microseconds: sched 2
                                 (past it the factorization stops and its status
                                 reads SPC_ERR_TIMEOUT) and the solves' level
                                 launches (past it the solution holds NaN); 0 =
                                 default (ten seconds)                          */
    int32_t debug_flags;      /* bit 0: withhold one dependency count (sched 2) and
                                 one count of every solve wait, so that the bounded
                                 waits fire (testing only); bit 1: sched 2
                                 records when every task starts and finishes
                                 (spc_numeric_task_log); default 0               */
    int32_t precision;        /* 0 = FP64 factor (default); 1 = FP32 factor on FP32
                                 matrix cores with FP32 accumulation, for use with
                                 spc_solve_refine (FP64 iterative refinement)     */
    int32_t threads;          /* host threads of spc_analyze_batch (matrices are
                                 analysed side by side); 0 = default: the host's
                                 hardware threads, at most 16                     */
    int32_t small_w;          /* level-set schedules: supernodes of at most small_w
                                 columns and small_r rows below the diagonal block
                                 are factored and solved by a lane group each, the
                                 others by workgroup kernels on 64 x 64 tiles.
                                 small_w 1..16, or -1 for none; 0 = default (16) */
    int32_t small_r;          /* 1..64; 0 = default (64)                           */
    int32_t deterministic;    /* 1 (default): every target supernode receives its
                                 update contributions in one fixed order -- level
                                 by level, and inside a level the sources in
                                 increasing order (the non-decreasing (target,
                                 source) order of Section III-D) -- so a factor
                                 has the same bits on every run, alone or beside
                                 other work.  0: contributions to a target that
                                 several sources of a level share are atomic adds
                                 in arrival order (equal to rounding).  With
                                 sched 1 the lookahead is then off (one stream,
                                 level by level); sched 2 requires 0 (its queue
                                 order is dynamic): SPC_ERR_ARG otherwise.      */
    int32_t workers;          /* sched 2: persistent workgroups taking tasks;
                                 0 = as many as fit on the device at once        */
    int32_t solve_tail;       /* 1: with deterministic = 0, the solves' top
                                 levels of the supernodal elimination tree
                                 (levels above the last one with more than 128
                                 supernodes or any small one) run as one
                                 persistent launch of dependent tasks, the
                                 counters of Section IV applied to the two
                                 solves (forward updates by atomic adds);
                                 0 (default): every level as its own launches,
                                 which measures faster on MI355X (a task's
                                 signal costs a device-scope memory round trip,
                                 about as much as a launch)                     */
    int32_t upd_chunk;        /* update tiles (Section III-A, U and A tasks):
                                 columns of the source panel staged through LDS
                                 per step, 8, 16 or 32; 0 = default (16).  A
                                 tile shape the batch autotuner searches; every
                                 value computes the same products in the same
                                 order                                          */
} spc_options;

typedef struct spc_symbolic spc_symbolic;
typedef struct spc_numeric spc_numeric;

typedef struct spc_symbolic_info {
    int64_t n;             /* order of A                                            */
    int64_t nnz_a;         /* stored entries of the lower triangle of A            */
    int64_t nnz_l;         /* entries of the exact structure of L                   */
    int64_t nnz_stored;    /* entries the supernodal storage holds (>= nnz_l)       */
    int64_t nsup;          /* supernodes after cap split and amalgamation           */
    int64_t nlevels;       /* levels of the supernodal elimination tree             */
    int64_t npairs;        /* (source, target) update pairs                         */
    int64_t nrel;          /* relative indices stored for the scatter              */
    int64_t factor_bytes;  /* device bytes one numeric factor holds                */
    int64_t plan_bytes;    /* device bytes of the shared symbolic plan             */
    double flops;          /* sum_j colcount(j)^2 over the exact structure          */
    double flops_stored;   /* the same sum over the stored (amalgamated) structure  */
    int32_t max_width;     /* widest supernode                                      */
    int32_t max_below;     /* most rows below a diagonal block                      */
    int64_t nbatch;        /* independent matrices (1 unless spc_analyze_batch)     */
    int64_t solve_bytes_per_rhs; /* device work bytes a solve holds per right-hand side
                                    (solution vector, forward contributions of every
                                    below-diagonal row, backward partial sums), plus
                                    16 (tail_supernodes + 1) bytes once per solve  */
    int32_t tail_levels;   /* top levels whose solves run in the persistent launch
                              (spc_options.solve_tail; 0 = none)                  */
    int32_t tail_supernodes; /* supernodes on those levels                         */
} spc_symbolic_info;

/* Fills *opt with the defaults (sn_cap 150, sched 0, no amalgamation, no budget,
 * default spin limit, no debug flags, default threads and small-supernode
 * limits, deterministic order, default workers). */
void spc_default_options(spc_options* opt);

/* Symbolic analysis on the host (no device work).  colptr/rowind/perm are
 * host arrays borrowed for the call; the pattern is copied into the handle.
 * opt may be NULL (defaults).  On success *out owns the analysis; release it
 * with spc_symbolic_free.  Errors: SPC_ERR_ARG, SPC_ERR_PATTERN, SPC_ERR_OOM. */
spc_status spc_analyze(int64_t n, const int64_t* colptr, const int32_t* rowind,
                       const int32_t* perm, const spc_options* opt, spc_symbolic** out);

spc_status spc_symbolic_info_get(const spc_symbolic* sym, spc_symbolic_info* info);

/* Batched analysis of `count` independent SPD matrices (matrix k: order n[k],
 * lower CSC colptr[k] / rowind[k], optional ordering perm[k] or NULL): one
 * symbolic handle for their block-diagonal direct sum, matrix k taking rows
 * and columns [o_k, o_k + n[k]) with o_k = n[0] + ... + n[k-1].  Its
 * elimination forest is the union of theirs (Section II-B), so supernodes,
 * levels and update pairs never cross two matrices, and one factorization
 * or solve launch covers every matrix.  Values for spc_factor are the
 * matrices' value arrays one after the other; right-hand sides and solutions
 * are the matrices' blocks stacked by rows.  spc_solve_refine measures and
 * meets tol for every matrix separately (berr: count values per column).
 * Every matrix is validated as by spc_analyze; the first failing one (in
 * order) gives the status.  The matrices are analysed on up to opt->threads
 * host threads and the results joined; the handle is the same, field by
 * field, as spc_analyze of the block-diagonal matrix, whatever the count. */
spc_status spc_analyze_batch(int32_t count, const int64_t* n, const int64_t* const* colptr,
                             const int32_t* const* rowind, const int32_t* const* perm,
                             const spc_options* opt, spc_symbolic** out);

/* Host copies of the analysis, for checking.  Each output may be NULL.
 *   parent[n]    elimination tree of P A P^T (-1 = root), Section II-B;
 *   colcount[n]  column counts of L including the diagonal;
 *   sn_ptr[nsup+1] first column of each supernode, then n;
 *   sn_parent[nsup] supernodal elimination tree (-1 = root). */
spc_status spc_symbolic_export(const spc_symbolic* sym, int32_t* parent, int32_t* colcount,
                               int32_t* sn_ptr, int32_t* sn_parent);

/* Supernode row lists: rowptr[nsup+1] (int64) and rows[rowptr[nsup]] (int32):
 * the supernode's own columns, then the sorted rows below its diagonal block.
 * Supernode s stores a column-major (rowptr[s+1]-rowptr[s]) x width block. */
spc_status spc_symbolic_export_rows(const spc_symbolic* sym, int64_t* rowptr, int32_t* rows);

/* Update pairs and relative indices.  For pair p (npairs of them, grouped by
 * source): src[p], tgt[p], seg[2p..2p+1] = [begin, end) of the source's
 * below-diagonal rows that fall in the target's columns, rel_off[p] = offset of
 * the pair's relative indices in rel[nrel]; for every below-diagonal row i of
 * the source with i >= begin, rel[rel_off[p] + i - begin] is that row's
 * position in the target's row list.  Any output may be NULL. */
spc_status spc_symbolic_export_pairs(const spc_symbolic* sym, int32_t* src, int32_t* tgt,
                                     int32_t* seg, int64_t* rel_off, int32_t* rel);

/* Task order of the device task-queue schedule (sched 2), computed on the
 * host for `workers` device workers (> 0).  The tasks follow the paper's
 * factorization, update and aggregation tasks (Section III-A) at tile
 * granularity: kind 0 = F(s) diagonal factorization of supernode s, kind 1 =
 * T(s, a) panel solve of 64-row block a of s, kind 2 = U(s, a, b) the 64 x 64
 * update tile (row block a, column block b, a >= b) of s scatter-added into
 * its targets.  cnt0[t] is the initial dependency counter of F(t)
 * (Section IV): the number of (update tile, distinct target t) pairs.
 * *ntasks receives the task count; tasks (4 int32 per task: kind, s, a, b, in
 * start order) and cnt0 (nsup entries) may be NULL to query the size first.
 * Host only; needs no device. */
spc_status spc_symbolic_export_tasks(const spc_symbolic* sym, int32_t workers, int64_t* ntasks,
                                     int32_t* tasks, int32_t* cnt0);

/* Releases the handle.  Returns SPC_ERR_BUSY (and frees nothing) while a
 * numeric factor created from it is alive.  NULL is accepted. */
spc_status spc_symbolic_free(spc_symbolic* sym);

/* Numeric factorization on the current HIP device, ordered on stream.
 * values_dev: device array of nnz_a doubles aligned with the analyzed pattern.
 * The call returns once the work is enqueued; the factor status becomes known
 * through spc_numeric_status (which synchronizes) or the next spc_solve.  On
 * success *out owns the factor's device memory; it references sym, so free it
 * first.  Errors: SPC_ERR_ARG, SPC_ERR_OOM (allocation or mem_budget_bytes),
 * SPC_ERR_HIP. */
spc_status spc_factor(const spc_symbolic* sym, const double* values_dev, void* stream,
                      spc_numeric** out);

/* Factor again with fresh values on the same pattern, reusing num's memory:
 * the symbolic analysis (Section II-B) depends on the pattern alone, so only
 * the numeric tasks of Section III-A run again.  values_dev, stream, status
 * and errors as spc_factor. */
spc_status spc_refactor(spc_numeric* num, const double* values_dev, void* stream);

/* Synchronizes the factor's stream and returns its status: 0, the 1-based
 * failing pivot column (> 0: the diagonal entry under the square root of
 * equation (1)'s column recurrence was not positive, so A is not positive
 * definite), SPC_ERR_TIMEOUT or SPC_ERR_HIP. */
spc_status spc_numeric_status(spc_numeric* num);

/* x = A^{-1} b for nrhs right-hand sides: b_dev and x_dev are column-major
 * device arrays (leading dimensions ldb, ldx >= n) of doubles; x_dev may equal
 * b_dev when ldx == ldb.  Synchronizes on the factor status first: a failed
 * factor returns its status (> 0) and leaves x_dev untouched.  Enqueued on
 * stream, otherwise asynchronous.  The workgroups of a level wait on each
 * other through device-side counts (bounded by spin_limit); a wait past its
 * bound leaves NaN in x_dev. */
spc_status spc_solve(spc_numeric* num, int32_t nrhs, const double* b_dev, int64_t ldb,
                     double* x_dev, int64_t ldx, void* stream);

/* spc_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result, bit for bit, with the solve's work (the solution vector,
 * the forward contributions and the backward partial sums, sized by
 * spc_symbolic_info.solve_bytes_per_rhs times nrhs, plus the persistent
 * launch's counters) in one static device
 * array of 64 MiB that each device holds from the library's load until the
 * process ends, instead of the factor's allocated work, and the level sweeps
 * launched directly on stream instead of replayed from a graph.  It allocates
 * nothing (no hipMalloc, hipFree or graph instantiation); the factor itself
 * comes from spc_factor.  Work larger than the array: SPC_ERR_TOO_LARGE,
 * before any device work.  Every call on a device shares that device's array,
 * so calls that overlap on one device (different streams or threads) race.
 * Arguments, status and synchronization as spc_solve. */
spc_status spc_solve_noalloc(spc_numeric* num, int32_t nrhs, const double* b_dev, int64_t ldb,
                             double* x_dev, int64_t ldx, void* stream);

/* Host copy of the factor in the stored (supernodal) column structure:
 * Sp[n+1] (int64) and Si (int32) give, for column j of supernode s, the rows
 * j..last(s) then the rows below the supernode's diagonal block; Sx holds the
 * values.  Entries outside the exact structure of L are explicit zeros: the
 * stored structure is that of the amalgamated supernodes (Section II-B), a
 * superset of the exact structure; L itself is the unique factor of
 * equation (1).
 * Synchronizes.  Any output may be NULL; sizes are n+1 and nnz_stored. */
spc_status spc_factor_export(spc_numeric* num, int64_t* Sp, int32_t* Si, double* Sx);

/* Mixed-precision solve: iterative refinement in FP64 around the factor
 * (an extension of the solves of Section II-A; the paper works in one
 * precision).  x_0 = 0; each step forms r = b - A x in FP64 from a copy of A
 * taken at factorization time, the normwise backward error
 * eta_c = ||r_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf) of every column,
 * and, while some eta_c > tol, solves L L^T d = r / ||r|| in the factor's
 * precision and adds ||r|| d to x in FP64.  Two steps in a row in which the
 * worst eta does not halve count as a stall: on an FP32 factor the
 * corrections then continue with an FP64 factor of the same matrix (made
 * from the copy of A on first need, kept until the next factorization, about
 * twice the FP32 factor's bytes; counted in spc_numeric_info's
 * refine_fallbacks); on an FP64 factor the refinement stops.  b_dev, x_dev:
 * column-major device arrays (ldb, ldx >= n) of doubles that must not
 * overlap.  Returns SPC_OK once every column meets tol,
 * SPC_ERR_NOT_CONVERGED after max_iter corrections (FP32 and FP64 ones
 * together) or a stall of the FP64 corrections (x holds the last iterate),
 * the FP64 fallback factor's status, or the factor's status.  *iters
 * (may be NULL) receives the number of corrections; berr (host, may be NULL)
 * the final eta: nrhs entries, or for a batch analysis nrhs x nbatch entries
 * (berr[c * nbatch + k]: matrix k, column c), each matrix's norms taken over
 * its own rows.  Synchronizes stream once per step. */
spc_status spc_solve_refine(spc_numeric* num, int32_t nrhs, const double* b_dev, int64_t ldb,
                            double* x_dev, int64_t ldx, double tol, int32_t max_iter,
                            void* stream, int32_t* iters, double* berr);

/* Facts about a numeric factor.  fp64_blocks: for an FP32 factor, the number
 * of diagonal blocks whose FP32 factorization met a pivot at most 1e-3 times
 * its starting diagonal entry and that were factored again in FP64 (the
 * result is stored in FP32).  Synchronizes the factor's stream. */
typedef struct spc_numeric_info {
    int32_t precision;     /* 0 FP64, 1 FP32 */
    int32_t sched;
    int64_t factor_bytes;  /* device bytes held by the factor (estimate) */
    int64_t fp64_blocks;
    int64_t refine_fallbacks; /* spc_solve_refine calls that switched to an FP64 factor */
} spc_numeric_info;

spc_status spc_numeric_info_get(spc_numeric* num, spc_numeric_info* out);

/* Per-kernel-class device times of the most recent factorization, measured
 * with HIP events recorded on the factor's stream around every launch while
 * timing is enabled (spc_numeric_set_timing).  Classes: 0 value load (fill +
 * load), 1 diagonal factorization, 2 panel solve, 3 update + scatter, 4 the
 * persistent task-queue kernel (schedule 2: all of 1-3 in one launch), 5 the
 * small-supernode kernel (1-3 for supernodes of at most 16 columns and 64 rows
 * below the diagonal block, one wavefront each).
 * ms[c] is the summed duration of class c, launches[c] its launch count.
 * Synchronizes the stream.  SPC_ERR_ARG if timing was never enabled. */
typedef struct spc_kernel_times {
    double ms[6];
    int64_t launches[6];
    double total_ms; /* from the first to the last recorded event */
} spc_kernel_times;

spc_status spc_numeric_set_timing(spc_numeric* num, int32_t enable);
spc_status spc_numeric_get_timing(spc_numeric* num, spc_kernel_times* out);

/* Execution log of the device task queue (sched 2, analysed with debug_flags
 * bit 1): *ntasks tasks in ticket order (tasks: 4 int32 each, kind, s, a, b,
 * as spc_symbolic_export_tasks) and, per task, two stamps of one device
 * clock: stamps[2q] when task q's inputs were complete (its dependency waits
 * over, Section IV), stamps[2q + 1] when its results were written, before
 * its successors were signalled.  A correct run has every stamp of a task
 * above the finishing stamp of each task it depends on.  tasks and stamps
 * may be NULL (query the count first).  Synchronizes.  SPC_ERR_ARG without a
 * log. */
spc_status spc_numeric_task_log(spc_numeric* num, int64_t* ntasks, int32_t* tasks,
                                int32_t* stamps);

/* Releases the factor's device memory (synchronizing its stream). NULL is accepted. */
void spc_numeric_free(spc_numeric* num);

/* Measurement helper (not part of the method): what the current device's
 * matrix cores and HBM deliver to kernels that do nothing else -- 16 x 16 x 4
 * FP64 and FP32 matrix-core products issued from registers (8 independent
 * accumulators per wave, 8 waves per SIMD) and a 512 MiB streaming copy
 * (bytes read + written per second).  Allocates 1 GiB for the copy and
 * synchronizes the device. */
typedef struct spc_ceilings {
    double fp64_mfma_tflops, fp32_mfma_tflops, copy_gbs;
} spc_ceilings;

spc_status spc_measure_ceilings(spc_ceilings* out);

/* Static English text for a status code. */
const char* spc_status_string(spc_status st);

/* ------------------------------------------------------------------------
 * Request server (continuous batching over resident patterns)
 *
 * Serves factor+solve and solve-only requests on the current device.  Each
 * added pattern keeps numeric factors resident in HBM; a factor+solve
 * request refactors an idle one of its pattern with fresh values (a new one
 * is created when the predicted bytes, spc_symbolic_info.factor_bytes plus
 * work vectors for max_nrhs columns, fit the budget after evicting idle
 * factors least recently used first) and solves; a completed, successful
 * factorization becomes the pattern's current factor, which solve-only
 * requests use.  Up to max_inflight requests run at once on separate
 * streams, so their kernels overlap on the device; requests that arrive
 * meanwhile are admitted in arrival order as slots and memory free up.  A
 * worker thread schedules; submit and wait are thread safe.  The caller's
 * device buffers (values, b, x) must stay valid until the request's wait
 * returns.  A request's device work is ordered after everything enqueued on
 * its `stream` before spc_server_submit (an event recorded there at
 * submission), so values, b and x may still be being written on that stream.  This extends the paper's factor/solve split (Section II-A) to a
 * stream of requests; the paper itself serves none.
 * ------------------------------------------------------------------------ */
typedef struct spc_server spc_server;

typedef struct spc_server_options {
    int32_t max_inflight;      /* requests on the device at once, 1..64 (default 8)  */
    int32_t max_nrhs;          /* most right-hand sides of one request (default 64) */
    int64_t mem_budget_bytes;  /* bytes for resident factors and their work vectors;
                                  0 = 80% of the device's free memory at creation   */
} spc_server_options;

typedef struct spc_request {
    int32_t pattern;        /* from spc_server_add_pattern                           */
    int32_t kind;           /* 0: factor `values` then solve; 1: solve with the
                               pattern's current factor                              */
    int32_t nrhs;           /* 0..max_nrhs                                           */
    int32_t reserved;
    const double* values;   /* device, nnz_a values of the pattern (kind 0)          */
    const double* b;        /* device, column-major n x nrhs, leading dimension ldb  */
    int64_t ldb;
    double* x;              /* device, column-major n x nrhs, leading dimension ldx  */
    int64_t ldx;
    void* stream;           /* hipStream_t that produced values / b and last used x
                               (NULL = the default stream)                           */
} spc_request;

typedef struct spc_request_result {
    int32_t status;         /* 0; a failed pivot column (> 0, kind 0); SPC_ERR_OOM (the
                               pattern cannot fit the budget); SPC_ERR_NOT_FACTORED
                               (kind 1 with no current factor); SPC_ERR_HIP         */
    int32_t reserved;
    double queue_ms;        /* submit to admission                                   */
    double latency_ms;      /* submit to completion of its device work               */
} spc_request_result;

/* bytes_in_use and peak_bytes count the resident factors with their work
 * vectors, plus each pattern's device plan from its first factor on (plans
 * stay until the symbolic handle is freed, so eviction does not return them). */
typedef struct spc_server_stats {
    int64_t submitted, completed, rejected, evictions;
    int64_t bytes_in_use, peak_bytes, budget_bytes;
    int32_t peak_inflight, resident_factors;
} spc_server_stats;

void spc_server_default_options(spc_server_options* opt);
spc_status spc_server_create(const spc_server_options* opt, spc_server** out);
/* Registers a symbolic handle and makes its device plan on the server's
 * device now (SPC_ERR_OOM if it does not fit), so that the pattern's first
 * request does not build it.  The server holds a reference to the handle
 * until spc_server_destroy: spc_symbolic_free returns SPC_ERR_BUSY meanwhile. */
spc_status spc_server_add_pattern(spc_server* srv, spc_symbolic* sym, int32_t* pattern);
/* Queues a request; *ticket identifies it.  SPC_ERR_ARG on bad sizes. */
spc_status spc_server_submit(spc_server* srv, const spc_request* req, int64_t* ticket);
/* Blocks until the request has completed; fills *out (may be NULL) and
 * forgets the ticket. */
spc_status spc_server_wait(spc_server* srv, int64_t ticket, spc_request_result* out);
spc_status spc_server_stats_get(spc_server* srv, spc_server_stats* out);
/* Completes every queued request, then frees the resident factors. */
spc_status spc_server_destroy(spc_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* SPCHOL_H */
