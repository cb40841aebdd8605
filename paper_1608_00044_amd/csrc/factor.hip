// Numeric supernodal Cholesky on gfx950: value load and the task kernels, in
// FP64 (v_mfma_f64_16x16x4) or FP32 (v_mfma_f32_16x16x4_f32, FP32
// accumulation) arithmetic; every kernel is a template on the real type R.
//
// Tasks (Section III-A of arXiv:1608.00044), per supernode s of width w with
// r rows below its diagonal block, stored as a column-major (w + r) x w block:
//   F  (k_potrf, k_trsm):  L11 = chol(A11), blocked by 16-column panels in
//                          LDS, then L21 = A21 L11^{-T} on matrix cores using
//                          the inverses of the 16 x 16 diagonal blocks;
//   U  (k_update):         the lower triangle of L21 L21^T in 64 x 64 tiles on
//                          FP64 matrix cores (v_mfma_f64_16x16x4);
//   A  (k_update epilogue): each tile entry is subtracted from the target
//                          supernode that owns its column, at the row given by
//                          the precomputed relative index (an atomic add when
//                          sibling supernodes of one level share the target).
// Dependencies (Section II-C) are met by running the supernodal elimination
// tree level by level: every supernode of level l only receives updates from
// descendants, which all sit on lower levels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "runtime.hpp"

namespace spc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Matrix-core tile 16 x 16 x 4 in FP64 or FP32.  Operands: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16].  The accumulator layouts differ:
// register q of lane l holds D[row(q, l / 16)][l % 16] with row = 4q + l/16 for
// v_mfma_f64_16x16x4_f64 and row = 4 (l/16) + q for v_mfma_f32_16x16x4_f32.
template <class R> struct Mx;
template <> struct Mx<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc mfma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lk) { return 4 * q + lk; }
};
template <> struct Mx<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc mfma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lk) { return 4 * lk + q; }
};

#define HIP_TRY(x)                               \
    do {                                         \
        if ((x) != hipSuccess) return ERR_HIP;   \
    } while (0)

// ---------------------------------------------------------------------------
// value load
// ---------------------------------------------------------------------------

template <class R>
__global__ void k_fill(R* __restrict__ p, int64_t n, R v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// arena[slot[k]] = values[k]: every input entry of A goes to its place in the
// supernodal storage of P A P^T.
template <class R>
__global__ void k_load(const double* __restrict__ values, const int64_t* __restrict__ slot,
                       R* __restrict__ arena, int64_t nnz) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        arena[slot[k]] = (R)values[k];
}

// ---------------------------------------------------------------------------
// F: diagonal block factorization (blocked POTRF)
// ---------------------------------------------------------------------------

// Value of a double held by one lane of the wave (the lane index must be
// wave-uniform): two v_readlane_b32, no LDS round trip.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

constexpr int kPotrfThreads = 256;
constexpr int kDs = kPanel + 1;  // padded row stride of the dense 16 x 16 panel block
// FP32 diagonal factorization: a pivot at most this fraction of the diagonal
// entry it started from (before the block's own elimination) marks the block
// for FP64 (the block lost about log10(1/kPivotTau) digits to cancellation).
constexpr float kPivotTau = 1e-3f;

// 1/sqrt(d) from the hardware estimate refined by two Newton steps, and sqrt(d)
// as d/sqrt(d); within a few units in the last place of the rounded values.
__device__ __forceinline__ void rsqrt_sqrt(double d, double& rs, double& sq) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * (1.5 - 0.5 * d * y * y);
    y = y * (1.5 - 0.5 * d * y * y);
    rs = y;
    sq = d * y;
}
// FP32: the estimate of v_rsq_f32 refined by one Newton step.
__device__ __forceinline__ void rsqrt_sqrt(float d, float& rs, float& sq) {
    float y = __builtin_amdgcn_rsqf(d);
    y = y * (1.5f - 0.5f * d * y * y);
    rs = y;
    sq = d * y;
}

// Column factorization of one panel by one wave, in registers: the jb
// columns j0 .. j0 + jb - 1 over every row from j0 to w - 1 of the packed
// lower triangle T (entry (i, j) at cst(j) + i).  Lane l holds rows
// j0 + l + 64 q (q < NQ, with NQ chunks covering the w - j0 rows).  For each
// column c the pivot comes from the lane that holds row c (v_readlane) and the
// column is scaled by 1/sqrt(pivot).  Columns go in pairs (c, c + 1): column
// c + 1 is updated by column c with L(c + 1, c) read from its lane, then lanes
// 0-15 put both columns' diagonal-block parts L(j0 .. j0 + 15, c .. c + 1) in
// the LDS array colbuf, and every lane reads those values back (same address,
// one broadcast read per pair) to update the panel's later columns.  Entries
// above the diagonal hold garbage in registers and are never stored or
// broadcast.  1/L(c, c) goes to rdiag[c].
// Without kCheck the smallest column with a pivot that is not positive is
// recorded (global column + 1) with atomicMin on *status; with kCheck (FP32
// pass) a pivot at most kPivotTau times its starting diagonal entry d0[c]
// sets *unstable.  kFull: jb == kPanel (every panel but the last).
template <int NQ, bool kFull, class C, bool kCheck, class Cst>
__device__ __forceinline__ void panel_columns_q(C* __restrict__ T, C* __restrict__ rdiag,
                                                C* __restrict__ colbuf, Cst cst, int w, int j0,
                                                int jb, int lane, int first,
                                                int32_t* __restrict__ status,
                                                const C* __restrict__ d0, int* unstable) {
    C x[NQ][kPanel];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int k = 0; k < kPanel; ++k) {
            const int i = j0 + lane + 64 * q;
            const bool in = (kFull || k < jb) && i < w && i >= j0 + k;
            x[q][k] = T[in ? cst(j0 + k) + i : 0];
            if (!in) x[q][k] = C(0);
        }
    const C piv0 = kCheck ? kPivotTau * d0[lane < jb ? j0 + lane : 0] : C(0);
    C rsv = C(0);   // lane k keeps 1/L(j0 + k, j0 + k)
    int bad = kPanel;  // first failing column of the panel
    // column k: pivot, square root, scaling (lane k keeps L(k, k))
    auto factor_column = [&](int k) {
        const C d = lane_value(x[0][k], k);
        const bool fail = kCheck ? !(d > lane_value(piv0, k)) : !(d > C(0));
        bad = (fail && bad == kPanel) ? k : bad;
        C rs, l;
        rsqrt_sqrt(d, rs, l);
        rsv = lane == k ? rs : rsv;
        x[0][k] = lane == k ? l : x[0][k] * rs;
#pragma unroll
        for (int q = 1; q < NQ; ++q) x[q][k] *= rs;
    };
    // Two columns per step: column k + 1 takes column k's term through a
    // register broadcast of L(k + 1, k), then both columns go through colbuf
    // once for the later columns.  Every product and its order are those of
    // the column-by-column form (column k's term first).
#pragma unroll
    for (int k = 0; k < kPanel; k += 2) {
        const bool has1 = kFull || k + 1 < jb;
        if (kFull || k < jb) {
            factor_column(k);
            if (has1) {
                const C a = lane_value(x[0][k], k + 1);
#pragma unroll
                for (int q = 0; q < NQ; ++q) x[q][k + 1] -= x[q][k] * a;
                factor_column(k + 1);
            }
            if (k + 2 < kPanel && (kFull || k + 2 < jb)) {
                if (lane < kPanel) {
                    colbuf[k * kPanel + lane] = x[0][k];
                    colbuf[(k + 1) * kPanel + lane] = x[0][k + 1];
                }
                __builtin_amdgcn_wave_barrier();
                C l0[kPanel], l1[kPanel];
#pragma unroll
                for (int j = k + 2; j < kPanel; ++j) {
                    l0[j] = colbuf[k * kPanel + j];
                    l1[j] = colbuf[(k + 1) * kPanel + j];
                }
#pragma unroll
                for (int j = k + 2; j < kPanel; ++j) {
                    if (kFull || j < jb) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            x[q][j] -= x[q][k] * l0[j];
                            x[q][j] -= x[q][k + 1] * l1[j];
                        }
                    }
                }
            }
        }
    }
    if (lane < jb) rdiag[j0 + lane] = rsv;
    if (bad < kPanel && lane == 0) {
        if (kCheck) *unstable = 1;
        else atomicMin(status, first + j0 + bad + 1);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int k = 0; k < kPanel; ++k) {
            const int i = j0 + lane + 64 * q;
            if ((kFull || k < jb) && i < w && i >= j0 + k) T[cst(j0 + k) + i] = x[q][k];
        }
}

// Panel j0 of width jb: the register factorization sized to its rows (kW:
// the widest block the instance handles; at most 64 needs one row chunk).
template <class C, bool kCheck, int kW, class Cst>
__device__ __forceinline__ void panel_columns(C* __restrict__ T, C* __restrict__ rdiag,
                                              C* __restrict__ colbuf, Cst cst, int w, int j0,
                                              int jb, int lane, int first,
                                              int32_t* __restrict__ status,
                                              const C* __restrict__ d0, int* unstable) {
    static_assert(kMaxWidth <= 192, "three 64-row chunks per lane");
    const int rows = w - j0;
#define SPC_PANEL(NQ, FULL)                                                                   \
    panel_columns_q<NQ, FULL, C, kCheck>(T, rdiag, colbuf, cst, w, j0, jb, lane, first, status, \
                                         d0, unstable)
    if (jb < kPanel) {  // the last panel: fewer than 16 rows
        SPC_PANEL(1, false);
    } else if (kW <= 64 || rows <= 64) {
        SPC_PANEL(1, true);
    } else if constexpr (kW > 64) {
        if (rows <= 128) SPC_PANEL(2, true);
        else SPC_PANEL(3, true);
    }
#undef SPC_PANEL
}

// Inverses of the diagonal blocks of every panel (lower triangular, jb x jb),
// all at once: lane 16 g + c of wave v takes column c of panel 4 v + g (and
// panel 4 v + g + 16 k beyond that) and forms it by forward substitution,
// row by row, with the row's entries loaded before its products.  Written
// compactly (row major, stride jb) to inv_g at p * 256.
template <class C, class S, class Cst>
__device__ __forceinline__ void panel_inverses(const C* __restrict__ T,
                                               const C* __restrict__ rdiag, S* __restrict__ inv_g,
                                               Cst cst, int w, int npanel, int wave, int lane) {
    const int c = lane & 15;
    for (int p = 4 * wave + (lane >> 4); p < npanel; p += 16) {
        const int j0 = p * kPanel, jb = min(kPanel, w - j0);
        C x[kPanel];
#pragma unroll
        for (int rr = 0; rr < kPanel; ++rr) {
            C lrow[kPanel];
#pragma unroll
            for (int k = 0; k < kPanel; ++k) {
                const bool in = k < rr && rr < jb;
                lrow[k] = T[in ? cst(j0 + k) + j0 + rr : 0];
                if (!in) lrow[k] = C(0);
            }
            C acc = (rr == c) ? C(1) : C(0);
#pragma unroll
            for (int k = 0; k < kPanel; ++k)
                if (k < rr) acc -= lrow[k] * x[k];
            x[rr] = rr < jb ? acc * rdiag[rr < jb ? j0 + rr : 0] : C(0);
        }
        if (c < jb) {
#pragma unroll
            for (int rr = 0; rr < kPanel; ++rr)
                if (rr < jb) inv_g[p * kPanel * kPanel + rr * jb + c] = (S)x[rr];
        }
    }
}

// Trailing-update block (bi, bj) of panel j0 (16 x 16 blocks of the
// trailing lower triangle starting at row and column t0; K = 16 on the matrix
// cores), in place in the packed triangle.
template <class C, class Cst>
__device__ __forceinline__ void trailing_block(C* __restrict__ T, Cst cst, int dummy, int w,
                                               int j0, int t0, int bi, int bj, int lr, int lk) {
    const int row0 = t0 + bi * kPanel, col0 = t0 + bj * kPanel;
    const int ra = row0 + lr, rb = col0 + lr;
    const bool oka = ra < w, okb = rb < w;
    C cv[4], av[4], bv[4];
    int ci[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = row0 + Mx<C>::row(q, lk), cc = col0 + lr;
        const bool ok = rr < w && cc < w && rr >= cc;
        ci[q] = ok ? cst(cc) + rr : dummy;
        cv[q] = T[ci[q]];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = j0 + 4 * kk + lk;
        const C ta = T[oka ? cst(k) + ra : dummy];
        const C tb = T[okb ? cst(k) + rb : dummy];
        av[kk] = oka ? -ta : C(0);
        bv[kk] = okb ? tb : C(0);
    }
    typename Mx<C>::acc acc = {cv[0], cv[1], cv[2], cv[3]};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = Mx<C>::mfma(av[kk], bv[kk], acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) T[ci[q]] = acc[q];
}

// Diagonal factorization of supernode s by one workgroup of 4 waves, on the
// w x w block held in LDS (T) as a packed lower triangle, column major: entry
// (i, j) at cst(j) + i, plus one dummy slot that absorbs masked accesses.
// Right-looking by 16-column panels:
//   1. the four waves update the next panel's columns with the current
//      panel (16 x 16 blocks, K = 16 on the matrix cores);
//   2. wave 0 factors the next panel column by column in registers
//      (panel_columns: its diagonal block and every row below it at once),
//      while waves 1-3 update the rest of the trailing triangle and then
//      write the current panel's columns back to the block;
// so the chain from panel to panel is one block update and one register
// column factorization, and only the last panel is written after it.  The
// inverses of the 16 x 16 diagonal blocks (for the panel and triangular
// solves) are formed at the end by all four waves.  The block is loaded by
// packed index with many loads per thread in flight.
// Storage type S, compute type C.  Without kCheck a pivot that is not
// positive records its global column with atomicMin on *status (the smallest
// failing column wins).  With kCheck (FP32 pass) nothing is recorded: if any
// pivot is not above kPivotTau times its starting diagonal entry the block's
// input values go back to global memory (from a copy in LDS) and the
// function returns true, so that the caller can factor it again in FP64.
template <class S, class C, bool kCheck, int kW = kMaxWidth>
__device__ __forceinline__ bool potrf_task(int s, const KArgs& a, S* __restrict__ arena,
                                           S* __restrict__ dinv, int32_t* __restrict__ status,
                                           C* __restrict__ T) {
    __shared__ C rdiag[kMaxWidth];
    __shared__ C colbuf[kPanel * kPanel];  // one column of the panel's diagonal block
    __shared__ C d0[kCheck ? kMaxWidth : 1];
    __shared__ int unstable;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    S* __restrict__ base = arena + a.sn_off[s];
    S* __restrict__ inv_g = dinv + a.inv_off[s];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int nwave = kPotrfThreads / 64;
    auto cst = [w](int j) { return (j * (2 * w - j - 1)) >> 1; };
    const int dummy = w * (w + 1) / 2;  // masked accesses land here
    if (kCheck && tid == 0) unstable = 0;
    // The lower triangle folded into a (w + 1) x ceil(w / 2) rectangle:
    // rectangle column pc holds column pc (rows pc .. w - 1) followed by
    // column w - 1 - pc (rows w - 1 - pc .. w - 1); for odd w the middle
    // column is taken once.  Wave v loads rectangle columns v, v + 4, ...,
    // lane l their entries l, l + 64 and l + 128, in rounds of kRound
    // rectangle columns with every load of a round in flight.
    const int hw = (w + 1) >> 1, w1 = w + 1;
    constexpr int kRect = ((kW + 1) / 2 + nwave - 1) / nwave;  // per wave
    // FP32 pass: a copy of the input block after the triangle (the LDS holds
    // an FP64 triangle, room for two FP32 ones), written back if a pivot
    // fails the check, so that the FP64 pass starts from the input
    C* __restrict__ Tb = T + dummy + 1;
    constexpr int kRound = (kRect + 1) / 2;
    for (int t0 = 0; t0 * nwave < hw; t0 += kRound) {
        C v[kRound][3];
        int at[kRound][3];
#pragma unroll
        for (int t = 0; t < kRound; ++t) {
            const int pc = wave + nwave * (t0 + t), pj = w - 1 - pc;
            const S* __restrict__ c0 = base + (int64_t)pc * ld;
            const S* __restrict__ c1 = base + (int64_t)pj * ld;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int q = lane + 64 * u;
                const bool first = q < w - pc;
                const int j = first ? pc : pj, i = first ? pc + q : pj + q - (w - pc);
                const bool ok = pc < hw && q < w1 && (first || pj != pc);
                v[t][u] = ok ? (C)(first ? c0 : c1)[i] : C(0);
                at[t][u] = ok ? cst(j) + i : dummy;
            }
        }
#pragma unroll
        for (int t = 0; t < kRound; ++t)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                T[at[t][u]] = v[t][u];
                if (kCheck) {
                    Tb[at[t][u]] = v[t][u];
                    const int pc = wave + nwave * (t0 + t), q = lane + 64 * u;
                    // the diagonal entries: q = 0 of column pc and q = w - pc of w - 1 - pc
                    if (pc < hw && q == 0) d0[pc] = v[t][u];
                    if (pc < hw && q == w - pc && w - 1 - pc != pc) d0[w - 1 - pc] = v[t][u];
                }
            }
    }
    __syncthreads();
    const int npanel = (w + kPanel - 1) / kPanel;
    // panel q's columns (rows q * 16 .. w - 1) back to the block, round robin
    // over waves wv0 .. 3
    auto emit = [&](int q, int wv0) {
        const int j0 = q * kPanel, jb = min(kPanel, w - j0);
        for (int k = wave - wv0; k < jb; k += nwave - wv0) {
            const int j = j0 + k, cj = cst(j);
            S* __restrict__ col = base + (int64_t)j * ld;
            C v[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int i = j + lane + 64 * u;
                v[u] = T[i < w ? cj + i : dummy];
            }
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int i = j + lane + 64 * u;
                if (i < w) col[i] = (S)v[u];
            }
        }
    };
    if (wave == 0)
        panel_columns<C, kCheck, kW>(T, rdiag, colbuf, cst, w, 0, min(kPanel, w), lane, first,
                                 status, d0, &unstable);
    __syncthreads();
    for (int p = 0; p + 1 < npanel; ++p) {
        const int j0 = p * kPanel, t0 = j0 + kPanel;
        const int nbr = (w - t0 + kPanel - 1) / kPanel;  // trailing block rows
        // 1. the next panel's column of blocks
        for (int bi = wave; bi < nbr; bi += nwave)
            trailing_block<C>(T, cst, dummy, w, j0, t0, bi, 0, lr, lk);
        __syncthreads();
        // 2. wave 0 factors the next panel; waves 1-3 update the other columns
        if (wave == 0) {
            panel_columns<C, kCheck, kW>(T, rdiag, colbuf, cst, w, t0, min(kPanel, w - t0), lane,
                                     first, status, d0, &unstable);
        } else {
            const int nblk = nbr * (nbr - 1) / 2;  // blocks (bi, bj), 1 <= bj <= bi
            for (int b = wave - 1; b < nblk; b += nwave - 1) {
                int bi = (int)((sqrtf(8.0f * b + 1.0f) + 1.0f) * 0.5f);
                bi -= (bi * (bi - 1) / 2 > b);
                bi += ((bi + 1) * bi / 2 <= b);
                const int bj = b - bi * (bi - 1) / 2 + 1;
                trailing_block<C>(T, cst, dummy, w, j0, t0, bi, bj, lr, lk);
            }
            emit(p, 1);
        }
        __syncthreads();
    }
    emit(npanel - 1, 0);
    if (!kCheck || !unstable) {  // uniform: read after the last barrier
        panel_inverses<C, S>(T, rdiag, inv_g, cst, w, npanel, wave, lane);
        return false;
    }
    // a failed check: the input block back by the rectangle columns of the
    // load, after every emitted store has completed
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kRect; ++t) {
        const int pc = wave + nwave * t, pj = w - 1 - pc;
        S* __restrict__ c0 = base + (int64_t)pc * ld;
        S* __restrict__ c1 = base + (int64_t)pj * ld;
        C v[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int q = lane + 64 * u;
            const bool first = q < w - pc;
            const int j = first ? pc : pj, i = first ? pc + q : pj + q - (w - pc);
            const bool ok = pc < hw && q < w1 && (first || pj != pc);
            v[u] = Tb[ok ? cst(j) + i : dummy];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int q = lane + 64 * u;
            const bool first = q < w - pc;
            const bool ok = pc < hw && q < w1 && (first || pj != pc);
            if (ok) (first ? c0 : c1)[first ? pc + q : pj + q - (w - pc)] = (S)v[u];
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // before the FP64 pass reloads it
    return true;
}

// Diagonal factorization in the factor's precision.  FP64 factors: one FP64
// pass.  FP32 factors: an FP32 pass; a block it flags as unstable (a pivot
// ratio below kPivotTau) is factored again from its unchanged FP32 input in
// FP64 arithmetic and rounded to FP32, and counted in *fallbacks.  T must
// hold the packed triangle in the compute type of either pass.
template <int kW = kMaxWidth>
__device__ __forceinline__ void diag_factor(int s, const KArgs& a, double* arena, double* dinv,
                                            int32_t* status, int32_t* fallbacks, void* T) {
    potrf_task<double, double, false, kW>(s, a, arena, dinv, status, (double*)T);
}
template <int kW = kMaxWidth>
__device__ __forceinline__ void diag_factor(int s, const KArgs& a, float* arena, float* dinv,
                                            int32_t* status, int32_t* fallbacks, void* T) {
    if (potrf_task<float, float, true, kW>(s, a, arena, dinv, status, (float*)T)) {
        __syncthreads();
        potrf_task<float, double, false, kW>(s, a, arena, dinv, status, (double*)T);
        if (threadIdx.x == 0) atomicAdd(fallbacks, 1);
    }
}

// Level-set form: one workgroup per supernode of the level.  The instance
// for blocks of at most 64 columns (kNarrow) holds a quarter of the
// registers of the general one (one row chunk per lane), so that several
// workgroups share a compute unit on levels of many such blocks.
constexpr int kNarrow = 64;
// The narrow instances are held to three (FP64) or four (FP32) waves per SIMD:
// a level's many narrow blocks then share each compute unit three or four at
// a time, at the price of a few spilled registers.
template <class R, int kW>
constexpr int potrf_waves() { return kW > kNarrow ? 1 : (sizeof(R) == 4 ? 4 : 3); }

template <class R, int kW>
__global__ __launch_bounds__(kPotrfThreads, (potrf_waves<R, kW>())) void k_potrf(
    const int32_t* __restrict__ level_sn, KArgs a, R* __restrict__ arena, R* __restrict__ dinv,
    int32_t* __restrict__ status) {
    extern __shared__ double T[];
    diag_factor<kW>(level_sn[blockIdx.x], a, arena, dinv, status, status + 1, T);
}

// ---------------------------------------------------------------------------
// inverse of L11 for the solves
// ---------------------------------------------------------------------------

// L11^{-1} of every large supernode (list), packed lower triangle by columns
// after the supernode's panel inverses in dinv, and its transpose packed
// upper by columns after it, so that each solve applies
// the diagonal block as one triangular matrix-vector product instead of a
// chain of w dependent steps.  One workgroup per supernode, computing in
// FP64 whatever the storage type S: L11 (from the factor) and the panel
// inverses D_i^{-1} go to LDS; wave p forms block column p of X = L11^{-1}
// by block forward substitution on the matrix cores,
//   X_pp = D_p^{-1},  X_ip = D_i^{-1} (-sum_{p <= k < i} L_ik X_kp),
// right-looking: after X_ip is formed, B_j -= L_ji X_ip for every j > i,
// with the running right-hand sides B_j in accumulator registers.  The FP64
// accumulator layout of a 16 x 16 block is the B-operand layout of the next
// product, so X_ip feeds the updates without a trip through LDS.
constexpr int kLinvThreads = 64 * ((kMaxWidth + kPanel - 1) / kPanel);

template <class S>
__global__ __launch_bounds__(kLinvThreads) void k_linv(const int32_t* __restrict__ list, KArgs a,
                                                       const S* __restrict__ arena,
                                                       S* __restrict__ dinv) {
    constexpr int NP = (kMaxWidth + kPanel - 1) / kPanel;
    extern __shared__ double sm_linv[];
    const int s = list[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int np = (w + kPanel - 1) / kPanel;
    const S* __restrict__ base = arena + a.sn_off[s];
    const S* __restrict__ inv_g = dinv + a.inv_off[s];
    S* __restrict__ out = dinv + a.inv_off[s] + inverse_elems(w);
    S* __restrict__ outT = out + (w * (w + 1) / 2);  // L11^{-T}, packed upper by columns
    const int ntri = w * (w + 1) / 2;
    double* T = sm_linv;               // packed L11, then a zero slot for masked reads
    double* D = sm_linv + ntri + 1;    // panel inverses, 16 x 16 each, zero padded
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    auto cst = [w](int j) { return (j * (2 * w - j - 1)) >> 1; };
    {
        constexpr int kU = 8;
        for (int e0 = tid; e0 < ntri; e0 += kU * kLinvThreads) {
            double v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + u * kLinvThreads;
                int i = 0, j = 0;
                if (e < ntri) tri_entry(e, w, i, j);
                v[u] = e < ntri ? (double)base[i + (int64_t)j * ld] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (e0 + u * kLinvThreads < ntri) T[e0 + u * kLinvThreads] = v[u];
        }
        if (tid == 0) T[ntri] = 0.0;
        for (int e = tid; e < np * kPanel * kPanel; e += kLinvThreads) {
            const int p = e >> 8, m = (e >> 4) & 15, k = e & 15;
            const int jb = min(kPanel, w - p * kPanel);
            D[e] = (m < jb && k < jb) ? (double)inv_g[p * kPanel * kPanel + m * jb + k] : 0.0;
        }
    }
    __syncthreads();
    const int p = wave;
    if (p >= np) return;
    const int lr = lane & 15, lk = lane >> 4;
    const int c = p * kPanel + lr;  // this lane's column of X
    v4d B[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) B[j][q] = (j == p && 4 * q + lk == lr) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (i < p || i >= np) continue;
        // X_ip = D_i^{-1} B_i
        v4d X = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            X = __builtin_amdgcn_mfma_f64_16x16x4f64(D[i * 256 + lr * kPanel + 4 * kk + lk],
                                                    B[i][kk], X, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = i * kPanel + 4 * q + lk;
            if (r < w && r >= c) {
                out[cst(c) + r] = (S)X[q];
                outT[((r * (r + 1)) >> 1) + c] = (S)X[q];
            }
        }
        // B_j -= L_ji X_ip for the block rows below
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if (j <= i || j >= np) continue;
            const int row = j * kPanel + lr;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int col = i * kPanel + 4 * kk + lk;
                const double l = -T[(row < w && col < w) ? cst(col) + row : ntri];
                B[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(l, X[kk], B[j], 0, 0, 0);
            }
        }
    }
}

size_t linv_lds(int wmax) {
    const int np = (wmax + kPanel - 1) / kPanel;
    return ((size_t)wmax * (wmax + 1) / 2 + 1 + (size_t)np * kPanel * kPanel) * sizeof(double);
}

// ---------------------------------------------------------------------------
// F: panel solve L21 = A21 L11^{-T}
// ---------------------------------------------------------------------------

constexpr int kTrsmThreads = 256;

// The operands of panel p in the panel solve are rows 16p .. 16p + 15 of L11,
// columns 0 .. 16p - 1.  The staged form copies them once per workgroup into
// LDS as slab p: entry (16p + i, k) at slab_base(p) + 16k + i, rows past w
// clamped to row w - 1 (finite values that only reach output columns past w,
// which are never stored).
__host__ __device__ constexpr int slab_base(int p) { return 128 * p * (p - 1); }
__host__ __device__ constexpr int slab_elems(int np) { return np > 1 ? slab_base(np) : 0; }

// Every wave of the workgroup issues a share of the slab copies: direct
// global-to-LDS loads of one dword per lane, 256 contiguous LDS bytes (whole
// 16-row columns of a slab) per instruction, no register round trip.
template <class R, int NP>
__device__ __forceinline__ void stage_slabs(const R* __restrict__ L, int ld, int w,
                                            R* __restrict__ Ls, int wave, int lane) {
    constexpr int kD = sizeof(R) / 4;   // dwords per entry
    constexpr int kCols = 4 / kD;       // slab columns per instruction
    const int e = lane / kD, i = e & 15, kl = e >> 4;
    const int half = lane % kD;
#pragma unroll
    for (int p = 1; p < NP; ++p) {
        const char* src = (const char*)(L + min(16 * p + i, w - 1)) + 4 * half;
        for (int g = wave; g < 16 * p / kCols; g += kTrsmThreads / 64) {
            const int64_t k = g * kCols + kl;
            __builtin_amdgcn_global_load_lds((const void*)(src + k * ld * (int64_t)sizeof(R)),
                                             (void*)(Ls + slab_base(p) + g * kCols * 16), 4, 0,
                                             0);
        }
        // at most 20 copies per slab and wave: the count of loads in flight
        // stays within what the wait counter holds
        asm volatile("s_waitcnt vmcnt(32)" ::: "memory");
    }
}

// Panel solve for the 16 rows [row0, row0 + 16) of a panel, one wave, with
// NP 16-column panels (w <= 16 NP).  Everything stays in registers:
//   xo[p][q]  = X[row(q, lk)][16p + lr]  (matrix-core output layout)
//   xa[p][kk] = X[lr][16p + 4kk + lk]    (matrix-core A-operand layout)
// Panel p: B = X[:, p] - sum_{p' < p} X[:, p'] L[p, p']^T on
// the matrix cores with L read from the supernode block, or (kStaged) from
// the workgroup's LDS slabs (the next panel's operands are prefetched into
// registers while the current panel runs), then X[:, p] = B inv(D_p)^T; a
// 16 x 16 LDS tile converts between the layouts.  kStaged: every wave of the
// workgroup calls this (active: its rows start inside the block), copies its
// share of the slabs, and meets the others at one barrier.  kLean: no
// prefetch (each panel loads its own operands) and every finished panel goes
// to memory at once, so that fewer registers are live (FP64: 243 instead of
// 371, two waves per SIMD instead of one); the products are the same.
template <class R, int NP, bool kStaged = false, bool kLean = false>
__device__ __forceinline__ void trsm_rows(const R* __restrict__ L, int ld,
                                          const R* __restrict__ inv, R* __restrict__ P, int w,
                                          int r, int row0, R* __restrict__ tr, int lane,
                                          R* __restrict__ Ls = nullptr, int wave = 0,
                                          bool active = true) {
    typedef typename Mx<R>::acc Acc;
    const int lr = lane & 15, lk = lane >> 4;
    R xo[NP][4], xa[NP][4];
    // operands of panel p: L[16p + lr][16pp + 4kk + lk] for pp < p, and inv(D_p);
    // the next panel's are loaded while the current one runs (two register sets)
    R lv0[4 * NP], lv1[4 * NP], iv0[4], iv1[4];
    auto fetch = [&](int p, R* lv, R* iv) {
        const int col = 16 * p + lr;
        const bool okc = col < w;
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            if (pp < p) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 16 * pp + 4 * kk + lk;
                    const R v = kStaged ? Ls[slab_base(p) + 16 * k + lr]
                                        : L[okc ? col + (int64_t)k * ld : 0];
                    lv[4 * pp + kk] = okc ? v : R(0);
                }
            }
        }
        const int jbp = min(kPanel, w - kPanel * p);  // the inverse is jbp x jbp
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int c = 4 * kk + lk;
            const bool in = lr < jbp && c < jbp;
            const R v = inv[in ? p * kPanel * kPanel + lr * jbp + c : 0];
            iv[kk] = in ? v : R(0);
        }
    };
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = row0 + Mx<R>::row(q, lk), col = 16 * p + lr;
            const bool ok = row < r && col < w;
            const R v = P[ok ? row + (int64_t)col * ld : 0];
            xo[p][q] = ok ? v : R(0);
        }
    if constexpr (kStaged) {
        if constexpr (NP > 1) stage_slabs<R, NP>(L, ld, w, Ls, wave, lane);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (!active) return;
    }
    fetch(0, lv0, iv0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        R* lv = (p & 1) ? lv1 : lv0;
        R* iv = (p & 1) ? iv1 : iv0;
        if constexpr (kLean) {
            lv = lv0; iv = iv0;
            if (p > 0) fetch(p, lv0, iv0);
        } else if (p + 1 < NP) fetch(p + 1, (p & 1) ? lv0 : lv1, (p & 1) ? iv0 : iv1);
        Acc acc = {xo[p][0], xo[p][1], xo[p][2], xo[p][3]};
#pragma unroll
        for (int pp = 0; pp < p; ++pp)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = Mx<R>::mfma(-xa[pp][kk], lv[4 * pp + kk], acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) tr[Mx<R>::row(q, lk) * 17 + lr] = acc[q];
        __builtin_amdgcn_wave_barrier();
        R bA[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) bA[kk] = tr[lr * 17 + 4 * kk + lk];
        __builtin_amdgcn_wave_barrier();
        Acc out = {R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) out = Mx<R>::mfma(bA[kk], iv[kk], out);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xo[p][q] = out[q];
            tr[Mx<R>::row(q, lk) * 17 + lr] = out[q];
            if constexpr (kLean) {
                const int row = row0 + Mx<R>::row(q, lk), col = 16 * p + lr;
                if (row < r && col < w) P[row + (int64_t)col * ld] = out[q];
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xa[p][kk] = tr[lr * 17 + 4 * kk + lk];
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (!kLean) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = row0 + Mx<R>::row(q, lk), col = 16 * p + lr;
                if (row < r && col < w) P[row + (int64_t)col * ld] = xo[p][q];
            }
    }
}

// One workgroup of 4 waves per 64-row block of a panel, 16 rows per wave:
// L21 = A21 L11^{-T} by blocked forward substitution over 16-column panels
// with the inverses of the diagonal blocks from k_potrf.

// kStaged: the L11 operands come from LDS slabs at Ls (slab_elems of the
// block's panel count), copied once per workgroup instead of once per wave.
template <class R, int kMaxNP = 10, bool kStaged = false, bool kLean = false>
__device__ __forceinline__ void trsm_task(RowBlock wb, const KArgs& a, R* __restrict__ arena,
                                          const R* __restrict__ dinv, R* __restrict__ Ls = nullptr) {
    __shared__ R trs[kTrsmThreads / 64][16 * 17];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const R* __restrict__ L = arena + a.sn_off[s];
    R* __restrict__ P = arena + a.sn_off[s] + w;
    const R* __restrict__ inv = dinv + a.inv_off[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row0 = wb.rb * kTile + wave * 16;
    const bool active = row0 < r;
    if (!kStaged && !active) return;  // no barrier follows
    R* tr = trs[wave];
#define SPC_TRSM(NP) \
    trsm_rows<R, NP, kStaged, kLean>(L, ld, inv, P, w, r, row0, tr, lane, Ls, wave, active)
    // an instance for at most kMaxNP panels compiles (and holds registers
    // for) no more
    switch ((w + kPanel - 1) / kPanel) {
        case 1: SPC_TRSM(1); break;
        case 2: SPC_TRSM(2); break;
        case 3: SPC_TRSM(3); break;
        case 4: SPC_TRSM(4); break;
        default:
            if constexpr (kMaxNP > 4) {
                switch ((w + kPanel - 1) / kPanel) {
                    case 5: SPC_TRSM(5); break;
                    case 6: SPC_TRSM(6); break;
                    case 7: SPC_TRSM(7); break;
                    case 8: SPC_TRSM(8); break;
                    case 9: SPC_TRSM(9); break;
                    default: SPC_TRSM(10); break;
                }
            }
            break;
    }
#undef SPC_TRSM
}

// kW: the widest supernode of the launch (kNarrow: four panels at most).  The
// FP32 instance stages its operands in LDS (the launch brings
// slab_elems(ceil(wmax / 16)) entries of dynamic LDS, at most 45 KiB): it
// then holds 124 instead of 197 registers and runs three workgroups per
// compute unit instead of two.  FP64 reads L11 from memory (staged, one
// workgroup per compute unit either way, it measured slower); its lean form
// (kLean) serves launches of more blocks than compute units with blocks
// wider than kNarrow, where a second wave per SIMD hides the loads, and the
// prefetching form the others: there each block runs alone on its compute
// unit, or (at most four panels) the prefetching form already runs three
// workgroups per compute unit and measured faster.
template <class R>
constexpr bool trsm_staged() { return sizeof(R) == 4; }

template <class R, int kW, bool kLean = false>
__global__ __launch_bounds__(kTrsmThreads) void k_trsm(const RowBlock* __restrict__ work, KArgs a,
                                                       R* __restrict__ arena,
                                                       const R* __restrict__ dinv) {
    extern __shared__ double Tsl[];
    trsm_task<R, (kW + kPanel - 1) / kPanel, trsm_staged<R>(), kLean>(
        work[blockIdx.x], a, arena, dinv, reinterpret_cast<R*>(Tsl));
}

static_assert(kMaxWidth <= 10 * kPanel, "k_trsm instantiates at most 10 panels");
static_assert(slab_elems(10) * sizeof(float) <= 65536,
              "the FP32 panel solve's slabs fit the default dynamic LDS limit");

// ---------------------------------------------------------------------------
// U + A: update tiles on FP64 MFMA with relative-index scatter
// ---------------------------------------------------------------------------

// K columns staged per step: 16 by default; 8 or 32 by the analysis option
// upd_chunk (one of the tile shapes the batch autotuner searches).
constexpr int kChunkDefault = 16;
constexpr int kLdsStride = kTile + 2;  // padded row count of a staged K column
constexpr int kCtPad = kTile + 1;

// XCD-aware tile order: consecutive dispatches go round-robin over the 8
// XCDs, so block b runs on XCD b % 8.  Give each XCD a contiguous range of
// tiles (the tiles of one source share its panel in that XCD's L2).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, rem = nb & 7;
    const int64_t x = b & 7, j = b >> 3;
    return x * q + (x < rem ? x : rem) + j;
}

// 256 threads = 4 waves in a 2 x 2 grid, each wave a 32 x 32 quarter of the
// 64 x 64 tile as 2 x 2 blocks of 16 x 16 x 4 matrix-core products.  The K dimension (the
// source width w) goes through LDS in chunks of 16 columns, double buffered:
// the next chunk is loaded into registers while the current one feeds the
// matrix cores.  Operand lanes: lane l holds element (row l % 16, k l / 16) of
// each 16 x 4 slice; A and B are both rows of the same column-major panel
// (a diagonal tile stages them once).  The result goes to LDS, then every
// entry (i, c), i >= c, is subtracted from the target that owns the column's
// row: target block + rel[i] + (row(c) - first(t)) * ld(t), with a plain
// read-modify-write when the pair's target has no other source in this
// level and an atomic add otherwise.
// Forms of a launch's scatter: kAtomic (shared targets by atomic adds), and
// those of the deterministic order: kRound (every target of the launch has one
// writer) and kScratch (shared pairs go to the scratch for the apply pass).
enum { kAtomic = 0, kRound = 1, kScratch = 2 };

// Update tile by one workgroup of 4 waves.  If coltgt is given (an LDS array
// of kTile entries), it receives each column's target supernode (-1 past the
// panel), in non-decreasing order.  Entries of a pair whose target no other
// source of the level touches (pair_excl) are plain read-modify-writes; the
// others atomic adds (kAtomic), plain read-modify-writes (kRound), or stores
// of the negated entry to the source's packed block in the scratch at
// scr_off[s] (kScratch; column c, row i >= c at c (2r - c + 1) / 2 + i - c).
template <class R, int kMode = kAtomic, int kChunk = kChunkDefault,
          bool kDma = sizeof(R) == 4 && kChunk == kChunkDefault>
__device__ __forceinline__ void update_task(UpdTile tile, const KArgs& a,
                                            const uint8_t* __restrict__ pair_excl,
                                            R* __restrict__ arena, int* coltgt,
                                            const int64_t* __restrict__ scr_off = nullptr,
                                            R* __restrict__ scratch = nullptr) {
    typedef typename Mx<R>::acc Acc;
    __shared__ R lds[2 * 2 * kChunk * kLdsStride > kTile * kCtPad
                              ? 2 * 2 * kChunk * kLdsStride
                              : kTile * kCtPad];
    __shared__ int64_t colbase[kTile];
    __shared__ int64_t relbase[kTile];
    __shared__ int colexcl[kTile];
    const int s = tile.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const int i0 = tile.bi * kTile, c0 = tile.bj * kTile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const bool diag = tile.bi == tile.bj;
    const bool skip = diag && wr < wc;  // strictly upper quarter of a diagonal tile
    // staging: thread -> row (tid & 63), columns kq * kPerT .. of the chunk
    const int srow = tid & 63, kq = tid >> 6;
    const bool va = i0 + srow < r, vb = c0 + srow < r;
    R* As = lds;                               // [buf][k][row]
    R* Bs = lds + 2 * kChunk * kLdsStride;     // [buf][k][row]
    const int nchunk = (w + kChunk - 1) / kChunk;
    constexpr int kPerT = kChunk / 4;  // chunk columns staged per thread
    R ra[kPerT], rb[kPerT];
    auto fetch = [&](int chunk) {
#pragma unroll
        for (int u = 0; u < kPerT; ++u) {
            const int k = chunk * kChunk + kq * kPerT + u;
            const bool vk = k < w;
            const R* __restrict__ col = P + (int64_t)k * ld;
            ra[u] = (vk && va) ? col[i0 + srow] : R(0);
            rb[u] = (!diag && vk && vb) ? col[c0 + srow] : R(0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < kPerT; ++u) {
            As[(buf * kChunk + kq * kPerT + u) * kLdsStride + srow] = ra[u];
            if (!diag) Bs[(buf * kChunk + kq * kPerT + u) * kLdsStride + srow] = rb[u];
        }
    };
    // kDma (FP32, 16-column chunks): full chunks of full tiles go from global
    // memory straight to LDS, 4 bytes a lane and a column of 64 rows per
    // instruction, without the register round trip; wave kq takes columns
    // kq * kPerT .. as in fetch.  The same bits as the register path.
    const bool full_rows = i0 + kTile <= r && (diag || c0 + kTile <= r);
    auto direct = [&](int chunk) { return kDma && full_rows && (chunk + 1) * kChunk <= w; };
    auto dma = [&](int chunk, int buf) {
        constexpr int kIns = (int)sizeof(R) / 4;
#pragma unroll
        for (int u = 0; u < kPerT; ++u) {
            const int kc = kq * kPerT + u, k = chunk * kChunk + kc;
            const char* colA = (const char*)(P + (int64_t)k * ld + i0);
            const char* colB = (const char*)(P + (int64_t)k * ld + c0);
#pragma unroll
            for (int h = 0; h < kIns; ++h) {
                __builtin_amdgcn_global_load_lds(
                    (const void*)(colA + (h * 64 + lane) * 4),
                    (void*)((char*)(As + (buf * kChunk + kc) * kLdsStride) + h * 256), 4, 0, 0);
                if (!diag)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)(colB + (h * 64 + lane) * 4),
                        (void*)((char*)(Bs + (buf * kChunk + kc) * kLdsStride) + h * 256), 4, 0,
                        0);
            }
        }
    };
    // the first chunk's loads go out before the column -> target lookups,
    // whose chain of dependent loads then hides under them
    if (direct(0)) dma(0, 0);
    else fetch(0);
    // per column: the target's column base and relative-index base, and its
    // form: 1 plain, 0 atomic, 2 scratch (colbase then holds the column's
    // base in the scratch block, row gi at colbase + gi)
    int64_t my_colbase = 0, my_relbase = 0;
    int my_excl = kMode == kRound ? 1 : 0;
    if (tid < kTile) {
        const int gc = c0 + tid;
        if (coltgt) coltgt[tid] = -1;
        if (gc < r) {
            const int64_t at = rp + w + gc;
            const int p = a.rowpair[at];
            const int t = a.pair_tgt[p];
            if (coltgt) coltgt[tid] = t;
            my_colbase = a.sn_off[t] + (int64_t)(a.rows[at] - a.sn_first[t]) * a.sn_ld[t];
            my_relbase = a.pair_rel[p] - a.pair_seg[p];
            if (kMode != kRound) my_excl = pair_excl ? pair_excl[p] : 0;
            if (kMode == kScratch && !my_excl) {
                my_excl = 2;
                my_colbase = scr_off[s] + (int64_t)gc * (2 * r - gc + 1) / 2 - gc;
            }
        }
    }
    Acc acc[2][2];
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n) acc[m][n] = Acc{R(0), R(0), R(0), R(0)};
    if (direct(0)) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the DMA written
    else stash(0);
    __syncthreads();
    const R* Bsrc = diag ? As : Bs;
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const bool dnext = ch + 1 < nchunk && direct(ch + 1);
        if (dnext) dma(ch + 1, buf ^ 1);
        else if (ch + 1 < nchunk) fetch(ch + 1);
        if (!skip) {
#pragma unroll
            for (int kk = 0; kk < kChunk / 4; ++kk) {
                const int krow = (buf * kChunk + kk * 4 + lk) * kLdsStride;
                const R a0 = As[krow + wr * 32 + lr];
                const R a1 = As[krow + wr * 32 + 16 + lr];
                const R b0 = Bsrc[krow + wc * 32 + lr];
                const R b1 = Bsrc[krow + wc * 32 + 16 + lr];
                acc[0][0] = Mx<R>::mfma(a0, b0, acc[0][0]);
                acc[0][1] = Mx<R>::mfma(a0, b1, acc[0][1]);
                acc[1][0] = Mx<R>::mfma(a1, b0, acc[1][0]);
                acc[1][1] = Mx<R>::mfma(a1, b1, acc[1][1]);
            }
        }
        if (ch == 0 && tid < kTile) {
            colbase[tid] = my_colbase;
            relbase[tid] = my_relbase;
            colexcl[tid] = my_excl;
        }
        if (dnext) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        else if (ch + 1 < nchunk) stash(buf ^ 1);
        __syncthreads();
    }
    R* Ct = lds;  // the staging buffers are free now
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n)
            for (int q = 0; q < 4; ++q) {
                const int i = wr * 32 + m * 16 + Mx<R>::row(q, lk);
                const int c = wc * 32 + n * 16 + lr;
                Ct[c * kCtPad + i] = acc[m][n][q];
            }
    __syncthreads();
    // thread -> row i = tid & 63 of the tile, columns c = tid / 64 + 4 u
    // (u < 16); every relative index is loaded before the first update is
    // issued (loading them earlier costs registers, and occupancy, that the
    // K loop needs)
    constexpr int kPer = kTile * kTile / 256;
    const int i = tid & (kTile - 1), gi = i0 + i;
    int64_t dst[kPer];
    bool ok[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = (tid >> 6) + 4 * u, gc = c0 + c;
        ok[u] = gi < r && gc < r && gi >= gc;
        if (kMode == kScratch && colexcl[c] == 2) dst[u] = colbase[c] + gi;
        else dst[u] = ok[u] ? colbase[c] + a.rel[relbase[c] + gi] : 0;
    }
    R old[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = (tid >> 6) + 4 * u;
        old[u] = (ok[u] && colexcl[c] == 1) ? arena[dst[u]] : R(0);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        if (!ok[u]) continue;
        const int c = (tid >> 6) + 4 * u;
        const R v = Ct[c * kCtPad + i];
        if (colexcl[c] == 1) arena[dst[u]] = old[u] - v;
        else if (kMode == kScratch && colexcl[c] == 2) scratch[dst[u]] = -v;
        else unsafeAtomicAdd(arena + dst[u], -v);
    }
}

template <class R, int kMode, int kChunk>
__global__ __launch_bounds__(256) void k_update(const UpdTile* __restrict__ tiles, int64_t ntiles,
                                                KArgs a, const uint8_t* __restrict__ pair_excl,
                                                R* __restrict__ arena,
                                                const int64_t* __restrict__ scr_off,
                                                R* __restrict__ scratch) {
    update_task<R, kMode, kChunk>(tiles[xcd_tile(blockIdx.x, ntiles)], a, pair_excl, arena,
                                  nullptr, scr_off, scratch);
}

// The k_update instance of a scatter form and K chunk.
template <class R, int kMode>
auto update_kernel(int chunk) {
    return chunk == 8 ? k_update<R, kMode, 8>
                      : (chunk == 32 ? k_update<R, kMode, 32> : k_update<R, kMode, 16>);
}

// ---------------------------------------------------------------------------
// Task-queue schedule: one persistent kernel, dependency counters in HBM
// ---------------------------------------------------------------------------
//
// The paper's dynamic scheduling (Section IV) on one GPU: every workgroup is
// a worker that takes the next task of a fixed topological order with an
// atomic ticket, waits until the task's inputs are done, runs it and
// signals its successors:
//   F(s)       waits until cntF[s] == 0 (all updates into s have landed);
//              runs the diagonal factorization; sets doneF[s];
//   T(s, b)    waits for doneF[s]; solves row block b; sets doneT;
//   U(s, i, j) waits for doneT of row blocks i and j; computes the tile and
//              scatter-adds it (atomic adds); decrements cntF[t] once for
//              every distinct target t of its columns.
// The lowest unfinished ticket always has its inputs done, so the queue
// cannot deadlock whatever the number of resident workers.  Every wait is
// bounded: past the deadline the worker raises the abort flag and records
// the error, and every worker exits at its next poll.
//
// State layout (int32): cntF[nsup], doneF[nsup], doneT[nrowblk], ctrl[4]
// with ctrl = {ticket, abort, error, clock}.  With a log (two int32 per
// task), a task's entry gets a stamp of the clock when its inputs are done
// and another when its results are written, before its successors are
// signalled.

__global__ void k_sched_reset(const int32_t* __restrict__ cnt0, int32_t* __restrict__ state,
                              int64_t nsup, int64_t total) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        state[i] = i < nsup ? cnt0[i] : 0;
}

// Bounded wait of one thread until *p == want.  Returns false on abort.  The
// polls are relaxed (an acquiring load invalidates the caches on every poll);
// the caller acquires once, after the last wait.
__device__ bool wait_eq(const int32_t* p, int32_t want, int32_t* ctrl, uint64_t deadline) {
    for (;;) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) return true;
        if (__hip_atomic_load(ctrl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() > deadline) {
            __hip_atomic_store(ctrl + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctrl + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

constexpr int kSchedThreads = 256;
static_assert(kSchedThreads == kPotrfThreads && kSchedThreads == kTrsmThreads,
              "one workgroup shape runs every task kind");

template <class R>
__global__ __launch_bounds__(kSchedThreads) void k_sched(
    const Task* __restrict__ tasks, int64_t ntasks, const int32_t* __restrict__ rb_base, KArgs a,
    R* __restrict__ arena, R* __restrict__ dinv, int32_t* __restrict__ status,
    int32_t* __restrict__ state, int64_t nsup, int64_t nrowblk, uint64_t wait_ticks,
    int32_t* __restrict__ log) {
    extern __shared__ double T[];
    __shared__ int32_t sh_ticket;
    __shared__ int coltgt[kTile];
    int32_t* cntF = state;
    int32_t* doneF = state + nsup;
    int32_t* doneT = doneF + nsup;
    int32_t* ctrl = doneT + nrowblk;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            int32_t t = atomicAdd(ctrl, 1);
            if (t < ntasks) {
                const Task tk = tasks[t];
                const uint64_t deadline = wall_clock64() + wait_ticks;
                bool ok;
                if (tk.kind == kTaskF) {
                    ok = wait_eq(cntF + tk.s, 0, ctrl, deadline);
                } else if (tk.kind == kTaskT) {
                    ok = wait_eq(doneF + tk.s, 1, ctrl, deadline);
                } else {
                    const int32_t rb = rb_base[tk.s];
                    ok = wait_eq(doneT + rb + tk.a, 1, ctrl, deadline) &&
                         (tk.a == tk.b || wait_eq(doneT + rb + tk.b, 1, ctrl, deadline));
                }
                if (!ok) t = -1;
                else if (log) log[2 * (int64_t)t] = atomicAdd(ctrl + 3, 1);
                // acquire, once per task: the L1 of this CU and the lines of
                // this XCD's L2 that other XCDs may have written are invalidated
                // before any wave of the workgroup reads the task's inputs
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            sh_ticket = t;
        }
        __syncthreads();
        const int32_t t = sh_ticket;
        if (t < 0 || t >= ntasks) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every wave, after the barrier
        const Task tk = tasks[t];
        if (tk.kind == kTaskF) {
            diag_factor(tk.s, a, arena, dinv, status, status + 1, T);
        } else if (tk.kind == kTaskT) {
            trsm_task<R>(RowBlock{tk.s, tk.a}, a, arena, dinv);
        } else {
            update_task<R>(UpdTile{tk.s, tk.a, tk.b}, a, nullptr, arena, coltgt);
        }
        // release, once per task: every wave's stores and adds have reached
        // this XCD's L2 (a wait for the wave's outstanding memory operations,
        // which the compiler may not move anything across, then the barrier);
        // one write-back of that L2 then makes them visible to every XCD
        // before the signal
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (log && tid == 0) log[2 * (int64_t)t + 1] = atomicAdd(ctrl + 3, 1);
        if (tk.kind == kTaskF) {
            if (tid == 0)
                __hip_atomic_store(doneF + tk.s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (tk.kind == kTaskT) {
            if (tid == 0)
                __hip_atomic_store(doneT + rb_base[tk.s] + tk.a, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else if (tid < kTile) {
            const int tg = coltgt[tid];
            if (tg >= 0 && (tid == 0 || coltgt[tid - 1] != tg))
                __hip_atomic_fetch_add(cntF + tg, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------


static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

namespace {

int take_event(spc_numeric* num) {
    if (num->next_event == num->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        num->events.push_back(e);
    }
    return (int)num->next_event++;
}

// Records an event before a launch group when timing is on; returns its index or -1.
int mark_begin(spc_numeric* num, hipStream_t st) {
    if (!num->timing) return -1;
    int e = take_event(num);
    if (e >= 0 && hipEventRecord(num->events[e], st) != hipSuccess) return -1;
    return e;
}

void mark_end(spc_numeric* num, hipStream_t st, int cls, int a) {
    if (a < 0) return;
    int b = take_event(num);
    if (b < 0 || hipEventRecord(num->events[b], st) != hipSuccess) return;
    num->marks.push_back(spc_numeric::Mark{cls, a, b});
}

}  // namespace

// Launches of one level: diagonal factorizations and panel solves, then the
// update tiles [u0, u1) of the level's list.
namespace {

template <class R>
void launch_ft(spc_numeric* num, const DevicePlan* P, const Symbolic& S, const KArgs& a,
               int32_t l, hipStream_t st) {
    const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
    const int wmax = P->level_maxw[l];
    // room for the packed triangle in FP64 (also the FP32 kernel's fallback pass)
    const size_t lds_tri = ((size_t)wmax * (wmax + 1) / 2 + 1) * sizeof(double);
    int ev;
    if (nbig > 0) {
        ev = mark_begin(num, st);
        auto kern = wmax <= kNarrow ? k_potrf<R, kNarrow> : k_potrf<R, kMaxWidth>;
        hipLaunchKernelGGL(kern, dim3(nbig), dim3(kPotrfThreads), lds_tri, st,
                           P->level_sn + n0, a, (R*)num->arena, (R*)num->dinv, num->status_dev);
        mark_end(num, st, 1, ev);
    }
    if (n1 - n0 > nbig) {  // small supernodes: factor, update and scatter, one wave each
        ev = mark_begin(num, st);
        launch_small_factor(num, a, P->level_sn + n0 + nbig, n1 - n0 - nbig, P->small_maxw[l],
                            P->small_maxr[l], P->small_maxm[l], st);
        // deterministic order: the shared targets take the small sources'
        // blocks from the scratch, one wave per target, sources in order
        mark_end(num, st, 5, ev);
    }
    const int64_t rb0 = P->rowblk_ptr[l], rb1 = P->rowblk_ptr[l + 1];
    if (rb1 > rb0) {
        ev = mark_begin(num, st);
        auto kern = wmax <= kNarrow ? k_trsm<R, kNarrow> : k_trsm<R, kMaxWidth>;
        if constexpr (sizeof(R) == 8)
            if (wmax > kNarrow && rb1 - rb0 > P->ncu) kern = k_trsm<R, kMaxWidth, true>;
        const size_t lds_slab =
            trsm_staged<R>() ? (size_t)slab_elems((wmax + kPanel - 1) / kPanel) * sizeof(R) : 0;
        hipLaunchKernelGGL(kern, dim3((unsigned)(rb1 - rb0)), dim3(kTrsmThreads), lds_slab, st,
                           P->rowblk + rb0, a, (R*)num->arena, (const R*)num->dinv);
        mark_end(num, st, 2, ev);
    }
}

// Update tiles [u0, u1).  exclusive_ok: plain read-modify-writes for the
// pairs whose target no other source of the level touches, atomic adds for
// the rest.  Deterministic order (level >= 0): the level's large sources in
// rounds (one launch each, all plain) or in the apply form (shared pairs to
// the scratch), then the level's apply pass (small sources, and large ones
// in the apply form).
template <class R>
void launch_update(spc_numeric* num, const DevicePlan* P, const KArgs& a, int64_t u0, int64_t u1,
                   bool exclusive_ok, hipStream_t st, int32_t level = -1) {
    if (num->det && level >= 0) {
        const std::vector<int64_t>& rp = P->round_ptr[level];
        const bool apply = P->level_apply[level];
        for (size_t r = 0; r + 1 < rp.size(); ++r) {
            if (rp[r + 1] <= rp[r]) continue;
            const int ev = mark_begin(num, st);
            const int ch = num->sym->S.opt.upd_chunk;
            auto kern = apply ? update_kernel<R, kScratch>(ch) : update_kernel<R, kRound>(ch);
            hipLaunchKernelGGL(kern, dim3((unsigned)(rp[r + 1] - rp[r])), dim3(256), 0, st,
                               P->tiles + rp[r], rp[r + 1] - rp[r], a,
                               (const uint8_t*)P->pair_excl, (R*)num->arena,
                               (const int64_t*)P->scr_off, (R*)num->det_scratch);
            mark_end(num, st, 3, ev);
        }
        if (P->app_ptr[level + 1] > P->app_ptr[level]) {
            const int ev = mark_begin(num, st);
            launch_small_apply(num, P->app_ptr[level], P->app_ptr[level + 1], st);
            mark_end(num, st, 5, ev);
        }
        return;
    }
    if (u1 <= u0) return;
    const int ev = mark_begin(num, st);
    auto kern = update_kernel<R, kAtomic>(num->sym->S.opt.upd_chunk);
    hipLaunchKernelGGL(kern, dim3((unsigned)(u1 - u0)), dim3(256), 0, st,
                       P->tiles + u0, u1 - u0, a,
                       exclusive_ok ? (const uint8_t*)P->pair_excl : nullptr, (R*)num->arena,
                       (const int64_t*)nullptr, (R*)nullptr);
    mark_end(num, st, 3, ev);
}

// Factorization driver.  sched 0: one stream, level by level (every
// dependency points to a lower level of the supernodal elimination tree).
// sched 1: the same order with a one-level lookahead on two streams: the
// diagonal factorizations, panel solves and the update tiles that feed the
// next level run on the caller's stream; the other ("bulk") update tiles of
// level l run on a second stream concurrently with level l + 1, and level l
// waits only for the bulk tiles of levels <= l - 2.  Concurrent tiles may hit
// one target, so the lookahead uses atomic adds throughout.  Without
// per-launch timing, sched 0 and 1 are captured into a graph on the first
// factorization and replayed after.  sched 2: one persistent launch of the
// task queue.
// The inverses of every large diagonal block, once the factorization is done
// (nothing in it reads them; the solves do).
template <class R>
void launch_linv(spc_numeric* num, const DevicePlan* P, const KArgs& a, hipStream_t st) {
    if (P->nbig == 0) return;
    const int ev = mark_begin(num, st);
    hipLaunchKernelGGL(k_linv<R>, dim3((unsigned)P->nbig), dim3(kLinvThreads),
                       linv_lds(P->big_maxw), st, (const int32_t*)P->big_sn, a,
                       (const R*)num->arena, (R*)num->dinv);
    mark_end(num, st, 1, ev);
}

template <class R>
int32_t run_factor_t(spc_numeric* num, const double* values, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const KArgs a = kargs(P);
    R* arena = (R*)num->arena;
    int ev = mark_begin(num, st);
    if (S.arena > 0)
        hipLaunchKernelGGL(k_fill<R>, dim3(grid_for(S.arena, 256)), dim3(256), 0, st, arena,
                           S.arena, R(0));
    // status[0]: smallest failing column (INT32_MAX = none); status[1]: FP64 fallbacks
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, num->status_dev, (int64_t)1,
                       (int32_t)INT32_MAX);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, num->status_dev + 1, (int64_t)1,
                       (int32_t)0);
    if (S.nnz_a > 0)
        hipLaunchKernelGGL(k_load<R>, dim3(grid_for(S.nnz_a, 256)), dim3(256), 0, st, values,
                           P->slot, arena, S.nnz_a);
    mark_end(num, st, 0, ev);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    if (num->sched == 2) {
        const int64_t total = 2 * S.nsup + P->nrowblk + 4;
        hipLaunchKernelGGL(k_sched_reset, dim3(grid_for(total, 256)), dim3(256), 0, st, P->cnt0,
                           num->sched_state, S.nsup, total);
        if (P->ntasks > 0) {
            const size_t lds_tri = ((size_t)P->max_w * (P->max_w + 1) / 2 + 1) * sizeof(double);
            int per_cu = 0, ncu = 0, dev = 0, clock_khz = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
            HIP_TRY(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sched<R>,
                                                                kSchedThreads, lds_tri));
            int64_t workers =
                std::min<int64_t>(P->ntasks, (int64_t)std::max(1, ncu) * std::max(1, per_cu));
            if (S.opt.workers > 0) workers = std::min<int64_t>(workers, S.opt.workers);
            const uint64_t ticks =
                (uint64_t)num->spin_limit * (uint64_t)std::max(1, clock_khz) / 1000;
            ev = mark_begin(num, st);
            hipLaunchKernelGGL(k_sched<R>, dim3((unsigned)workers), dim3(kSchedThreads), lds_tri,
                               st, (const Task*)P->tasks, P->ntasks, (const int32_t*)P->rb_base,
                               a, arena, (R*)num->dinv, num->status_dev, num->sched_state,
                               S.nsup, P->nrowblk, ticks, num->task_log);
            mark_end(num, st, 4, ev);
        }
        launch_linv<R>(num, P, a, st);
    } else {
        // sched 0 (or fewer than two levels): one stream m, level by level.
        // sched 1: the lookahead on m and the bulk stream.
        auto enqueue = [&](hipStream_t m) -> int32_t {
            if (num->sched == 0 || nl < 2) {
                for (int32_t l = 0; l < nl; ++l) {
                    launch_ft<R>(num, P, S, a, l, m);
                    launch_update<R>(num, P, a, P->tile_ptr[l], P->tile_ptr[l + 1], true, m, l);
                }
                launch_linv<R>(num, P, a, m);
                return OK;
            }
            hipStream_t sb = num->bulk;
            // events: [0] start, [1 + 2l] panel solves of level l done, [2 + 2l]
            // bulk of level l done
            if (num->sync_ev.size() < (size_t)(2 * nl + 1)) {
                const size_t old = num->sync_ev.size();
                num->sync_ev.resize((size_t)(2 * nl + 1));
                for (size_t i = old; i < num->sync_ev.size(); ++i)
                    HIP_TRY(hipEventCreateWithFlags(&num->sync_ev[i], hipEventDisableTiming));
            }
            hipEvent_t* E = num->sync_ev.data();
            HIP_TRY(hipEventRecord(E[0], m));
            HIP_TRY(hipStreamWaitEvent(sb, E[0], 0));
            for (int32_t l = 0; l < nl; ++l) {
                if (l >= 2) HIP_TRY(hipStreamWaitEvent(m, E[2 + 2 * (l - 2)], 0));
                launch_ft<R>(num, P, S, a, l, m);
                HIP_TRY(hipEventRecord(E[1 + 2 * l], m));
                const int64_t u0 = P->tile_ptr[l], uc = u0 + P->tile_crit[l];
                const int64_t u1 = P->tile_ptr[l + 1];
                launch_update<R>(num, P, a, u0, uc, false, m);
                HIP_TRY(hipStreamWaitEvent(sb, E[1 + 2 * l], 0));
                launch_update<R>(num, P, a, uc, u1, false, sb);
                HIP_TRY(hipEventRecord(E[2 + 2 * l], sb));
            }
            HIP_TRY(hipStreamWaitEvent(m, E[2 + 2 * (nl - 1)], 0));
            launch_linv<R>(num, P, a, m);
            return OK;
        };
        if (num->timing) return enqueue(st);  // per-launch events: launch directly
        // the level launches depend only on the plan and this factor's
        // buffers: capture them once (the bulk stream joins the capture
        // through the events), replay them on every factorization
        if (!num->factor_exec) {
            if (!num->capture)
                HIP_TRY(hipStreamCreateWithFlags(&num->capture, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(num->capture, hipStreamCaptureModeThreadLocal));
            const int32_t e = enqueue(num->capture);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(num->capture, &g);
            if (e != OK || ce != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return e != OK ? e : ERR_HIP;
            }
            if (hipGraphInstantiate(&num->factor_exec, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                num->factor_exec = nullptr;
                return ERR_HIP;
            }
            num->factor_graph = g;
        }
        HIP_TRY(hipGraphLaunch(num->factor_exec, st));
    }
    return OK;
}

}  // namespace

int32_t run_factor(spc_numeric* num, const double* values, hipStream_t st) {
    num->stream = st;
    num->factored = false;
    num->fb_current = false;  // an FP64 fallback factor belongs to the previous values
    num->status_known = false;
    num->marks.clear();
    num->next_event = 0;
    const int32_t r = num->prec == 1 ? run_factor_t<float>(num, values, st)
                                     : run_factor_t<double>(num, values, st);
    if (r != OK) return r;
    HIP_TRY(hipGetLastError());
    num->factored = true;
    return OK;
}

int32_t configure_solve_kernels();

int32_t configure_kernels() {
    static int done = 0;
    static int32_t result = OK;
    if (done) return result;
    done = 1;
    result = configure_solve_kernels();
    const int lds_max = (int)(((size_t)kMaxWidth * (kMaxWidth + 1) / 2 + 1) * sizeof(double));
    const void* big[] = {(const void*)k_potrf<double, kMaxWidth>,
                         (const void*)k_potrf<float, kMaxWidth>,
                         (const void*)k_potrf<double, kNarrow>,
                         (const void*)k_potrf<float, kNarrow>,
                         (const void*)k_sched<double>, (const void*)k_sched<float>};
    for (const void* f : big)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) !=
            hipSuccess)
            result = ERR_HIP;
    const void* linv[] = {(const void*)k_linv<double>, (const void*)k_linv<float>};
    for (const void* f : linv)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)linv_lds(kMaxWidth)) != hipSuccess)
            result = ERR_HIP;
    return result;
}

}  // namespace spc
