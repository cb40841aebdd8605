// Supernodal triangular solves on gfx950 (the two solves of Section II-A of
// arXiv:1608.00044): y = L^{-1} P b by a forward sweep over the supernodal
// elimination tree from the leaves, then z = L^{-T} y from the root back, and
// x = P^T z.  Both sweeps go level by level; within a level every supernode
// is independent.  A large supernode's diagonal block is applied as one
// product with L11^{-1}, which the factorization forms, so no kernel walks
// the w columns of a block one after another.  Per level:
//   forward:  k_fwd_level  -- per 64-row block of a supernode's rows below:
//                             z_s = L11^{-1} y_s (every block of s forms the
//                             same z_s), then y[rows below] -= L21 z_s; a row
//                             that another source of the level also updates
//                             gets its value in a contribution slot instead,
//             k_fwd_reduce -- which one thread per such row subtracts, sources
//                             in increasing order;
//   backward: k_bwd_cols   -- partial sums of L21^T y[rows below], one
//                             workgroup per group of kColGroup columns and
//                             chunk of kRowChunk rows, summed in a fixed tree;
//             k_bwd_diag   -- x_s = L11^{-T} (z_s - t_s), t_s the chunks'
//                             partial sums in chunk order, on the matrix
//                             cores.
// Small supernodes (a group of lanes each) go through k_small_fwd/bwd.
// No update is an atomic add: every sum has one fixed order, so a solve has
// the same bits on every run.  Several right-hand sides go through every
// kernel in groups of eight, so the factor is read once per group.
// The level sweeps are captured once per right-hand-side count into a HIP
// graph and replayed, so a solve costs three launches on the host.  The
// kernels are templates on the factor's real type R: an FP32 factor is
// solved in FP32 arithmetic with FP32 work vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/spchol.h"
#include "runtime.hpp"

namespace spc {

#define HIP_TRY(x)                               \
    do {                                         \
        if ((x) != hipSuccess) return ERR_HIP;   \
    } while (0)

template <class R>
__global__ void k_gather(const double* __restrict__ b, int64_t ldb,
                         const int32_t* __restrict__ perm, R* __restrict__ y, int64_t n,
                         int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        y[e] = (R)b[perm[i] + c * ldb];
    }
}

template <class R>
__global__ void k_scatter(const R* __restrict__ y, const int32_t* __restrict__ perm,
                          double* __restrict__ x, int64_t ldx, int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        x[perm[i] + c * ldx] = (double)y[e];
    }
}

template <class R>
__global__ void k_zero(R* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = R(0);
}

// Value held by lane `lane` (wave-uniform) of the wave, as v_readlane.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Right-hand sides go through the level kernels NR at a time (NR = 1, or
// kRhs for several): the factor's blocks are read once per group and every
// thread keeps NR partial sums.
constexpr int kRhs = 8;

// Row i's partial sums over this wave's columns k = wave + 4u of a packed
// triangle already in registers (m[u] = entry (i, k), zero outside the
// triangle), into red[wave][.][i].
template <class R, int NR, int KW>
__device__ __forceinline__ void tri_rows(const R (&m)[KW], const R (*__restrict__ ys)[NR],
                                         R (*__restrict__ red)[NR][kMaxWidth], int w, int i,
                                         int wave) {
    R acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = wave + 4 * u;
        if (k < w) {
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] += m[u] * ys[k][c];
        }
    }
    if (i < w) {
#pragma unroll
        for (int c = 0; c < NR; ++c) red[wave][c][i] = acc[c];
    }
}

// Products with a diagonal block's inverse, one matrix-vector product per
// right-hand side: lane = row of a 64-row chunk, wave = every 4th column
// k = wave + 4u, the waves' partial sums into red[wave][c][i].  kUpper =
// false: z = L11^{-1} v with L11^{-1} packed lower by columns (entry (i, k) at
// k (2w - k - 1) / 2 + i); kUpper = true: x = L11^{-T} v with L11^{-T} packed
// upper by columns (entry (i, k) at k (k + 1) / 2 + i): both read
// consecutive rows at consecutive addresses.  tri_first loads, early, the
// chunk with the most columns (the last rows for the lower triangle, the
// first for the upper) into registers; tri_rest forms every chunk's sums,
// the other chunks' entries loaded 16 at a time.
constexpr int kTriKW = (kMaxWidth + 3) / 4;

template <bool kUpper>
__device__ __forceinline__ int tri_first_chunk(int w) { return kUpper ? 0 : (w - 1) >> 6; }
template <bool kUpper>
__device__ __forceinline__ bool tri_in(int w, int i, int k) {
    return kUpper ? (k >= i && k < w) : (k <= i && i < w);
}
template <bool kUpper>
__device__ __forceinline__ int tri_at(int w, int i, int k) {
    return kUpper ? ((k * (k + 1)) >> 1) + i : ((k * (2 * w - k - 1)) >> 1) + i;
}

template <class R, bool kUpper>
__device__ __forceinline__ void tri_first(const R* __restrict__ M, int w, int wave, int lane,
                                          R (&m)[kTriKW]) {
    const int i = 64 * tri_first_chunk<kUpper>(w) + lane;
#pragma unroll
    for (int u = 0; u < kTriKW; ++u) {
        const int k = wave + 4 * u;
        m[u] = tri_in<kUpper>(w, i, k) ? M[tri_at<kUpper>(w, i, k)] : R(0);
    }
}

template <class R, int NR, bool kUpper>
__device__ __forceinline__ void tri_rest(const R* __restrict__ M, int w, const R (&m)[kTriKW],
                                         const R (*__restrict__ ys)[NR],
                                         R (*__restrict__ red)[NR][kMaxWidth], int wave, int lane) {
    const int qa = tri_first_chunk<kUpper>(w), nq = (w + 63) >> 6;
    tri_rows<R, NR, kTriKW>(m, ys, red, w, 64 * qa + lane, wave);
    for (int q = 0; q < nq; ++q) {
        if (q == qa) continue;
        const int i = 64 * q + lane;
        // the columns that meet rows [64q, 64q + 64)
        const int u_lo = kUpper ? 16 * q : 0;
        const int u_hi = kUpper ? kTriKW : min(kTriKW, 16 * (q + 1));
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
        for (int u0 = u_lo; u0 < u_hi; u0 += 16) {
            R lb[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = wave + 4 * (u0 + u);
                lb[u] = (u0 + u < kTriKW && tri_in<kUpper>(w, i, k)) ? M[tri_at<kUpper>(w, i, k)]
                                                                     : R(0);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = wave + 4 * (u0 + u);
                if (u0 + u < kTriKW && k < w) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += lb[u] * ys[k][c];
                }
            }
        }
        if (i < w) {
#pragma unroll
            for (int c = 0; c < NR; ++c) red[wave][c][i] = acc[c];
        }
    }
}

// The same lower product as tri_first + tri_rest with no early registers:
// each wave's columns eight loads at a time (FP64 with eight right-hand
// sides, where the early chunk would cost occupancy).
template <class R, int NR>
__device__ __forceinline__ void tri_lower_batched(const R* __restrict__ M, int w,
                                                  const R (*__restrict__ ys)[NR],
                                                  R (*__restrict__ red)[NR][kMaxWidth], int wave,
                                                  int lane) {
    constexpr int kB = 8;
    for (int q = 0; q < 3; ++q) {
        if (64 * q >= w) break;
        const int i = 64 * q + lane;
        const int kend = min(w, 64 * q + 64);
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
        for (int k0 = wave; k0 < kend; k0 += 4 * kB) {
            R lx[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int k = k0 + 4 * u;
                lx[u] = (k < kend && tri_in<false>(w, i, k)) ? M[tri_at<false>(w, i, k)] : R(0);
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                if (k0 + 4 * u < kend) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += lx[u] * ys[k0 + 4 * u][c];
                }
            }
        }
        if (i < w) {
#pragma unroll
            for (int c = 0; c < NR; ++c) red[wave][c][i] = acc[c];
        }
    }
}

// Forward, one level, large supernodes: one workgroup per 64-row block of a
// supernode's rows below its diagonal block (one block when there are none):
//   z_s = L11^{-1} y_s          as one product with the inverse the
//                               factorization formed (tri_first / tri_rest;
//                               its largest chunk loaded with the block's
//                               rows, before y_s);
//                               every workgroup of s forms the same z_s, the
//                               first writes it to zb (y_s itself stays: the
//                               others still read it);
//   y[rows(i)] -= L21[i] z_s    the block's 64 rows (loaded before z_s is
//                               formed, so that their latency overlaps it),
//                               lane = row, wave = every 4th column, waves
//                               meet in LDS; a row no other source of the
//                               level updates is updated in place (its only
//                               writer), a shared row's sum goes to its
//                               contribution slot for k_fwd_reduce.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_fwd_level(const RowBlock* __restrict__ work, KArgs a,
                                                   const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, R* __restrict__ zb,
                                                   int64_t n, int nrhs, SolveBufs<R> sb) {
    static_assert(kMaxWidth <= 192, "three 64-row chunks of the diagonal block");
    constexpr int KW = kTriKW;  // columns per wave
    __shared__ R ys[kMaxWidth][NR];
    __shared__ R red[4][NR][kMaxWidth];
    const RowBlock wb = work[blockIdx.x];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const R* __restrict__ Li = dinv + a.inv_off[s] + inverse_elems(w);
    const int32_t* __restrict__ below = a.rows + rp + w;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i0 = wb.rb * kTile, m = max(0, min(kTile, r - i0));
    // FP64 with several right-hand sides: no early inverse chunk (occupancy)
    constexpr bool kEarly = NR == 1 || sizeof(R) == 4;
    R la[KW];
    if (kEarly) tri_first<R, false>(Li, w, wave, lane, la);
    R lv[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = wave + 4 * u;
        lv[u] = (lane < m && k < w) ? P[i0 + lane + (int64_t)k * ld] : R(0);
    }
    const int64_t slot = rp + w + i0 + tid;
    const int32_t row = tid < m ? below[i0 + tid] : 0;
    const bool sh = tid < m && sb.shared[slot];
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        R yold[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            yold[c] = (tid < m && !sh && c < nc) ? y[(int64_t)(c0 + c) * n + row] : R(0);
        for (int e = tid; e < w * NR; e += 256) {
            const int k = e / NR, c = e % NR;
            ys[k][c] = c < nc ? y[(int64_t)(c0 + c) * n + first + k] : R(0);
        }
        __syncthreads();
        if (kEarly) tri_rest<R, NR, false>(Li, w, la, ys, red, wave, lane);
        else tri_lower_batched<R, NR>(Li, w, ys, red, wave, lane);
        __syncthreads();
        for (int e = tid; e < w * NR; e += 256) {
            const int k = e / NR, c = e % NR;
            ys[k][c] = (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]);
        }
        __syncthreads();
        if (wb.rb == 0) {
            for (int e = tid; e < w * NR; e += 256) {
                const int k = e / NR, c = e % NR;
                if (c < nc) zb[(int64_t)(c0 + c) * n + first + k] = ys[k][c];
            }
        }
        if (m > 0) {
            R acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
            for (int u = 0; u < KW; ++u) {
                const int k = wave + 4 * u;
                if (k < w) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += lv[u] * ys[k][c];
                }
            }
#pragma unroll
            for (int c = 0; c < NR; ++c) red[wave][c][lane] = acc[c];
            __syncthreads();
            if (tid < m) {
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    if (c >= nc) break;
                    const R v = (red[0][c][tid] + red[1][c][tid]) +
                                (red[2][c][tid] + red[3][c][tid]);
                    if (sh) sb.cb[(int64_t)(c0 + c) * sb.nslots + slot] = v;
                    else y[(int64_t)(c0 + c) * n + row] = yold[c] - v;
                }
            }
        }
        __syncthreads();
    }
}

// Matrix-core step 16 x 16 x 4 in the solve's arithmetic.  Operands: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register q of
// lane l holds D[row(q, l / 16)][l % 16], row = 4q + l/16 (FP64) or
// 4 (l/16) + q (FP32).
template <class R> struct SMx;
template <> struct SMx<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mfma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lk) { return 4 * q + lk; }
};
template <> struct SMx<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mfma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lk) { return 4 * lk + q; }
};

// x^T = u^T L11^{-1} on the matrix cores: x[k][c] = sum_{i >= k}
// L11^{-1}[i][k] u[i][c], with u^T as the A operand (right-hand sides as its
// 16 rows, zero past NR) and 16-column blocks of the packed inverse (Li, by
// columns) as B.  Column block j goes to wave (j / 4 even ? j % 4 : 3 - j % 4)
// counted from the last block, which spreads the blocks' falling cost over
// the four waves; each wave issues eight operand loads before their products.
template <class R, int NR>
__device__ __forceinline__ void inv_upper(const R* __restrict__ Li, int w,
                                          const R (*__restrict__ us)[NR], R* __restrict__ y,
                                          int64_t n, int first, int c0, int nc, int wave,
                                          int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    const int np = (w + 15) / 16;
    auto cst = [w](int q) { return (q * (2 * w - q - 1)) >> 1; };
    for (int j = 0; j < np; ++j) {
        const int jr = np - 1 - j;
        if ((((jr >> 2) & 1) ? 3 - (jr & 3) : (jr & 3)) != wave) continue;
        const int col = 16 * j + lr;
        typename SMx<R>::acc acc = {R(0), R(0), R(0), R(0)};
        for (int i0 = 16 * j; i0 < w; i0 += 32) {
            R av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 4 * u + lk;
                av[u] = (i < w && lr < NR) ? us[i < w ? i : 0][lr < NR ? lr : 0] : R(0);
                bv[u] = (i < w && col < w && i >= col) ? Li[cst(col) + i] : R(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + 4 * u < w) acc = SMx<R>::mfma(av[u], bv[u], acc);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = SMx<R>::row(q, lk);
            if (c < nc && col < w) y[(int64_t)(c0 + c) * n + first + col] = acc[q];
        }
    }
}

// Shared rows of a level, forward: y[row] -= the row's contribution slots,
// sources in increasing order, one thread per row and right-hand side; each
// thread issues its slots' loads eight at a time.
template <class R>
__global__ __launch_bounds__(256) void k_fwd_reduce(const int32_t* __restrict__ red_row,
                                                    const int64_t* __restrict__ red_ptr,
                                                    const int32_t* __restrict__ red_slot,
                                                    int64_t count, R* __restrict__ y, int64_t n,
                                                    int nrhs, SolveBufs<R> sb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count * nrhs) return;
    const int64_t k = e % count, c = e / count;
    const R* __restrict__ cbc = sb.cb + c * sb.nslots;
    R* __restrict__ yc = y + c * n;
    const int64_t q0 = red_ptr[k], q1 = red_ptr[k + 1];
    R v = yc[red_row[k]];
    for (int64_t q = q0; q < q1; q += 8) {
        R t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = q + u < q1 ? cbc[red_slot[q + u]] : R(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q + u < q1) v -= t[u];
    }
    yc[red_row[k]] = v;
}

// Backward, below the diagonal block: sum_i L21[i][k] y[rows(i)] for the
// kColGroup columns k of group g of supernode s, over the rows i of chunk h:
// thread tid takes rows tid, tid + 256, ... (coalesced down each column of
// the column-major panel), then the 256 partial sums of every (column,
// right-hand side) meet in a fixed tree: across each wave by butterfly
// shuffles, then the four waves in order, into the chunk's partial sum (pb,
// one writer per entry, no atomics).  NR right-hand sides at a time.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_cols(const ColBlk* __restrict__ work, KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ y, R* __restrict__ pb,
                                                  const int64_t* __restrict__ pb_off,
                                                  int64_t pb_total, int64_t n, int nrhs) {
    constexpr int G = kColGroup;
    __shared__ R part[4][G * NR];
    const ColBlk wb = work[blockIdx.x];
    const int s = wb.s, g = wb.g, h = wb.h;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int64_t rp = a.rowptr[s];
    const int k0 = g * G, kc = min(G, w - k0);
    const int rb0 = h * kRowChunk;
    const int r = min((int)(a.rowptr[s + 1] - rp) - w - rb0, kRowChunk);  // rows of the chunk
    const R* __restrict__ P = arena + a.sn_off[s] + w + rb0 + (int64_t)k0 * ld;
    const int32_t* __restrict__ below = a.rows + rp + w + rb0;
    R* __restrict__ out = pb + pb_off[s] + (int64_t)h * w + k0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // GC columns per pass (all G for one right-hand side; with several, two
    // at a time so that the accumulators stay in registers)
    constexpr int GC = NR == 1 ? G : 2;
    constexpr int kU = NR == 1 ? 4 : 1;  // rows per step, every load of a step first
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int kg = 0; kg < G; kg += GC) {
            R acc[GC][NR];
#pragma unroll
            for (int k = 0; k < GC; ++k)
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[k][c] = R(0);
            for (int i0 = tid; i0 < r; i0 += 256 * kU) {
                R yv[kU][NR], pv[kU][GC];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int i = i0 + 256 * u;
                    const int32_t row = i < r ? below[i] : 0;
#pragma unroll
                    for (int c = 0; c < NR; ++c)
                        yv[u][c] = (i < r && c < nc) ? y[(int64_t)(c0 + c) * n + row] : R(0);
#pragma unroll
                    for (int k = 0; k < GC; ++k)
                        pv[u][k] = (i < r && kg + k < kc) ? P[i + (int64_t)(kg + k) * ld] : R(0);
                }
#pragma unroll
                for (int u = 0; u < kU; ++u)
#pragma unroll
                    for (int k = 0; k < GC; ++k)
#pragma unroll
                        for (int c = 0; c < NR; ++c) acc[k][c] += pv[u][k] * yv[u][c];
            }
#pragma unroll
            for (int k = 0; k < GC; ++k)
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    R v = acc[k][c];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                    if (lane == 0) part[wave][(kg + k) * NR + c] = v;
                }
        }
        __syncthreads();
        if (tid < G * NR) {
            const int k = tid / NR, c = tid % NR;
            if (k < kc && c < nc)
                out[(int64_t)(c0 + c) * pb_total + k] =
                    (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
        }
        __syncthreads();
    }
}

// k_bwd_cols for several right-hand sides (NR = kRhs = 8): 256 rows of the
// chunk at a time are staged in LDS, the block's kColGroup columns of L21
// and the rows' entries of y, every load coalesced and issued at once; then
// thread (column k, right-hand side c, quarter q) sums its quarter of the
// staged rows, and the four quarters meet in order.  One workgroup per
// (supernode, column group, row chunk), as k_bwd_cols, with no shuffles.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_cols_multi(const ColBlk* __restrict__ work,
                                                        KArgs a, const R* __restrict__ arena,
                                                        const R* __restrict__ y,
                                                        R* __restrict__ pb,
                                                        const int64_t* __restrict__ pb_off,
                                                        int64_t pb_total, int64_t n, int nrhs) {
    constexpr int G = kColGroup;
    static_assert(G * NR * 4 == 256, "one thread per (column, right-hand side, quarter)");
    constexpr int kRows = 256;
    __shared__ R Ls[kRows][G + 1];
    __shared__ R Xs[kRows][NR + 1];
    __shared__ R part[4][G][NR];
    const ColBlk wb = work[blockIdx.x];
    const int s = wb.s, g = wb.g, h = wb.h;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int64_t rp = a.rowptr[s];
    const int k0 = g * G, kc = min(G, w - k0);
    const int rb0 = h * kRowChunk;
    const int r = min((int)(a.rowptr[s + 1] - rp) - w - rb0, kRowChunk);  // rows of the chunk
    const R* __restrict__ P = arena + a.sn_off[s] + w + rb0 + (int64_t)k0 * ld;
    const int32_t* __restrict__ below = a.rows + rp + w + rb0;
    R* __restrict__ out = pb + pb_off[s] + (int64_t)h * w + k0;
    const int tid = threadIdx.x;
    const int k = tid % G, c = (tid / G) % NR, q = tid / (G * NR);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        R acc = R(0);
        for (int i0 = 0; i0 < r; i0 += kRows) {
            const int i = i0 + tid;
            const int32_t row = i < r ? below[i] : 0;
            R lv[G], xv[NR];
#pragma unroll
            for (int kk = 0; kk < G; ++kk)
                lv[kk] = (i < r && kk < kc) ? P[i + (int64_t)kk * ld] : R(0);
#pragma unroll
            for (int cc = 0; cc < NR; ++cc)
                xv[cc] = (i < r && cc < nc) ? y[(int64_t)(c0 + cc) * n + row] : R(0);
#pragma unroll
            for (int kk = 0; kk < G; ++kk) Ls[tid][kk] = lv[kk];
#pragma unroll
            for (int cc = 0; cc < NR; ++cc) Xs[tid][cc] = xv[cc];
            __syncthreads();
            const int j0 = q * (kRows / 4);
#pragma unroll 8
            for (int j = j0; j < j0 + kRows / 4; ++j) acc += Ls[j][k] * Xs[j][c];
            __syncthreads();
        }
        part[q][k][c] = acc;
        __syncthreads();
        if (tid < G * NR) {
            const int kk = tid % G, cc = tid / G;
            if (kk < kc && cc < nc)
                out[(int64_t)(c0 + cc) * pb_total + kk] =
                    (part[0][kk][cc] + part[1][kk][cc]) + (part[2][kk][cc] + part[3][kk][cc]);
        }
        __syncthreads();
    }
}

// Backward, diagonal block, one workgroup per large supernode of the level:
// t_s = the chunks' partial sums in chunk order, then
// x_s = L11^{-T} (z_s - t_s) into y, which now holds the solution of every
// supernode done so far: one right-hand side by tri_first / tri_rest with the
// packed L11^{-T}, eight on the matrix cores (inv_upper).
template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_diag(const int32_t* __restrict__ level_sn, KArgs a,
                                                  const R* __restrict__ dinv,
                                                  R* __restrict__ y, const R* __restrict__ zb,
                                                  const R* __restrict__ pb,
                                                  const int64_t* __restrict__ pb_off,
                                                  int64_t pb_total, int64_t n, int nrhs) {
    __shared__ R us[kMaxWidth][NR];
    __shared__ R red[4][NR][kMaxWidth];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], first = a.sn_first[s];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const int nh = r > 0 ? (r + kRowChunk - 1) / kRowChunk : 0;
    const R* __restrict__ Lt = dinv + a.inv_off[s] + inverse_elems(w) + w * (w + 1) / 2;
    const R* __restrict__ ps = pb + (r > 0 ? pb_off[s] : 0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    R la[kTriKW];
    if (NR == 1) tri_first<R, true>(Lt, w, wave, lane, la);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < w * NR; e += 256) {
            const int k = e / NR, c = e % NR;
            R t = R(0);
            if (c < nc) {
                const R* __restrict__ pk = ps + (int64_t)(c0 + c) * pb_total + k;
                for (int h0 = 0; h0 < nh; h0 += 8) {
                    R v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) v[j] = h0 + j < nh ? pk[(int64_t)(h0 + j) * w] : R(0);
#pragma unroll
                    for (int j = 0; j < 8; ++j) t += v[j];
                }
            }
            us[k][c] = c < nc ? zb[(int64_t)(c0 + c) * n + first + k] - t : R(0);
        }
        __syncthreads();
        if (NR == 1) {
            tri_rest<R, NR, true>(Lt, w, la, us, red, wave, lane);
            __syncthreads();
            for (int e = tid; e < w * NR; e += 256) {
                const int k = e / NR, c = e % NR;
                if (c < nc)
                    y[(int64_t)(c0 + c) * n + first + k] =
                        (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]);
            }
        } else {
            // eight right-hand sides fill half of the matrix-core operand
            inv_upper<R, NR>(Lt - w * (w + 1) / 2, w, us, y, n, first, c0, nc, wave, lane);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// the tail of the elimination tree: both sweeps in one persistent launch
// ---------------------------------------------------------------------------
//
// The top levels of a nested-dissection tree hold few supernodes each (the
// 64^3 problem: 73 of its 82 levels hold at most 103, the last 29 one each),
// and each level costs a few dependent launches whatever its work.  Those
// levels run instead as tasks of one launch: workgroups take tasks in a
// fixed topological order by an atomic ticket and wait on dependency
// counters before running them, the counters of the paper's task queue
// (Section IV) applied to the two solves:
//   F(t)     forward, diagonal block: waits until every row of t has its
//            updates from the tail's sources (turn[t] == rows updated), then
//            z_t = L11^{-1} y_t in place, sets ready[t];
//   R(s, b)  forward, 64-row block b below source s: its part of L21 is loaded
//            before the wait on ready[s], then y[rows] -= L21[b] z_s by atomic
//            adds, and each target's count (turn) grows by the block's rows
//            in it;
//   C(s, b)  backward, 64-row block b below s: its part of L21 is loaded
//            before it waits for the solution of every supernode its rows
//            belong to; writes the block's partial sums of L21^T x[rows] (one
//            writer per entry) and counts itself in cntB[s];
//   B(s)     backward, diagonal block: waits for ready[s] and all its C
//            blocks, then
//            x_s = L11^{-T} (z_s - the partial sums in block order) in place,
//            sets done[s].
// The forward updates of a row from several sources land in arrival order
// (the atomic contribution order: equal to rounding from run to run; the
// deterministic order sweeps these levels one by one instead).  A worker takes its next ticket only after its task is done, and a
// task waits only on tasks of smaller tickets, so the lowest unfinished
// ticket can always run: no deadlock for any number of resident workers.
// Every wait is bounded: past the deadline the worker sets the error and
// abort words, and every worker leaves at its next wait.
//
// State (int32, zeroed before each launch): turn, ready, cntB, done (one per
// tail supernode), then ticket, abort, error.

// Data that one task writes and another reads in the same launch (y, z, x,
// the partial sums) is stored and loaded at device scope, coherent across the
// eight XCDs' L2 caches without a cache writeback or invalidation: a signal
// follows its task's stores once they are complete (a wait for each wave's
// outstanding memory operations that the compiler cannot reorder around, then
// the workgroup barrier), and a waiter loads the data only after it has seen
// the signal.  Acquire/release fences would write back or invalidate a whole L2
// on every task, which costs more than the solve's work.
template <class T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of one thread until *p == want (device-scope polls).
__device__ __forceinline__ bool tail_wait(const int32_t* p, int32_t want, int32_t* ctrl,
                                          uint64_t deadline) {
    for (;;) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) return true;
        if (__hip_atomic_load(ctrl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() > deadline) {
            __hip_atomic_store(ctrl + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctrl + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__global__ void k_tail_reset(int32_t* __restrict__ state, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        state[i] = 0;
}

template <class R, int NR>
__global__ __launch_bounds__(256, 2) void k_tail(const TailTask* __restrict__ tasks, int64_t ntasks,
                                              const TailSeg* __restrict__ segs, KArgs a,
                                              const R* __restrict__ arena,
                                              const R* __restrict__ dinv, R* __restrict__ y,
                                              R* __restrict__ pb,
                                              const int64_t* __restrict__ pb_off,
                                              int64_t pb_total, int64_t n, int nrhs,
                                              int32_t* __restrict__ state, int32_t ntail,
                                              uint64_t wait_ticks) {
    static_assert(kMaxWidth <= 192, "three 64-lane column sets");
    constexpr int KW = kTriKW;  // columns per wave
    __shared__ R ys[kMaxWidth][NR];
    __shared__ R red[4][NR][kMaxWidth];
    __shared__ int32_t sh_ticket, sh_ok;
    int32_t* turn = state;
    int32_t* ready = turn + ntail;
    int32_t* cntB = ready + ntail;
    int32_t* done = cntB + ntail;
    int32_t* ctrl = done + ntail;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (;;) {
        if (tid == 0) sh_ticket = atomicAdd(ctrl, 1);
        __syncthreads();
        const int32_t t = sh_ticket;
        if (t >= ntasks) break;
        const TailTask tk = tasks[t];
        const int s = tk.s;
        const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
        const int64_t rp = a.rowptr[s];
        const int r = (int)(a.rowptr[s + 1] - rp) - w;
        const R* __restrict__ P = arena + a.sn_off[s] + w;  // rows below the diagonal block
        const R* __restrict__ Li = dinv + a.inv_off[s] + inverse_elems(w);
        const int32_t* __restrict__ below = a.rows + rp + w;
        const uint64_t deadline = wall_clock64() + wait_ticks;
        if (tk.kind == kTailR) {
            const int i0 = tk.rb * kTile, m = min(kTile, r - i0);
            R lv[KW];
#pragma unroll
            for (int u = 0; u < KW; ++u) {
                const int k = wave + 4 * u;
                lv[u] = (lane < m && k < w) ? P[i0 + lane + (int64_t)k * ld] : R(0);
            }
            const int32_t row = lane < m ? below[i0 + lane] : 0;
            if (tid == 0) sh_ok = tail_wait(ready + tk.u, 1, ctrl, deadline);
            __syncthreads();
            if (!sh_ok) break;
            for (int c0 = 0; c0 < nrhs; c0 += NR) {
                const int nc = min(NR, nrhs - c0);
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    ys[k][c] = c < nc ? ld_dev(y + (int64_t)(c0 + c) * n + first + k) : R(0);
                }
                __syncthreads();
                R acc[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
                for (int u = 0; u < KW; ++u) {
                    const int k = wave + 4 * u;
                    if (k < w) {
#pragma unroll
                        for (int c = 0; c < NR; ++c) acc[c] += lv[u] * ys[k][c];
                    }
                }
#pragma unroll
                for (int c = 0; c < NR; ++c) red[wave][c][lane] = acc[c];
                __syncthreads();
                if (tid < m) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        if (c >= nc) break;
                        const R v = (red[0][c][tid] + red[1][c][tid]) +
                                    (red[2][c][tid] + red[3][c][tid]);
                        unsafeAtomicAdd(y + (int64_t)(c0 + c) * n + row, -v);
                    }
                }
                __syncthreads();
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's stores and adds done
            __syncthreads();
            if (tid == 0)
                for (int32_t q = tk.a; q < tk.b; ++q)
                    __hip_atomic_fetch_add(turn + segs[q].u, segs[q].hi - segs[q].lo,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (tk.kind == kTailF) {
            // z = L11^{-1} y_s (tri_first before the wait, tri_rest after)
            R la[KW];
            tri_first<R, false>(Li, w, wave, lane, la);
            if (tid == 0) sh_ok = tk.a == 0 || tail_wait(turn + tk.u, tk.a, ctrl, deadline);
            __syncthreads();
            if (!sh_ok) break;
            for (int c0 = 0; c0 < nrhs; c0 += NR) {
                const int nc = min(NR, nrhs - c0);
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    ys[k][c] = c < nc ? ld_dev(y + (int64_t)(c0 + c) * n + first + k) : R(0);
                }
                __syncthreads();
                tri_rest<R, NR, false>(Li, w, la, ys, red, wave, lane);
                __syncthreads();
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    if (c < nc)
                        st_dev(y + (int64_t)(c0 + c) * n + first + k,
                               (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]));
                }
                __syncthreads();
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's stores and adds done
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(ready + tk.u, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (tk.kind == kTailC) {
            // lane = column (three 64-column sets), wave = 16 rows of the block
            const int i0 = tk.rb * kTile, m = min(kTile, r - i0);
            R pv[3][16];
#pragma unroll
            for (int cs = 0; cs < 3; ++cs) {
                const int k = lane + 64 * cs;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int i = 16 * wave + j;
                    pv[cs][j] = (i < m && k < w) ? P[i0 + i + (int64_t)k * ld] : R(0);
                }
            }
            if (tid == 0) {
                bool g = true;
                for (int32_t q = tk.a; q < tk.b && g; ++q)
                    g = tail_wait(done + segs[q].u, 1, ctrl, deadline);
                sh_ok = g;
            }
            __syncthreads();
            if (!sh_ok) break;
            R* __restrict__ out = pb + pb_off[s] + (int64_t)tk.rb * w;
            for (int c0 = 0; c0 < nrhs; c0 += NR) {
                const int nc = min(NR, nrhs - c0);
                for (int e = tid; e < kTile * NR; e += 256) {
                    const int i = e / NR, c = e % NR;
                    ys[i][c] = (i < m && c < nc) ? ld_dev(y + (int64_t)(c0 + c) * n + below[i0 + i])
                                                 : R(0);
                }
                __syncthreads();
#pragma unroll
                for (int cs = 0; cs < 3; ++cs) {
                    R acc[NR];
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
                    for (int j = 0; j < 16; ++j)
#pragma unroll
                        for (int c = 0; c < NR; ++c) acc[c] += pv[cs][j] * ys[16 * wave + j][c];
                    if (lane + 64 * cs < w) {
#pragma unroll
                        for (int c = 0; c < NR; ++c) red[wave][c][lane + 64 * cs] = acc[c];
                    }
                }
                __syncthreads();
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    if (c < nc)
                        st_dev(out + (int64_t)(c0 + c) * pb_total + k,
                               (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]));
                }
                __syncthreads();
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's stores and adds done
            __syncthreads();
            if (tid == 0)
                __hip_atomic_fetch_add(cntB + tk.u, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {  // kTailB
            // x = L11^{-T} (z_s - t_s) (tri_first before the wait, tri_rest after)
            const R* __restrict__ Lt = Li + w * (w + 1) / 2;
            R la[KW];
            tri_first<R, true>(Lt, w, wave, lane, la);
            // z_s written (a root has no C block to order it), then its C blocks
            if (tid == 0)
                sh_ok = tail_wait(ready + tk.u, 1, ctrl, deadline) &&
                        (tk.a == 0 || tail_wait(cntB + tk.u, tk.a, ctrl, deadline));
            __syncthreads();
            if (!sh_ok) break;
            const R* __restrict__ ps = pb + pb_off[s];
            for (int c0 = 0; c0 < nrhs; c0 += NR) {
                const int nc = min(NR, nrhs - c0);
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    R tsum = R(0);
                    if (c < nc) {
                        const R* __restrict__ pk = ps + (int64_t)(c0 + c) * pb_total + k;
                        for (int h0 = 0; h0 < tk.a; h0 += 8) {
                            R v[8];
#pragma unroll
                            for (int j = 0; j < 8; ++j)
                                v[j] = h0 + j < tk.a ? ld_dev(pk + (int64_t)(h0 + j) * w) : R(0);
#pragma unroll
                            for (int j = 0; j < 8; ++j) tsum += v[j];
                        }
                    }
                    ys[k][c] = c < nc ? ld_dev(y + (int64_t)(c0 + c) * n + first + k) - tsum : R(0);
                }
                __syncthreads();
                tri_rest<R, NR, true>(Lt, w, la, ys, red, wave, lane);
                __syncthreads();
                for (int e = tid; e < w * NR; e += 256) {
                    const int k = e / NR, c = e % NR;
                    if (c < nc)
                        st_dev(y + (int64_t)(c0 + c) * n + first + k,
                               (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]));
                }
                __syncthreads();
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's stores and adds done
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(done + tk.u, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// one right-hand side: each level's sweep in one launch, the diagonal block
// split over workgroups
// ---------------------------------------------------------------------------
//
// A large supernode's diagonal block costs a level kernel most of its time:
// its inverse (up to 11k entries) read by one workgroup.  Each level (below
// the tail) runs instead as one launch per direction whose workgroups split
// that product by parts of kPartRows rows, one workgroup per part, and
// exchange the parts through device-scope stores and a per-supernode count
// (zeroed before each solve; bounded waits as the tail's):
//   forward:  parts   z_s[part] = (L11^{-1} y_s)[part] to zb, then count;
//             blocks  (the 64-row blocks below, which load their part of L21
//                     first) wait for every part of s, then
//                     y[rows] -= L21 z_s as k_fwd_level;
//   backward: blocks  the partial sums of L21^T x[rows below] as k_bwd_cols,
//                     stored at device scope, then count;
//             parts   (which load their rows of L11^{-1} first) wait for
//                     every block of s, then
//                     x_s[part] = (L11^{-T} (z_s - t_s))[part] into y.
// Every waiting workgroup comes after all the workgroups it waits for in
// the launch (the device dispatches a launch's workgroups in index order),
// and those wait on nothing, so the waits end whatever the number of
// resident workgroups.  A part's product: 16 threads per row,
// each over every 16th column, then a butterfly over the 16; one fixed
// order, so a solve has the same bits on every run.  A wait that passes its
// bound sets the abort and error words and leaves NaN in its outputs.

__device__ __forceinline__ bool split_wait(const int32_t* p, int32_t want, int32_t* ctrl,
                                           uint64_t deadline) {
    return tail_wait(p, want, ctrl, deadline);
}

template <class R>
__global__ __launch_bounds__(256) void k_fwd_split(const RowBlock* __restrict__ parts,
                                                   int32_t nparts,
                                                   const RowBlock* __restrict__ work, KArgs a,
                                                   const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, R* __restrict__ zb,
                                                   int64_t n, SolveBufs<R> sb,
                                                   int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ ctrl, uint64_t ticks,
                                                   int32_t extra) {
    constexpr int KW = kTriKW;  // columns per wave
    constexpr int kPer = (kMaxWidth + 15) / 16;  // a part thread's columns
    __shared__ R ys[kMaxWidth];
    __shared__ R red[4][kTile];
    __shared__ int ok_sh;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if ((int)blockIdx.x < nparts) {
        const RowBlock pt = parts[blockIdx.x];
        const int s = pt.s, w = a.sn_w[s], first = a.sn_first[s];
        // L11^{-T}, packed upper by columns: row i of L11^{-1} is contiguous
        const R* __restrict__ LT = dinv + a.inv_off[s] + inverse_elems(w) + w * (w + 1) / 2;
        const int i = pt.rb * kPartRows + (tid >> 4), j = tid & 15;
        R lv[kPer], yv[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = j + 16 * t;
            const bool in = i < w && k <= i;
            lv[t] = in ? LT[(i * (i + 1) >> 1) + k] : R(0);
            yv[t] = in ? y[first + k] : R(0);
        }
        R acc = R(0);
#pragma unroll
        for (int t = 0; t < kPer; ++t) acc += lv[t] * yv[t];
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (j == 0 && i < w) st_dev(zb + first + i, acc);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(cnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const RowBlock wb = work[blockIdx.x - nparts];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const int i0 = wb.rb * kTile, m = max(0, min(kTile, r - i0));
    if (m == 0) return;  // a supernode with no rows below: its parts did the work
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const int32_t* __restrict__ below = a.rows + rp + w;
    R lv[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = wave + 4 * u;
        lv[u] = (lane < m && k < w) ? P[i0 + lane + (int64_t)k * ld] : R(0);
    }
    const int64_t slot = rp + w + i0 + tid;
    const int32_t row = tid < m ? below[i0 + tid] : 0;
    const bool sh = tid < m && sb.shared[slot];
    const R yold = (tid < m && !sh) ? y[row] : R(0);
    if (tid == 0)
        ok_sh = split_wait(cnt + s, (w + kPartRows - 1) / kPartRows + extra, ctrl,
                           wall_clock64() + ticks);
    __syncthreads();
    const bool ok = ok_sh;
    for (int k = tid; k < w; k += 256) ys[k] = ok ? ld_dev(zb + first + k) : R(NAN);
    __syncthreads();
    R acc = R(0);
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = wave + 4 * u;
        if (k < w) acc += lv[u] * ys[k];
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (tid < m) {
        const R v = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
        if (sh) sb.cb[slot] = v;
        else y[row] = yold - v;
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_bwd_split(const ColBlk* __restrict__ work,
                                                   int32_t nblk,
                                                   const RowBlock* __restrict__ parts, KArgs a,
                                                   const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, const R* __restrict__ zb,
                                                   R* __restrict__ pb,
                                                   const int64_t* __restrict__ pb_off,
                                                   int64_t pb_total, int64_t n,
                                                   int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ ctrl, uint64_t ticks,
                                                   int32_t extra) {
    constexpr int G = kColGroup;
    constexpr int kPer = (kMaxWidth + 15) / 16;
    __shared__ R part[4][G];
    __shared__ R us[kMaxWidth];
    __shared__ int ok_sh;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if ((int)blockIdx.x < nblk) {
        // partial sums of L21^T y[rows] for the block's columns and rows, as k_bwd_cols
        const ColBlk wb = work[blockIdx.x];
        const int s = wb.s, g = wb.g, h = wb.h;
        const int w = a.sn_w[s], ld = a.sn_ld[s];
        const int64_t rp = a.rowptr[s];
        const int k0 = g * G, kc = min(G, w - k0);
        const int rb0 = h * kRowChunk;
        const int r = min((int)(a.rowptr[s + 1] - rp) - w - rb0, kRowChunk);
        const R* __restrict__ P = arena + a.sn_off[s] + w + rb0 + (int64_t)k0 * ld;
        const int32_t* __restrict__ below = a.rows + rp + w + rb0;
        R* __restrict__ out = pb + pb_off[s] + (int64_t)h * w + k0;
        if (r <= 128) {
            // a short chunk: the waves split the columns instead of the rows.
            // r <= 64: wave q sums columns kQ q .. kQ q + kQ - 1 over every
            // row (lane = row); else waves 2c and 2c + 1 sum columns
            // 2 kQ c .. over rows 0-63 and 64-127.  Each column's sum takes
            // the same products in the same lanes and order as the general
            // path below, whose other waves add zeros here.
            constexpr int kQ = G / 4;
            static_assert(G % 4 == 0, "four waves share a column group");
            const bool one = r <= 64;
            const int c0 = one ? wave * kQ : (wave >> 1) * (2 * kQ);
            const int ncw = one ? kQ : 2 * kQ;
            const int i = one ? lane : lane + 64 * (wave & 1);
            const int32_t row = i < r ? below[i] : 0;
            const R yv = i < r ? y[row] : R(0);
            R v[2 * kQ];
#pragma unroll
            for (int k = 0; k < 2 * kQ; ++k) {
                const int c = c0 + k;
                const R pv = (k < ncw && i < r && c < kc) ? P[i + (int64_t)c * ld] : R(0);
                v[k] = R(0);
                v[k] += pv * yv;
            }
#pragma unroll
            for (int k = 0; k < 2 * kQ; ++k) {
                if (k < ncw) {
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
                    if (lane == 0) part[wave][c0 + k] = v[k];
                }
            }
            __syncthreads();
            if (tid < kc) {
                const int c = tid / (2 * kQ);
                st_dev(out + tid,
                       one ? part[tid / kQ][tid] : part[2 * c][tid] + part[2 * c + 1][tid]);
            }
        } else {
            R acc[G];
#pragma unroll
            for (int k = 0; k < G; ++k) acc[k] = R(0);
            for (int i0 = tid; i0 < r; i0 += 256 * 4) {
                R yv[4], pv[4][G];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + 256 * u;
                    const int32_t row = i < r ? below[i] : 0;
                    yv[u] = i < r ? y[row] : R(0);
#pragma unroll
                    for (int k = 0; k < G; ++k)
                        pv[u][k] = (i < r && k < kc) ? P[i + (int64_t)k * ld] : R(0);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < G; ++k) acc[k] += pv[u][k] * yv[u];
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                R v = acc[k];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                if (lane == 0) part[wave][k] = v;
            }
            __syncthreads();
            if (tid < kc)
                st_dev(out + tid, (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]));
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(cnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const RowBlock pt = parts[blockIdx.x - nblk];
    const int s = pt.s, w = a.sn_w[s], first = a.sn_first[s];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const int nh = r > 0 ? (r + kRowChunk - 1) / kRowChunk : 0;
    const int nblk_s = nh * ((w + G - 1) / G);
    // L11^{-1}, packed lower by columns: column i (rows i .. w - 1) is contiguous
    const R* __restrict__ Li = dinv + a.inv_off[s] + inverse_elems(w);
    const int p0 = pt.rb * kPartRows;
    const int i = p0 + (tid >> 4), j = tid & 15;
    R lv[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = i + j + 16 * t;
        lv[t] = (i < w && k < w) ? Li[((i * (2 * w - i - 1)) >> 1) + k] : R(0);
    }
    if (tid == 0)
        ok_sh = nblk_s == 0 || split_wait(cnt + s, nblk_s + extra, ctrl, wall_clock64() + ticks);
    __syncthreads();
    const bool ok = ok_sh;
    // u = z_s - t_s for the columns from the part's first row on, the chunks'
    // partial sums in chunk order
    for (int k = p0 + tid; k < w; k += 256) {
        R t = R(0);
        const R* __restrict__ pk = pb + (r > 0 ? pb_off[s] : 0) + k;
        for (int h0 = 0; h0 < nh; h0 += 8) {
            R v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = h0 + q < nh ? ld_dev(pk + (int64_t)(h0 + q) * w) : R(0);
#pragma unroll
            for (int q = 0; q < 8; ++q) t += v[q];
        }
        us[k] = ok ? zb[first + k] - t : R(NAN);
    }
    __syncthreads();
    R acc = R(0);
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = i + j + 16 * t;
        if (i < w && k < w) acc += lv[t] * us[k];
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (j == 0 && i < w) y[first + i] = acc;
}

// The same split launches for NR right-hand sides at a time (groups of NR
// columns in turn): a part stages y_s (or u) for its group in LDS, each
// thread keeps NR sums; the 64-row blocks below as k_fwd_level and the
// column blocks as k_bwd_cols_multi, with device-scope stores and counts.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_fwd_split_m(const RowBlock* __restrict__ parts,
                                                     int32_t nparts,
                                                     const RowBlock* __restrict__ work, KArgs a,
                                                     const R* __restrict__ arena,
                                                     const R* __restrict__ dinv,
                                                     R* __restrict__ y, R* __restrict__ zb,
                                                     int64_t n, int nrhs, SolveBufs<R> sb,
                                                     int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ ctrl, uint64_t ticks,
                                                     int32_t extra) {
    constexpr int KW = kTriKW;
    constexpr int kPer = (kMaxWidth + 15) / 16;
    __shared__ R ys[kMaxWidth][NR + 1];
    __shared__ R red[4][NR][kTile];
    __shared__ int ok_sh;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if ((int)blockIdx.x < nparts) {
        const RowBlock pt = parts[blockIdx.x];
        const int s = pt.s, w = a.sn_w[s], first = a.sn_first[s];
        const R* __restrict__ LT = dinv + a.inv_off[s] + inverse_elems(w) + w * (w + 1) / 2;
        const int i = pt.rb * kPartRows + (tid >> 4), j = tid & 15;
        R lv[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = j + 16 * t;
            lv[t] = (i < w && k <= i) ? LT[(i * (i + 1) >> 1) + k] : R(0);
        }
        const int kend = min(w, pt.rb * kPartRows + kPartRows);  // columns the part needs
        for (int c0 = 0; c0 < nrhs; c0 += NR) {
            const int nc = min(NR, nrhs - c0);
            for (int e = tid; e < kend * NR; e += 256) {
                const int k = e / NR, c = e % NR;
                ys[k][c] = c < nc ? y[(int64_t)(c0 + c) * n + first + k] : R(0);
            }
            __syncthreads();
            R acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
            for (int t = 0; t < kPer; ++t) {
                const int k = j + 16 * t;
                if (i < w && k <= i) {
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += lv[t] * ys[k][c];
                }
            }
#pragma unroll
            for (int c = 0; c < NR; ++c) {
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
                if (j == 0 && i < w && c < nc) st_dev(zb + (int64_t)(c0 + c) * n + first + i, acc[c]);
            }
            __syncthreads();
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(cnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const RowBlock wb = work[blockIdx.x - nparts];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const int i0 = wb.rb * kTile, m = max(0, min(kTile, r - i0));
    if (m == 0) return;
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const int32_t* __restrict__ below = a.rows + rp + w;
    R lv[KW];
#pragma unroll
    for (int u = 0; u < KW; ++u) {
        const int k = wave + 4 * u;
        lv[u] = (lane < m && k < w) ? P[i0 + lane + (int64_t)k * ld] : R(0);
    }
    const int64_t slot = rp + w + i0 + tid;
    const int32_t row = tid < m ? below[i0 + tid] : 0;
    const bool sh = tid < m && sb.shared[slot];
    if (tid == 0)
        ok_sh = split_wait(cnt + s, (w + kPartRows - 1) / kPartRows + extra, ctrl,
                           wall_clock64() + ticks);
    __syncthreads();
    const bool ok = ok_sh;
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        R yold[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            yold[c] = (tid < m && !sh && c < nc) ? y[(int64_t)(c0 + c) * n + row] : R(0);
        for (int e = tid; e < w * NR; e += 256) {
            const int k = e / NR, c = e % NR;
            ys[k][c] = c < nc ? (ok ? ld_dev(zb + (int64_t)(c0 + c) * n + first + k) : R(NAN))
                              : R(0);
        }
        __syncthreads();
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
        for (int u = 0; u < KW; ++u) {
            const int k = wave + 4 * u;
            if (k < w) {
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += lv[u] * ys[k][c];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) red[wave][c][lane] = acc[c];
        __syncthreads();
        if (tid < m) {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                if (c >= nc) break;
                const R v = (red[0][c][tid] + red[1][c][tid]) + (red[2][c][tid] + red[3][c][tid]);
                if (sh) sb.cb[(int64_t)(c0 + c) * sb.nslots + slot] = v;
                else y[(int64_t)(c0 + c) * n + row] = yold[c] - v;
            }
        }
        __syncthreads();
    }
}

template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_split_m(const ColBlk* __restrict__ work,
                                                     int32_t nblk,
                                                     const RowBlock* __restrict__ parts, KArgs a,
                                                     const R* __restrict__ arena,
                                                     const R* __restrict__ dinv,
                                                     R* __restrict__ y, const R* __restrict__ zb,
                                                     R* __restrict__ pb,
                                                     const int64_t* __restrict__ pb_off,
                                                     int64_t pb_total, int64_t n, int nrhs,
                                                     int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ ctrl, uint64_t ticks,
                                                     int32_t extra) {
    constexpr int G = kColGroup;
    static_assert(G * NR * 4 == 256, "one thread per (column, right-hand side, quarter)");
    constexpr int kRows = 256;
    constexpr int kPer = (kMaxWidth + 15) / 16;
    __shared__ R Ls[kRows][G + 1];
    __shared__ R Xs[kRows][NR + 1];
    __shared__ R part[4][G][NR];
    __shared__ int ok_sh;
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < nblk) {
        // the column block's partial sums, as k_bwd_cols_multi
        const ColBlk wb = work[blockIdx.x];
        const int s = wb.s, g = wb.g, h = wb.h;
        const int w = a.sn_w[s], ld = a.sn_ld[s];
        const int64_t rp = a.rowptr[s];
        const int k0 = g * G, kc = min(G, w - k0);
        const int rb0 = h * kRowChunk;
        const int r = min((int)(a.rowptr[s + 1] - rp) - w - rb0, kRowChunk);
        const R* __restrict__ P = arena + a.sn_off[s] + w + rb0 + (int64_t)k0 * ld;
        const int32_t* __restrict__ below = a.rows + rp + w + rb0;
        R* __restrict__ out = pb + pb_off[s] + (int64_t)h * w + k0;
        const int k = tid % G, c = (tid / G) % NR, q = tid / (G * NR);
        for (int c0 = 0; c0 < nrhs; c0 += NR) {
            const int nc = min(NR, nrhs - c0);
            R acc = R(0);
            for (int i0 = 0; i0 < r; i0 += kRows) {
                const int i = i0 + tid;
                const int32_t row = i < r ? below[i] : 0;
                R lv[G], xv[NR];
#pragma unroll
                for (int kk = 0; kk < G; ++kk)
                    lv[kk] = (i < r && kk < kc) ? P[i + (int64_t)kk * ld] : R(0);
#pragma unroll
                for (int cc = 0; cc < NR; ++cc)
                    xv[cc] = (i < r && cc < nc) ? y[(int64_t)(c0 + cc) * n + row] : R(0);
#pragma unroll
                for (int kk = 0; kk < G; ++kk) Ls[tid][kk] = lv[kk];
#pragma unroll
                for (int cc = 0; cc < NR; ++cc) Xs[tid][cc] = xv[cc];
                __syncthreads();
                const int j0 = q * (kRows / 4);
#pragma unroll 8
                for (int jj = j0; jj < j0 + kRows / 4; ++jj) acc += Ls[jj][k] * Xs[jj][c];
                __syncthreads();
            }
            part[q][k][c] = acc;
            __syncthreads();
            if (tid < G * NR) {
                const int kk = tid % G, cc = tid / G;
                if (kk < kc && cc < nc)
                    st_dev(out + (int64_t)(c0 + cc) * pb_total + kk,
                           (part[0][kk][cc] + part[1][kk][cc]) + (part[2][kk][cc] + part[3][kk][cc]));
            }
            __syncthreads();
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(cnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    R (*us)[NR + 1] = Xs;  // u = z_s - t_s by column, from the part's first row on
    const RowBlock pt = parts[blockIdx.x - nblk];
    const int s = pt.s, w = a.sn_w[s], first = a.sn_first[s];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const int nh = r > 0 ? (r + kRowChunk - 1) / kRowChunk : 0;
    const int nblk_s = nh * ((w + G - 1) / G);
    const R* __restrict__ Li = dinv + a.inv_off[s] + inverse_elems(w);
    const int p0 = pt.rb * kPartRows;
    const int i = p0 + (tid >> 4), j = tid & 15;
    R lv[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = i + j + 16 * t;
        lv[t] = (i < w && k < w) ? Li[((i * (2 * w - i - 1)) >> 1) + k] : R(0);
    }
    if (tid == 0)
        ok_sh = nblk_s == 0 || split_wait(cnt + s, nblk_s + extra, ctrl, wall_clock64() + ticks);
    __syncthreads();
    const bool ok = ok_sh;
    const R* __restrict__ ps = pb + (r > 0 ? pb_off[s] : 0);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < (w - p0) * NR; e += 256) {
            const int k = p0 + e / NR, c = e % NR;
            R t = R(0);
            if (c < nc) {
                const R* __restrict__ pk = ps + (int64_t)(c0 + c) * pb_total + k;
                for (int h0 = 0; h0 < nh; h0 += 8) {
                    R v[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        v[q] = h0 + q < nh ? ld_dev(pk + (int64_t)(h0 + q) * w) : R(0);
#pragma unroll
                    for (int q = 0; q < 8; ++q) t += v[q];
                }
            }
            us[k - p0][c] = c < nc ? (ok ? zb[(int64_t)(c0 + c) * n + first + k] - t : R(NAN)) : R(0);
        }
        __syncthreads();
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = i + j + 16 * t;
            if (i < w && k < w) {
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += lv[t] * us[k - p0][c];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
            if (j == 0 && i < w && c < nc) y[(int64_t)(c0 + c) * n + first + i] = acc[c];
        }
        __syncthreads();
    }
}

int32_t configure_solve_kernels() { return OK; }

namespace {

// The level sweeps of one solve on the work array (factor type): y, then z
// (the forward result of the large supernodes), the contribution slots and
// the backward partial sums, each nrhs columns; as enqueued on stream st.  Gather and scatter stay outside: they
// touch the caller's b and x, which change from call to call.
template <class R, int NR>
void enqueue_sweeps(spc_numeric* num, int32_t nrhs, R* work, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const int64_t n = S.n;
    const KArgs a = kargs(P);
    const R* arena = (const R*)num->arena;
    const R* dinv = (const R*)num->dinv;
    R* y = work;
    R* zb = y + n * nrhs;
    R* cb = zb + n * nrhs;
    R* pb = cb + P->nslots * nrhs;
    const SolveBufs<R> sb{cb, P->nslots, P->slot_shared};
    const int32_t nl = P->tail_l0;  // levels below the tail go level by level
    // the split level launches' counts (forward, backward, then the control
    // words: ctrl[1] abort, ctrl[2] error, as tail_wait uses them), zeroed here
    int32_t* cnt = (int32_t*)(pb + P->pb_total * nrhs) + tail_state_words(S);
    const int64_t cwords = split_state_words(S);
    uint64_t split_ticks = 0;
    if (nl > 0) {
        hipLaunchKernelGGL(k_tail_reset, dim3((unsigned)((cwords + 255) / 256)), dim3(256), 0,
                           st, cnt, cwords);
        int dev = 0, clock_khz = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
        const int64_t lim = S.opt.spin_limit > 0 ? S.opt.spin_limit : (int64_t)10000000;
        split_ticks = (uint64_t)lim * (uint64_t)std::max(1, clock_khz) / 1000;
    }
    int32_t* cnt_f = cnt;
    int32_t* cnt_b = cnt + S.nsup;
    int32_t* ctrl = cnt + 2 * S.nsup;
    // debug bit 0 withholds one count from every wait, so that each bound fires
    const int32_t extra = (S.opt.debug_flags & 1) ? 1 : 0;
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        launch_small_solve(num, a, P->small_rec + n0 + nbig, n1 - n0 - nbig, P->small_maxw[l],
                           P->small_maxm[l], y, cb, n, nrhs, true, st);
        const int64_t f0 = P->fwdblk_ptr[l], f1 = P->fwdblk_ptr[l + 1];
        const int64_t p0 = P->sspart_ptr[l], p1 = P->sspart_ptr[l + 1];
        if (p1 > p0) {
            if constexpr (NR == 1)
                hipLaunchKernelGGL(k_fwd_split<R>, dim3((unsigned)((p1 - p0) + (f1 - f0))),
                                   dim3(256), 0, st, P->sspart + p0, (int32_t)(p1 - p0),
                                   P->fwdblk + f0, a, arena, dinv, y, zb, n, sb, cnt_f, ctrl,
                                   split_ticks, extra);
            else
                hipLaunchKernelGGL((k_fwd_split_m<R, NR>),
                                   dim3((unsigned)((p1 - p0) + (f1 - f0))), dim3(256), 0, st,
                                   P->sspart + p0, (int32_t)(p1 - p0), P->fwdblk + f0, a, arena,
                                   dinv, y, zb, n, nrhs, sb, cnt_f, ctrl, split_ticks, extra);
        } else if (f1 > f0)
            hipLaunchKernelGGL((k_fwd_level<R, NR>), dim3((unsigned)(f1 - f0)), dim3(256), 0, st,
                               P->fwdblk + f0, a, arena, dinv, y, zb, n, nrhs, sb);
        const int64_t i0 = P->red_level_ptr[l], i1 = P->red_level_ptr[l + 1];
        if (i1 > i0) {
            const int64_t work_items = (i1 - i0) * nrhs;
            hipLaunchKernelGGL(k_fwd_reduce<R>, dim3((unsigned)((work_items + 255) / 256)),
                               dim3(256), 0, st, P->red_row + i0, P->red_ptr + i0,
                               (const int32_t*)P->red_slot, i1 - i0, y, n, nrhs, sb);
        }
    }
    if (P->ntail_tasks > 0) {
        int32_t* state = (int32_t*)(pb + P->pb_total * nrhs);
        const int64_t words = 4 * (int64_t)P->ntail + 4;
        hipLaunchKernelGGL(k_tail_reset, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                           state, words);
        int per_cu = 0, ncu = 0, dev = 0, clock_khz = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tail<R, NR>, 256, 0);
        const int64_t workers = std::min<int64_t>(
            P->ntail_tasks, (int64_t)std::max(1, ncu) * std::max(1, per_cu));
        const int64_t lim = S.opt.spin_limit > 0 ? S.opt.spin_limit : (int64_t)10000000;
        const uint64_t ticks = (uint64_t)lim *
                               (uint64_t)std::max(1, clock_khz) / 1000;
        hipLaunchKernelGGL((k_tail<R, NR>), dim3((unsigned)workers), dim3(256), 0, st,
                           (const TailTask*)P->tail_tasks, P->ntail_tasks,
                           (const TailSeg*)P->tail_segs, a, arena, dinv, y, pb,
                           (const int64_t*)P->pb_off, P->pb_total, n, nrhs, state, P->ntail,
                           ticks);
    }
    for (int32_t l = nl - 1; l >= 0; --l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        const int64_t g0 = P->colblk_ptr[l], g1 = P->colblk_ptr[l + 1];
        const int64_t p0 = P->sspart_ptr[l], p1 = P->sspart_ptr[l + 1];
        if (p1 > p0) {
            if constexpr (NR == 1)
                hipLaunchKernelGGL(k_bwd_split<R>, dim3((unsigned)((g1 - g0) + (p1 - p0))),
                                   dim3(256), 0, st, P->colblk + g0, (int32_t)(g1 - g0),
                                   P->sspart + p0, a, arena, dinv, y, (const R*)zb, pb,
                                   (const int64_t*)P->pb_off, P->pb_total, n, cnt_b, ctrl,
                                   split_ticks, extra);
            else
                hipLaunchKernelGGL((k_bwd_split_m<R, NR>),
                                   dim3((unsigned)((g1 - g0) + (p1 - p0))), dim3(256), 0, st,
                                   P->colblk + g0, (int32_t)(g1 - g0), P->sspart + p0, a, arena,
                                   dinv, y, (const R*)zb, pb, (const int64_t*)P->pb_off,
                                   P->pb_total, n, nrhs, cnt_b, ctrl, split_ticks, extra);
        } else if (g1 > g0) {
            if constexpr (NR == 1)
                hipLaunchKernelGGL((k_bwd_cols<R, NR>), dim3((unsigned)(g1 - g0)), dim3(256), 0,
                                   st, P->colblk + g0, a, arena, (const R*)y, pb,
                                   (const int64_t*)P->pb_off, P->pb_total, n, nrhs);
            else
                hipLaunchKernelGGL((k_bwd_cols_multi<R, NR>), dim3((unsigned)(g1 - g0)),
                                   dim3(256), 0, st, P->colblk + g0, a, arena, (const R*)y, pb,
                                   (const int64_t*)P->pb_off, P->pb_total, n, nrhs);
        }
        if (nbig > 0 && p1 <= p0)
            hipLaunchKernelGGL((k_bwd_diag<R, NR>), dim3((unsigned)nbig), dim3(256), 0, st,
                               P->level_sn + n0, a, dinv, y, (const R*)zb, (const R*)pb,
                               (const int64_t*)P->pb_off, P->pb_total, n, nrhs);
        launch_small_solve(num, a, P->small_rec + n0 + nbig, n1 - n0 - nbig, P->small_maxw[l],
                           P->small_maxm[l], y, cb, n, nrhs, false, st);
    }
}

size_t elem_size(const spc_numeric* num) { return num->prec == 1 ? sizeof(float) : sizeof(double); }

}  // namespace

void drop_solve_graphs(spc_numeric* num) {
    for (auto& g : num->solve_graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    num->solve_graphs.clear();
}

// y, z, contribution slots and partial sums per right-hand side, then the
// tail's task state (int32 words, rounded up to whole elements of 4 bytes or
// more).
int64_t solve_work_elems(const spc_numeric* num, int32_t nrhs) {
    const Symbolic& S = num->sym->S;
    const int64_t words = tail_state_words(S) + split_state_words(S);
    const int64_t esz = num->prec == 1 ? 4 : 8;
    return solve_work_elems_per_rhs(S) * (int64_t)nrhs + (words * 4 + esz - 1) / esz;
}

int64_t solve_work_elems_per_rhs(const Symbolic& S) {
    return 2 * S.n + (int64_t)S.rows.size() + solve_pb_elems(S);  // y, z, slots, partial sums
}

// Solve work for nrhs right-hand sides (factor type): the vectors y and z
// (n x nrhs each), the forward contribution slots (nslots x nrhs), the
// backward partial sums (pb_total x nrhs).
int32_t ensure_solve_work(spc_numeric* num, int32_t nrhs) {
    if (num->work_cols >= nrhs) return OK;
    if (num->work) {
        HIP_TRY(hipDeviceSynchronize());
        drop_solve_graphs(num);
        HIP_TRY(hipFree(num->work));
        num->work = nullptr;
        num->work_cols = 0;
    }
    const int64_t elems = std::max<int64_t>(solve_work_elems(num, nrhs), 1);
    if (hipMalloc(&num->work, elem_size(num) * (size_t)elems) != hipSuccess) return ERR_OOM;
    num->work_cols = nrhs;
    return OK;
}

// Replays (capturing on first use) the sweeps for nrhs columns on stream st.
int32_t run_sweeps(spc_numeric* num, int32_t nrhs, hipStream_t st) {
    spc_numeric::SolveGraph* sg = nullptr;
    for (auto& e : num->solve_graphs)
        if (e.nrhs == nrhs) sg = &e;
    if (!sg) {
        if (!num->capture) HIP_TRY(hipStreamCreateWithFlags(&num->capture, hipStreamNonBlocking));
        spc_numeric::SolveGraph e;
        e.nrhs = nrhs;
        HIP_TRY(hipStreamBeginCapture(num->capture, hipStreamCaptureModeThreadLocal));
        if (num->prec == 1) {
            float* y = (float*)num->work;
            if (nrhs == 1) enqueue_sweeps<float, 1>(num, nrhs, y, num->capture);
            else enqueue_sweeps<float, kRhs>(num, nrhs, y, num->capture);
        } else {
            double* y = (double*)num->work;
            if (nrhs == 1) enqueue_sweeps<double, 1>(num, nrhs, y, num->capture);
            else enqueue_sweeps<double, kRhs>(num, nrhs, y, num->capture);
        }
        const hipError_t ce = hipStreamEndCapture(num->capture, &e.graph);
        if (ce != hipSuccess || !e.graph) return ERR_HIP;
        if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(e.graph);
            return ERR_HIP;
        }
        num->solve_graphs.push_back(e);
        sg = &num->solve_graphs.back();
    }
    HIP_TRY(hipGraphLaunch(sg->exec, st));
    return OK;
}

namespace {

// Gather, sweeps and scatter of one solve on the work array `work` (factor
// type; solve_work_elems(num, nrhs) elements).  graph: the sweeps replay from
// the factor's captured graph (work must be num->work); otherwise they are
// launched directly on st.
int32_t enqueue_solve(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                      int64_t ldx, void* work, bool graph, hipStream_t st) {
    const DevicePlan* P = num->plan;
    const int64_t n = num->sym->S.n;
    const int64_t total = n * nrhs;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
    if (num->prec == 1)
        hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(256), 0, st, b, ldb, P->perm,
                           (float*)work, n, nrhs);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(g), dim3(256), 0, st, b, ldb, P->perm,
                           (double*)work, n, nrhs);
    if (graph) {
        const int32_t r = run_sweeps(num, nrhs, st);
        if (r != OK) return r;
    } else if (num->prec == 1) {
        if (nrhs == 1) enqueue_sweeps<float, 1>(num, nrhs, (float*)work, st);
        else enqueue_sweeps<float, kRhs>(num, nrhs, (float*)work, st);
    } else {
        if (nrhs == 1) enqueue_sweeps<double, 1>(num, nrhs, (double*)work, st);
        else enqueue_sweeps<double, kRhs>(num, nrhs, (double*)work, st);
    }
    if (num->prec == 1)
        hipLaunchKernelGGL(k_scatter<float>, dim3(g), dim3(256), 0, st, (const float*)work,
                           P->perm, x, ldx, n, nrhs);
    else
        hipLaunchKernelGGL(k_scatter<double>, dim3(g), dim3(256), 0, st, (const double*)work,
                           P->perm, x, ldx, n, nrhs);
    HIP_TRY(hipGetLastError());
    return OK;
}

}  // namespace

int32_t run_solve(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                  int64_t ldx, hipStream_t st) {
    if (num->sym->S.n == 0 || nrhs == 0) return OK;
    const int32_t r = ensure_solve_work(num, nrhs);
    if (r != OK) return r;
    // the sweeps replay from a graph captured once per right-hand-side count
    return enqueue_solve(num, nrhs, b, ldb, x, ldx, num->work, true, st);
}

// ---------------------------------------------------------------------------
// solve without allocation
// ---------------------------------------------------------------------------

// Work of spc_solve_noalloc: one static array per device, held until the
// process ends.  Every element a solve reads it has written first (the
// sweeps zero their own counts), so no part needs clearing between calls.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
__device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

// Device address of `scratch` on each device, taken once per device with that
// device current (host code never passes the symbol itself to a kernel).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return OK;
}

}  // namespace

}  // namespace spc

extern "C" spc_status spc_solve_noalloc(spc_numeric* num, int32_t nrhs, const double* b_dev,
                                        int64_t ldb, double* x_dev, int64_t ldx,
                                        void* stream) {
    using namespace spc;
    if (!num || nrhs < 0) return SPC_ERR_ARG;
    const int64_t n = num->sym->S.n;
    if (nrhs > 0 && n > 0 && (!b_dev || !x_dev || ldb < n || ldx < n)) return SPC_ERR_ARG;
    if (b_dev == x_dev && ldb != ldx) return SPC_ERR_ARG;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SPC_ERR_HIP;
    if (cur != num->device) return SPC_ERR_ARG;
    const size_t elem = num->prec == 1 ? sizeof(float) : sizeof(double);
    if ((size_t)solve_work_elems(num, nrhs) * elem > kNoAllocBytes) return SPC_ERR_TOO_LARGE;
    void* work = nullptr;
    int32_t st = scratch_on(cur, &work);
    if (st != OK) return st;
    st = num->status_known ? num->host_status : spc_numeric_status(num);
    if (st != SPC_OK) return st;
    if (n == 0 || nrhs == 0) return SPC_OK;
    return enqueue_solve(num, nrhs, b_dev, ldb, x_dev, ldx, work, false, (hipStream_t)stream);
}
