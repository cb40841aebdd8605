// Supernodal triangular solves on gfx950 (the two solves of Section II-A of
// arXiv:1608.00044): y = L^{-1} P b by a forward sweep over the supernodal
// elimination tree from the leaves, then z = L^{-T} y from the root back, and
// x = P^T z.  Both sweeps go level by level; within a level every supernode
// is independent.  Per level:
//   forward:  k_fwd_diag   -- y_s = L11^{-1} y_s, one workgroup per supernode,
//                             by 16-column panels using the inverted 16 x 16
//                             diagonal blocks the factorization kept;
//             k_fwd_gemv   -- y[rows below] -= L21 y_s for every 64-row block
//                             of the panel; a row that another source of the
//                             level also updates gets its value in a
//                             contribution slot instead,
//             k_fwd_reduce -- which one thread per such row subtracts, sources
//                             in increasing order;
//   backward: k_bwd_cols   -- partial sums of L21^T y[rows below], one
//                             workgroup per group of kColGroup columns and
//                             chunk of kRowChunk rows, summed in a fixed tree;
//             k_bwd_diag   -- y_s = L11^{-T} (y_s - t_s), t_s the chunks'
//                             partial sums in chunk order, panels in reverse.
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

// Threads of the diagonal-block solve kernels: eight waves, each solving its
// own right-hand sides after the workgroup has staged the block.
constexpr int kDiagThreads = 512;
constexpr int kDiagRegionMax = (kMaxWidth / kPanel) * kPanel * kPanel +
                               (kMaxWidth % kPanel) * (kMaxWidth % kPanel) +
                               kMaxWidth * (kMaxWidth + 1) / 2;

// Stages the supernode's region of dinv (compact diagonal-block inverses,
// then the packed L11) into LDS in one sweep with every load in flight: T gets
// the packed lower triangle (entry (i, j) at cst(j) + i), I every panel's
// inverse as a zero-padded 16 x 16 row-major block.
template <class R>
__device__ __forceinline__ void stage_block(R* __restrict__ T, R* __restrict__ I,
                                            const R* __restrict__ region, int w, int tid) {
    constexpr int kPer = (kDiagRegionMax + kDiagThreads - 1) / kDiagThreads;
    const int ninv = (int)inverse_elems(w);
    const int total = ninv + w * (w + 1) / 2;
    const int plast = w / kPanel, jbl = w % kPanel;  // trailing partial panel, if any
    R v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kDiagThreads;
        v[u] = e < total ? region[e] : R(0);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kDiagThreads;
        if (e >= total) continue;
        if (e >= ninv) {
            T[e - ninv] = v[u];
        } else {
            const int p = e >> 8, q = e & 255;
            if (p < plast) I[e] = v[u];  // full panel: already 16 x 16
            else I[p * kPanel * kPanel + (q / jbl) * kPanel + q % jbl] = v[u];
        }
    }
    if (jbl) {  // zero padding of the partial panel
        for (int e = tid; e < kPanel * kPanel; e += kDiagThreads)
            if ((e >> 4) >= jbl || (e & 15) >= jbl) I[plast * kPanel * kPanel + e] = R(0);
    }
}

// Right-hand sides go through the row-block kernels NR at a time (NR = 1,
// or kRhs for several): the block of L21 is read once per group and every
// thread keeps NR partial sums.
constexpr int kRhs = 8;
constexpr int kPs = kTile + 1;  // padded LDS column stride of a staged 64-row block of L21

// Stages rows [i0, i0 + 64) of the w columns of a panel block into LDS,
// column by column (Pl[k * kPs + i]), zero past the m valid rows; sixteen
// independent loads per thread in flight.
template <class R>
__device__ __forceinline__ void stage_rows(R* __restrict__ Pl, const R* __restrict__ P, int ld,
                                           int i0, int m, int w, int tid) {
    constexpr int kPer = (kTile * kMaxWidth + 255) / 256;
    const int total = kTile * w;
    R v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * 256, k = e >> 6, i = e & 63;
        v[u] = (e < total && i < m) ? P[i0 + i + (int64_t)k * ld] : R(0);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * 256;
        if (e < total) Pl[(e >> 6) * kPs + (e & 63)] = v[u];
    }
}

// Diagonal block, forward: y_s = L11^{-1} y_s.  The workgroup stages L11
// (packed lower triangle) and the 16 x 16 diagonal-block inverses in LDS;
// then each wave solves its own right-hand sides with no workgroup barrier,
// right-looking by panels:
//   y_p = inv(D_p) y_p                      (lane (j, part): four products,
//                                             the parts meet by cross-lane adds)
//   y[k] -= L[k, p] y_p for every k below   (one row per lane, the sixteen
//                                             y_p values broadcast in registers)
template <class R>
__global__ __launch_bounds__(kDiagThreads) void k_fwd_diag(const int32_t* __restrict__ level_sn,
                                                           KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ dinv, R* __restrict__ y,
                                                  int64_t n, int nrhs) {
    extern __shared__ double sm_raw[];
    R* sm = (R*)sm_raw;
    __shared__ R ys[kDiagThreads / 64][kMaxWidth + kPanel];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], first = a.sn_first[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];  // inverses, then packed L11
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = lane & 15, part = lane >> 4;
    const int npanel = (w + kPanel - 1) / kPanel;
    auto cst = [w](int q) { return (q * (2 * w - q - 1)) >> 1; };
    R* T = sm;
    R* I = sm + w * (w + 1) / 2;
    stage_block<R>(T, I, inv, w, tid);
    __syncthreads();
    R* yw = ys[wave];
    for (int c = wave; c < nrhs; c += kDiagThreads / 64) {
        R* __restrict__ yc = y + (int64_t)c * n;
        {
            R v[(kMaxWidth + 63) / 64];  // all of the wave's loads in flight at once
#pragma unroll
            for (int u = 0; u < (kMaxWidth + 63) / 64; ++u) {
                const int k = lane + 64 * u;
                v[u] = k < w ? yc[first + k] : R(0);
            }
#pragma unroll
            for (int u = 0; u < (kMaxWidth + 63) / 64; ++u)
                if (lane + 64 * u < w) yw[lane + 64 * u] = v[u];
        }
        __builtin_amdgcn_wave_barrier();
        for (int p = 0; p < npanel; ++p) {
            const int j0 = p * kPanel, jb = min(kPanel, w - j0);
            R o = R(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * part + q;
                o += I[p * kPanel * kPanel + j * kPanel + k] * (k < jb ? yw[j0 + k] : R(0));
            }
            o += __shfl_xor(o, 16, 64);
            o += __shfl_xor(o, 32, 64);
            R yp[kPanel];
#pragma unroll
            for (int q = 0; q < kPanel; ++q) yp[q] = lane_bcast(o, q);
            __builtin_amdgcn_wave_barrier();
            if (part == 0 && j < jb) yw[j0 + j] = o;
            for (int k = j0 + kPanel + lane; k < w; k += 64) {
                // every load of the row first, then two accumulation chains
                R tv[kPanel];
#pragma unroll
                for (int q = 0; q < kPanel; ++q) tv[q] = T[cst(j0 + q) + k];
                R acc0 = R(0), acc1 = R(0);
#pragma unroll
                for (int q = 0; q < kPanel; q += 2) {
                    acc0 += tv[q] * yp[q];
                    acc1 += tv[q + 1] * yp[q + 1];
                }
                yw[k] -= acc0 + acc1;
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int k = lane; k < w; k += 64) yc[first + k] = yw[k];
        __builtin_amdgcn_wave_barrier();
    }
}

// Below the diagonal block, forward: y[rows(i)] -= sum_k L21[i][k] y_s[k] for
// one 64-row block: the block is staged in LDS, thread (row, wave) sums every
// 4th column, the four waves meet in LDS; a row no other source of the level
// updates is updated in place (its only writer), a shared row's sum goes to
// its contribution slot for k_fwd_reduce.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_fwd_gemv(const RowBlock* __restrict__ work, KArgs a,
                                                  const R* __restrict__ arena, R* __restrict__ y,
                                                  int64_t n, int nrhs, SolveBufs<R> sb) {
    extern __shared__ double sm_raw[];
    R* Pl = (R*)sm_raw;
    __shared__ R ys[kMaxWidth][NR];
    __shared__ R red[4][NR][64];
    const RowBlock wb = work[blockIdx.x];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const int32_t* __restrict__ below = a.rows + rp + w;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i0 = wb.rb * kTile, m = min(kTile, r - i0);
    // the output row, its form and (in place) its current values are loaded
    // early so that their latency hides under the staging and the products
    const int64_t slot = rp + w + i0 + tid;
    const int32_t row = tid < m ? below[i0 + tid] : 0;
    const bool sh = tid < m && sb.shared[slot];
    stage_rows<R>(Pl, P, ld, i0, m, w, tid);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        R yold[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            yold[c] = (tid < m && !sh && c < nc) ? y[(int64_t)(c0 + c) * n + row] : R(0);
        {
            constexpr int kPer = (NR * kMaxWidth + 255) / 256;
            const float invw = 1.0f / (float)w;
            R v[kPer];
            int kk[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = tid + 256 * u;
                int c, k;
                divmod_small(e, w, invw, c, k);
                kk[u] = (e < NR * w) ? k * NR + c : -1;
                v[u] = (e < NR * w && c < nc) ? y[(int64_t)(c0 + c) * n + first + k] : R(0);
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u)
                if (kk[u] >= 0) (&ys[0][0])[kk[u]] = v[u];
        }
        __syncthreads();
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
        // kU columns per wave and step, every load of a step first (fewer with
        // several right-hand sides, whose values take kU * NR registers)
        constexpr int kU = NR == 1 ? 8 : 2;
        for (int k0 = wave; k0 < w; k0 += 4 * kU) {
            R pv[kU], yv[kU][NR];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int k = min(k0 + 4 * u, w - 1);
                const bool in = k0 + 4 * u < w;
                pv[u] = in ? Pl[k * kPs + lane] : R(0);
#pragma unroll
                for (int c = 0; c < NR; ++c) yv[u][c] = ys[k][c];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += pv[u] * yv[u][c];
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

// Below the diagonal block, backward: sum_i L21[i][k] y[rows(i)] for the
// kColGroup columns k of group g of supernode s, over the rows i of chunk h:
// thread tid takes rows tid, tid + 256, ... of the chunk (coalesced down each
// column of the column-major panel), then the 256 partial sums of every
// (column, right-hand side) meet in a fixed tree: across each wave by
// butterfly shuffles, then the four waves in order, into the chunk's partial
// sum (pb, one writer per entry, no atomics).  NR right-hand sides at a time.
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

// Diagonal block, backward: y_s = L11^{-T} (y_s - t_s), right-looking from
// the last panel:
//   y_p = inv(D_p)^T y_p;   y[k] -= L[p, k]^T y_p for every k left of the panel,
// one wave per right-hand side as in k_fwd_diag.
template <class R>
__global__ __launch_bounds__(kDiagThreads) void k_bwd_diag(const int32_t* __restrict__ level_sn,
                                                           KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ dinv, R* __restrict__ y,
                                                  const R* __restrict__ pb,
                                                  const int64_t* __restrict__ pb_off,
                                                  int64_t pb_total, int64_t n, int nrhs) {
    extern __shared__ double sm_raw[];
    R* sm = (R*)sm_raw;
    __shared__ R ys[kDiagThreads / 64][kMaxWidth + kPanel];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], first = a.sn_first[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];  // inverses, then packed L11
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = lane & 15, part = lane >> 4;
    const int npanel = (w + kPanel - 1) / kPanel;
    auto cst = [w](int q) { return (q * (2 * w - q - 1)) >> 1; };
    R* T = sm;
    R* I = sm + w * (w + 1) / 2;
    stage_block<R>(T, I, inv, w, tid);
    __syncthreads();
    R* yw = ys[wave];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const int nh = (r + kRowChunk - 1) / kRowChunk;  // row chunks with partial sums
    for (int c = wave; c < nrhs; c += kDiagThreads / 64) {
        R* __restrict__ yc = y + (int64_t)c * n;
        const R* __restrict__ pc = pb + (int64_t)c * pb_total + pb_off[s];
        {
            R v[(kMaxWidth + 63) / 64], t[(kMaxWidth + 63) / 64];
#pragma unroll
            for (int u = 0; u < (kMaxWidth + 63) / 64; ++u) {
                const int k = lane + 64 * u;
                v[u] = k < w ? yc[first + k] : R(0);
                R acc = R(0);  // the chunks' partial sums in chunk order, 4 loads at a time
                for (int h0 = 0; h0 < nh; h0 += 4) {
                    R pv[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        pv[q] = (k < w && h0 + q < nh) ? pc[(int64_t)(h0 + q) * w + k] : R(0);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (h0 + q < nh) acc += pv[q];
                }
                t[u] = acc;
            }
#pragma unroll
            for (int u = 0; u < (kMaxWidth + 63) / 64; ++u)
                if (lane + 64 * u < w) yw[lane + 64 * u] = v[u] - t[u];
        }
        __builtin_amdgcn_wave_barrier();
        for (int p = npanel - 1; p >= 0; --p) {
            const int j0 = p * kPanel, jb = min(kPanel, w - j0);
            R o = R(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * part + q;
                o += I[p * kPanel * kPanel + k * kPanel + j] * (k < jb ? yw[j0 + k] : R(0));
            }
            o += __shfl_xor(o, 16, 64);
            o += __shfl_xor(o, 32, 64);
            R yp[kPanel];
#pragma unroll
            for (int q = 0; q < kPanel; ++q) yp[q] = lane_bcast(o, q);  // zero past jb
            __builtin_amdgcn_wave_barrier();
            if (part == 0 && j < jb) yw[j0 + j] = o;
            for (int k = lane; k < j0; k += 64) {
                // row j0 + q of column k (past the last row, any entry of the
                // column: it meets yp[q] = 0)
                const int ck = cst(k) + j0;
                R tv[kPanel];
#pragma unroll
                for (int q = 0; q < kPanel; ++q) tv[q] = T[q < jb ? ck + q : ck];
                R acc0 = R(0), acc1 = R(0);
#pragma unroll
                for (int q = 0; q < kPanel; q += 2) {
                    acc0 += tv[q] * yp[q];
                    acc1 += tv[q + 1] * yp[q + 1];
                }
                yw[k] -= acc0 + acc1;
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int k = lane; k < w; k += 64) yc[first + k] = yw[k];
        __builtin_amdgcn_wave_barrier();
    }
}

// Dynamic LDS of the diagonal-block kernels: packed triangle + inverse blocks.
static size_t diag_lds(int wmax, size_t elem) {
    const int np = (wmax + kPanel - 1) / kPanel;
    return ((size_t)wmax * (wmax + 1) / 2 + (size_t)np * kPanel * kPanel) * elem;
}

int32_t configure_solve_kernels() {
    const int mx = (int)diag_lds(kMaxWidth, sizeof(double));
    const void* diag[] = {(const void*)k_fwd_diag<double>, (const void*)k_bwd_diag<double>,
                          (const void*)k_fwd_diag<float>, (const void*)k_bwd_diag<float>};
    for (const void* f : diag)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx) != hipSuccess)
            return ERR_HIP;
    const int mg = (int)(kMaxWidth * kPs * sizeof(double));
    const void* gemv[] = {(const void*)k_fwd_gemv<double, 1>, (const void*)k_fwd_gemv<float, 1>,
                          (const void*)k_fwd_gemv<double, kRhs>,
                          (const void*)k_fwd_gemv<float, kRhs>};
    for (const void* f : gemv)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mg) != hipSuccess)
            return ERR_HIP;
    return OK;
}

namespace {

// The level sweeps of one solve on the work array (y, then the contribution
// slots, then t, factor type), as enqueued on stream st.  Gather and scatter
// stay outside: they touch the caller's b and x, which change from call to
// call.
template <class R, int NR>
void enqueue_sweeps(spc_numeric* num, int32_t nrhs, R* work, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const int64_t n = S.n;
    const KArgs a = kargs(P);
    const R* arena = (const R*)num->arena;
    const R* dinv = (const R*)num->dinv;
    R* y = work;
    R* cb = y + n * nrhs;
    R* pb = cb + P->nslots * nrhs;
    const SolveBufs<R> sb{cb, P->nslots, P->slot_shared};
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        const size_t lds = diag_lds(P->level_maxw[l], sizeof(R));
        const size_t lds_rows = (size_t)P->level_maxw[l] * kPs * sizeof(R);
        if (nbig > 0)
            hipLaunchKernelGGL(k_fwd_diag<R>, dim3(nbig), dim3(kDiagThreads), lds, st,
                               P->level_sn + n0, a, arena, dinv, y, n, nrhs);
        launch_small_solve(num, a, P->level_sn + n0 + nbig, n1 - n0 - nbig, P->small_maxw[l],
                           P->small_maxm[l], y, cb, n, nrhs, true, st);
        const int64_t rb0 = P->rowblk_ptr[l], rb1 = P->rowblk_ptr[l + 1];
        if (rb1 > rb0)
            hipLaunchKernelGGL((k_fwd_gemv<R, NR>), dim3((unsigned)(rb1 - rb0)), dim3(256),
                               lds_rows, st, P->rowblk + rb0, a, arena, y, n, nrhs, sb);
        const int64_t i0 = P->red_level_ptr[l], i1 = P->red_level_ptr[l + 1];
        if (i1 > i0) {
            const int64_t work_items = (i1 - i0) * nrhs;
            hipLaunchKernelGGL(k_fwd_reduce<R>, dim3((unsigned)((work_items + 255) / 256)),
                               dim3(256), 0, st, P->red_row + i0, P->red_ptr + i0,
                               (const int32_t*)P->red_slot, i1 - i0, y, n, nrhs, sb);
        }
    }
    for (int32_t l = nl - 1; l >= 0; --l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        const int64_t g0 = P->colblk_ptr[l], g1 = P->colblk_ptr[l + 1];
        if (g1 > g0)
            hipLaunchKernelGGL((k_bwd_cols<R, NR>), dim3((unsigned)(g1 - g0)), dim3(256), 0, st,
                               P->colblk + g0, a, arena, (const R*)y, pb,
                               (const int64_t*)P->pb_off, P->pb_total, n, nrhs);
        if (nbig > 0)
            hipLaunchKernelGGL(k_bwd_diag<R>, dim3(nbig), dim3(kDiagThreads),
                               diag_lds(P->level_maxw[l], sizeof(R)), st, P->level_sn + n0, a,
                               arena, dinv, y, (const R*)pb, (const int64_t*)P->pb_off,
                               P->pb_total, n, nrhs);
        launch_small_solve(num, a, P->level_sn + n0 + nbig, n1 - n0 - nbig, P->small_maxw[l],
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

int64_t solve_work_elems(const spc_numeric* num, int32_t nrhs) {
    return solve_work_elems_per_rhs(num->sym->S) * (int64_t)nrhs;
}

int64_t solve_work_elems_per_rhs(const Symbolic& S) {
    int64_t pb = 0;
    for (int64_t s = 0; s < S.nsup; ++s)
        if (!is_small(S, s) && S.nbelow(s) > 0)
            pb += (int64_t)((S.nbelow(s) + kRowChunk - 1) / kRowChunk) * S.width(s);
    return S.n + (int64_t)S.rows.size() + pb;
}

// Solve work for nrhs right-hand sides (factor type): the vector y (n x nrhs),
// the forward contribution slots (nslots x nrhs) and the backward partial
// sums (pb_total x nrhs).
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
// process ends.  Every element a solve reads it has written first, so no
// part needs clearing between calls.
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
