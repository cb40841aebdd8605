// Supernodal triangular solves on gfx950 (the two solves of Section II-A of
// arXiv:1608.00044): y = L^{-1} P b by a forward sweep over the supernodal
// elimination tree from the leaves, then z = L^{-T} y from the root back, and
// x = P^T z.  Both sweeps go level by level; within a level every supernode
// is independent.  Each level is two launches:
//   forward:  k_fwd_diag  -- y_s = L11^{-1} y_s, one workgroup per supernode, by
//                            16-column panels using the inverted 16 x 16
//                            diagonal blocks the factorization kept;
//             k_fwd_gemv  -- y[rows below] -= L21 y_s for every 64-row block
//                            of every panel (atomic adds: sibling supernodes
//                            share ancestor rows);
//   backward: k_bwd_gemv  -- t_s += L21^T y[rows below], per 64-row block,
//                            one thread per column;
// Several right-hand sides go through every kernel in groups of eight, so the
// factor is read once per group.
//             k_bwd_diag  -- y_s = L11^{-T} (y_s - t_s), panels in reverse.
// The level sweeps are captured once per right-hand-side count into a HIP
// graph and replayed, so a solve costs three launches on the host.  The
// kernels are templates on the factor's real type R: an FP32 factor is
// solved in FP32 arithmetic with FP32 work vectors.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Stages the packed lower triangle of the w x w diagonal block (entry (i, j)
// at cst(j) + i) and the supernode's 16 x 16 inverse blocks into LDS, eight
// independent global loads per thread in flight.
template <class R>
__device__ __forceinline__ void stage_block(R* __restrict__ T, R* __restrict__ I,
                                            const R* __restrict__ L, const R* __restrict__ inv,
                                            int w, int ld, int npanel, int tid) {
    const int ww = w * w;
    for (int e0 = tid; e0 < ww; e0 += 24 * 256) {
        R v[24];
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            const int e = e0 + u * 256, i = e % w, j = e / w;
            const bool ok = e < ww && i >= j;
            v[u] = L[ok ? i + (int64_t)j * ld : 0];
        }
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            const int e = e0 + u * 256, i = e % w, j = e / w;
            if (e < ww && i >= j) T[((j * (2 * w - j - 1)) >> 1) + i] = v[u];
        }
    }
    // the inverses are stored compactly (the last panel as jb x jb); LDS
    // holds every panel as a zero-padded 16 x 16 block
    const int ni = npanel * kPanel * kPanel;
    for (int e0 = tid; e0 < ni; e0 += 8 * 256) {
        R v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256, p = e >> 8, r = (e >> 4) & 15, c = e & 15;
            const int jbp = min(kPanel, w - kPanel * p);
            const bool in = e < ni && r < jbp && c < jbp;
            const R t = inv[in ? p * kPanel * kPanel + r * jbp + c : 0];
            v[u] = in ? t : R(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + u * 256 < ni) I[e0 + u * 256] = v[u];
    }
}

// Right-hand sides are processed NR at a time (NR = 1, or kRhs for several):
// every kernel reads its part of L once per group of NR columns and keeps NR
// partial sums per thread.
constexpr int kRhs = 8;

// Forward, diagonal block: the block L11 (packed lower triangle) and its
// 16 x 16 diagonal-block inverses are staged in LDS by the workgroup; then for
// each 16-column panel p and each of the NR right-hand sides
//   t = y_p - L[p, <p] y_{<p}   (thread (j, part) sums every 16th column k,
//                                the 16 parts meet in LDS),
//   y_p = inv(D_p) t            (16 threads per right-hand side).
template <class R, int NR>
__global__ __launch_bounds__(256) void k_fwd_diag(const int32_t* __restrict__ level_sn, KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ dinv, R* __restrict__ y,
                                                  int64_t n, int nrhs) {
    extern __shared__ double sm_raw[];
    R* sm = (R*)sm_raw;
    __shared__ R ys[NR][kMaxWidth + kPanel];
    __shared__ R red[NR][16][17];
    __shared__ R tt[NR][16];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const R* __restrict__ L = arena + a.sn_off[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];
    const int tid = threadIdx.x, j = tid & 15, part = tid >> 4;
    const int jj = tid & 15, cc = tid >> 4;  // reduction stage: column cc, entry jj
    const int npanel = (w + kPanel - 1) / kPanel;
    auto cst = [w](int q) { return (q * (2 * w - q - 1)) >> 1; };
    R* T = sm;
    R* I = sm + w * (w + 1) / 2;
    stage_block<R>(T, I, L, inv, w, ld, npanel, tid);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < NR * w; e += 256) {
            const int c = e / w, k = e - c * w;
            ys[c][k] = c < nc ? y[(int64_t)(c0 + c) * n + first + k] : R(0);
        }
        __syncthreads();
        for (int p = 0; p < npanel; ++p) {
            const int j0 = p * kPanel, jb = min(kPanel, w - j0);
            R acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = R(0);
            if (j < jb)
                for (int k = part; k < j0; k += 16) {
                    const R l = T[cst(k) + j0 + j];
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += l * ys[c][k];
                }
#pragma unroll
            for (int c = 0; c < NR; ++c) red[c][part][j] = acc[c];
            __syncthreads();
            if (cc < NR) {
                R tot = R(0);
#pragma unroll
                for (int q = 0; q < 16; ++q) tot += red[cc][q][jj];
                tt[cc][jj] = (jj < jb) ? ys[cc][j0 + jj] - tot : R(0);
            }
            __syncthreads();
            if (cc < NR) {
                R out = R(0);
#pragma unroll
                for (int k = 0; k < kPanel; ++k)
                    out += I[p * kPanel * kPanel + jj * kPanel + k] * tt[cc][k];
                if (jj < jb) ys[cc][j0 + jj] = out;
            }
            __syncthreads();
        }
        for (int e = tid; e < nc * w; e += 256) {
            const int c = e / w, k = e - c * w;
            y[(int64_t)(c0 + c) * n + first + k] = ys[c][k];
        }
        __syncthreads();
    }
}

// Forward, below the diagonal block: y[rows(i)] -= sum_k L21[i][k] y_s[k];
// thread (row, wave) walks every 4th column; the four waves combine through
// LDS.  The block of L21 is read once per NR right-hand sides.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_fwd_gemv(const RowBlock* __restrict__ work, KArgs a,
                                                  const R* __restrict__ arena, R* __restrict__ y,
                                                  int64_t n, int nrhs) {
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
    const int i = wb.rb * kTile + lane;
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < NR * w; e += 256) {
            const int c = e / w, k = e - c * w;
            ys[k][c] = c < nc ? y[(int64_t)(c0 + c) * n + first + k] : R(0);
        }
        __syncthreads();
        R acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = R(0);
        if (i < r) {
#pragma unroll 4
            for (int k = wave; k < w; k += 4) {
                const R pv = P[i + (int64_t)k * ld];
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += pv * ys[k][c];
            }
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) red[wave][c][lane] = acc[c];
        __syncthreads();
        if (tid < 64 && i < r) {
            const int32_t row = below[i];
            for (int c = 0; c < nc; ++c)
                unsafeAtomicAdd(y + (int64_t)(c0 + c) * n + row,
                                -((red[0][c][lane] + red[1][c][lane]) +
                                  (red[2][c][lane] + red[3][c][lane])));
        }
        __syncthreads();
    }
}

// Backward, below the diagonal block: t_s[k] += sum_i L21[i][k] y[rows(i)]
// over one 64-row block: the gathered entries go to LDS, then thread k walks
// column k of the block (its own contiguous 64 entries) once per NR
// right-hand sides and adds one partial sum per column and right-hand side.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_gemv(const RowBlock* __restrict__ work, KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ y, R* __restrict__ tacc,
                                                  int64_t n, int nrhs) {
    __shared__ R xr[kTile][NR];
    const RowBlock wb = work[blockIdx.x];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ P = arena + a.sn_off[s] + w;
    const int32_t* __restrict__ below = a.rows + rp + w;
    const int tid = threadIdx.x;
    const int i0 = wb.rb * kTile, m = min(kTile, r - i0);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < NR * kTile; e += 256) {
            const int c = e / kTile, ii = e - c * kTile;
            xr[ii][c] = (c < nc && ii < m) ? y[(int64_t)(c0 + c) * n + below[i0 + ii]] : R(0);
        }
        __syncthreads();
        for (int k = tid; k < w; k += 256) {
            const R* __restrict__ col = P + i0 + (int64_t)k * ld;
            if (NR == 1) {
                R acc0 = R(0), acc1 = R(0), acc2 = R(0), acc3 = R(0);
                int i = 0;
                for (; i + 4 <= m; i += 4) {
                    acc0 += col[i] * xr[i][0];
                    acc1 += col[i + 1] * xr[i + 1][0];
                    acc2 += col[i + 2] * xr[i + 2][0];
                    acc3 += col[i + 3] * xr[i + 3][0];
                }
                for (; i < m; ++i) acc0 += col[i] * xr[i][0];
                unsafeAtomicAdd(tacc + (int64_t)c0 * n + first + k, (acc0 + acc1) + (acc2 + acc3));
            } else {
                R acc[NR];
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] = R(0);
                for (int i = 0; i < m; ++i) {
                    const R pv = col[i];
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += pv * xr[i][c];
                }
                for (int c = 0; c < nc; ++c)
                    unsafeAtomicAdd(tacc + (int64_t)(c0 + c) * n + first + k, acc[c]);
            }
        }
        __syncthreads();
    }
}

// Backward, diagonal block: y_s = L11^{-T} (y_s - t_s), panels from the last:
//   u = v_p - L[>p, p]^T y_{>p},   y_p = inv(D_p)^T u,
// with L11 and the inverses staged in LDS and the dot products split over
// the workgroup as in k_fwd_diag, NR right-hand sides at a time.
template <class R, int NR>
__global__ __launch_bounds__(256) void k_bwd_diag(const int32_t* __restrict__ level_sn, KArgs a,
                                                  const R* __restrict__ arena,
                                                  const R* __restrict__ dinv, R* __restrict__ y,
                                                  const R* __restrict__ tacc, int64_t n,
                                                  int nrhs) {
    extern __shared__ double sm_raw[];
    R* sm = (R*)sm_raw;
    __shared__ R ys[NR][kMaxWidth + kPanel];
    __shared__ R red[NR][16][17];
    __shared__ R tt[NR][16];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const R* __restrict__ L = arena + a.sn_off[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];
    const int tid = threadIdx.x, j = tid & 15, part = tid >> 4;
    const int jj = tid & 15, cc = tid >> 4;
    const int npanel = (w + kPanel - 1) / kPanel;
    auto cst = [w](int q) { return (q * (2 * w - q - 1)) >> 1; };
    R* T = sm;
    R* I = sm + w * (w + 1) / 2;
    stage_block<R>(T, I, L, inv, w, ld, npanel, tid);
    for (int c0 = 0; c0 < nrhs; c0 += NR) {
        const int nc = min(NR, nrhs - c0);
        for (int e = tid; e < NR * w; e += 256) {
            const int c = e / w, k = e - c * w;
            const int64_t at = (int64_t)(c0 + c) * n + first + k;
            ys[c][k] = c < nc ? y[at] - tacc[at] : R(0);
        }
        __syncthreads();
        for (int p = npanel - 1; p >= 0; --p) {
            const int j0 = p * kPanel, jb = min(kPanel, w - j0);
            R acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = R(0);
            if (j < jb)
                for (int k = j0 + kPanel + part; k < w; k += 16) {
                    const R l = T[cst(j0 + j) + k];
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += l * ys[c][k];
                }
#pragma unroll
            for (int c = 0; c < NR; ++c) red[c][part][j] = acc[c];
            __syncthreads();
            if (cc < NR) {
                R tot = R(0);
#pragma unroll
                for (int q = 0; q < 16; ++q) tot += red[cc][q][jj];
                tt[cc][jj] = (jj < jb) ? ys[cc][j0 + jj] - tot : R(0);
            }
            __syncthreads();
            if (cc < NR) {
                R out = R(0);
#pragma unroll
                for (int k = 0; k < kPanel; ++k)
                    out += I[p * kPanel * kPanel + k * kPanel + jj] * tt[cc][k];
                if (jj < jb) ys[cc][j0 + jj] = out;
            }
            __syncthreads();
        }
        for (int e = tid; e < nc * w; e += 256) {
            const int c = e / w, k = e - c * w;
            y[(int64_t)(c0 + c) * n + first + k] = ys[c][k];
        }
        __syncthreads();
    }
}

// Dynamic LDS of the diagonal-block kernels: packed triangle + inverse blocks.
static size_t diag_lds(int wmax, size_t elem) {
    const int np = (wmax + kPanel - 1) / kPanel;
    return ((size_t)wmax * (wmax + 1) / 2 + (size_t)np * kPanel * kPanel) * elem;
}

int32_t configure_solve_kernels() {
    const int mx = (int)diag_lds(kMaxWidth, sizeof(double));
    const void* fns[] = {(const void*)k_fwd_diag<double, 1>, (const void*)k_bwd_diag<double, 1>,
                         (const void*)k_fwd_diag<float, 1>, (const void*)k_bwd_diag<float, 1>,
                         (const void*)k_fwd_diag<double, kRhs>,
                         (const void*)k_bwd_diag<double, kRhs>,
                         (const void*)k_fwd_diag<float, kRhs>,
                         (const void*)k_bwd_diag<float, kRhs>};
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, mx) != hipSuccess)
            return ERR_HIP;
    return OK;
}

namespace {

// The level sweeps of one solve on the internal work vectors (y, t), as
// enqueued on stream st.  Gather and scatter stay outside: they touch the
// caller's b and x, which change from call to call.
template <class R, int NR>
void enqueue_sweeps(spc_numeric* num, int32_t nrhs, R* y, R* tacc, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const int64_t n = S.n;
    const KArgs a = kargs(P);
    const R* arena = (const R*)num->arena;
    const R* dinv = (const R*)num->dinv;
    const int64_t total = n * nrhs;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
    hipLaunchKernelGGL(k_zero<R>, dim3(g), dim3(256), 0, st, tacc, total);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        const size_t lds = diag_lds(P->level_maxw[l], sizeof(R));
        if (nbig > 0)
            hipLaunchKernelGGL((k_fwd_diag<R, NR>), dim3(nbig), dim3(256), lds, st,
                               P->level_sn + n0, a, arena, dinv, y, n, nrhs);
        launch_small_solve(num, a, P->level_sn + n0 + nbig, n1 - n0 - nbig, y, n, nrhs, true, st);
        const int64_t rb0 = P->rowblk_ptr[l], rb1 = P->rowblk_ptr[l + 1];
        if (rb1 > rb0)
            hipLaunchKernelGGL((k_fwd_gemv<R, NR>), dim3((unsigned)(rb1 - rb0)), dim3(256), 0, st,
                               P->rowblk + rb0, a, arena, y, n, nrhs);
    }
    for (int32_t l = nl - 1; l >= 0; --l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1], nbig = P->level_nbig[l];
        const int64_t rb0 = P->rowblk_ptr[l], rb1 = P->rowblk_ptr[l + 1];
        if (rb1 > rb0)
            hipLaunchKernelGGL((k_bwd_gemv<R, NR>), dim3((unsigned)(rb1 - rb0)), dim3(256), 0, st,
                               P->rowblk + rb0, a, arena, (const R*)y, tacc, n, nrhs);
        if (nbig > 0)
            hipLaunchKernelGGL((k_bwd_diag<R, NR>), dim3(nbig), dim3(256),
                               diag_lds(P->level_maxw[l], sizeof(R)), st, P->level_sn + n0, a,
                               arena, dinv, y, (const R*)tacc, n, nrhs);
        launch_small_solve(num, a, P->level_sn + n0 + nbig, n1 - n0 - nbig, y, n, nrhs, false,
                           st);
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

// Work vectors y and t (n x nrhs each, factor type) for nrhs right-hand sides.
int32_t ensure_solve_work(spc_numeric* num, int32_t nrhs) {
    const int64_t n = num->sym->S.n;
    if (num->work_cols >= nrhs) return OK;
    if (num->work) {
        HIP_TRY(hipDeviceSynchronize());
        drop_solve_graphs(num);
        HIP_TRY(hipFree(num->work));
        num->work = nullptr;
        num->work_cols = 0;
    }
    if (hipMalloc(&num->work, 2 * elem_size(num) * (size_t)n * nrhs) != hipSuccess)
        return ERR_OOM;
    num->work_cols = nrhs;
    return OK;
}

// Replays (capturing on first use) the sweeps for nrhs columns on stream st.
int32_t run_sweeps(spc_numeric* num, int32_t nrhs, hipStream_t st) {
    const int64_t n = num->sym->S.n;
    spc_numeric::SolveGraph* sg = nullptr;
    for (auto& e : num->solve_graphs)
        if (e.nrhs == nrhs) sg = &e;
    if (!sg) {
        if (!num->capture) HIP_TRY(hipStreamCreateWithFlags(&num->capture, hipStreamNonBlocking));
        spc_numeric::SolveGraph e;
        e.nrhs = nrhs;
        HIP_TRY(hipStreamBeginCapture(num->capture, hipStreamCaptureModeThreadLocal));
        const size_t half = (size_t)n * nrhs;
        if (num->prec == 1) {
            float* y = (float*)num->work;
            if (nrhs == 1) enqueue_sweeps<float, 1>(num, nrhs, y, y + half, num->capture);
            else enqueue_sweeps<float, kRhs>(num, nrhs, y, y + half, num->capture);
        } else {
            double* y = (double*)num->work;
            if (nrhs == 1) enqueue_sweeps<double, 1>(num, nrhs, y, y + half, num->capture);
            else enqueue_sweeps<double, kRhs>(num, nrhs, y, y + half, num->capture);
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

int32_t run_solve(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                  int64_t ldx, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const int64_t n = S.n;
    if (n == 0 || nrhs == 0) return OK;
    int32_t r = ensure_solve_work(num, nrhs);
    if (r != OK) return r;
    const int64_t total = n * nrhs;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
    if (num->prec == 1)
        hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(256), 0, st, b, ldb, P->perm,
                           (float*)num->work, n, nrhs);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(g), dim3(256), 0, st, b, ldb, P->perm,
                           (double*)num->work, n, nrhs);
    // the sweeps replay from a graph captured once per right-hand-side count
    r = run_sweeps(num, nrhs, st);
    if (r != OK) return r;
    if (num->prec == 1)
        hipLaunchKernelGGL(k_scatter<float>, dim3(g), dim3(256), 0, st, (const float*)num->work,
                           P->perm, x, ldx, n, nrhs);
    else
        hipLaunchKernelGGL(k_scatter<double>, dim3(g), dim3(256), 0, st, (const double*)num->work,
                           P->perm, x, ldx, n, nrhs);
    HIP_TRY(hipGetLastError());
    return OK;
}

}  // namespace spc
