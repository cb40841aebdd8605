// Supernodal triangular solves on gfx950 (the two solves of Section II-A of
// arXiv:1608.00044): y = L^{-1} P b by a forward sweep over the supernodal
// elimination tree from the leaves, then z = L^{-T} y from the root back, and
// x = P^T z.  Both sweeps go level by level; within a level every supernode
// is independent.  The forward sweep subtracts L21 y_s from the rows below
// each supernode with atomic adds (sibling supernodes share ancestor rows);
// the backward sweep only reads ancestor entries, which earlier levels of the
// reverse sweep have finished.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.hpp"

namespace spc {

#define HIP_TRY(x)                               \
    do {                                         \
        if ((x) != hipSuccess) return ERR_HIP;   \
    } while (0)

constexpr int kChunk = 2048;

__global__ void k_gather(const double* __restrict__ b, int64_t ldb,
                         const int32_t* __restrict__ perm, double* __restrict__ y, int64_t n,
                         int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        y[e] = b[perm[i] + c * ldb];
    }
}

__global__ void k_scatter(const double* __restrict__ y, const int32_t* __restrict__ perm,
                          double* __restrict__ x, int64_t ldx, int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        x[perm[i] + c * ldx] = y[e];
    }
}

// Forward: y_s = L11^{-1} y_s (column-oriented substitution in LDS), then
// y[rows below] -= L21 y_s.
__global__ __launch_bounds__(256) void k_fwd(const int32_t* __restrict__ level_sn, KArgs a,
                                             const double* __restrict__ arena,
                                             double* __restrict__ y, int64_t n, int nrhs) {
    __shared__ double ys[kMaxWidth];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const double* __restrict__ L = arena + a.sn_off[s];
    const int32_t* __restrict__ below = a.rows + rp + w;
    const int tid = threadIdx.x;
    for (int c = 0; c < nrhs; ++c) {
        double* __restrict__ yc = y + (int64_t)c * n;
        for (int k = tid; k < w; k += blockDim.x) ys[k] = yc[first + k];
        __syncthreads();
        for (int k = 0; k < w; ++k) {
            if (tid == 0) ys[k] /= L[k + (int64_t)k * ld];
            __syncthreads();
            const double yk = ys[k];
            for (int j = k + 1 + tid; j < w; j += blockDim.x) ys[j] -= L[j + (int64_t)k * ld] * yk;
            __syncthreads();
        }
        for (int k = tid; k < w; k += blockDim.x) yc[first + k] = ys[k];
        for (int i = tid; i < r; i += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < w; ++k) acc += L[w + i + (int64_t)k * ld] * ys[k];
            unsafeAtomicAdd(yc + below[i], -acc);
        }
        __syncthreads();
    }
}

// Backward: y_s -= L21^T y[rows below] (each wave reduces columns k = wave,
// wave + 4, ...; the gathered entries are staged in LDS by chunks), then
// y_s = L11^{-T} y_s by back substitution.
__global__ __launch_bounds__(256) void k_bwd(const int32_t* __restrict__ level_sn, KArgs a,
                                             const double* __restrict__ arena,
                                             double* __restrict__ y, int64_t n, int nrhs) {
    __shared__ double ys[kMaxWidth];
    __shared__ double xb[kChunk];
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const double* __restrict__ L = arena + a.sn_off[s];
    const int32_t* __restrict__ below = a.rows + rp + w;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int c = 0; c < nrhs; ++c) {
        double* __restrict__ yc = y + (int64_t)c * n;
        for (int k = tid; k < w; k += blockDim.x) ys[k] = yc[first + k];
        for (int i0 = 0; i0 < r; i0 += kChunk) {
            const int m = min(kChunk, r - i0);
            __syncthreads();
            for (int i = tid; i < m; i += blockDim.x) xb[i] = yc[below[i0 + i]];
            __syncthreads();
            for (int k = wave; k < w; k += 4) {
                const double* __restrict__ col = L + w + i0 + (int64_t)k * ld;
                double part = 0.0;
                for (int i = lane; i < m; i += 64) part += col[i] * xb[i];
                for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
                if (lane == 0) ys[k] -= part;
            }
        }
        __syncthreads();
        for (int k = w - 1; k >= 0; --k) {
            if (tid == 0) ys[k] /= L[k + (int64_t)k * ld];
            __syncthreads();
            const double yk = ys[k];
            for (int j = tid; j < k; j += blockDim.x) ys[j] -= L[k + (int64_t)j * ld] * yk;
            __syncthreads();
        }
        for (int k = tid; k < w; k += blockDim.x) yc[first + k] = ys[k];
        __syncthreads();
    }
}

int32_t run_solve(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                  int64_t ldx, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const int64_t n = S.n;
    if (n == 0 || nrhs == 0) return OK;
    if (num->work_cols < nrhs) {
        if (num->work) {
            HIP_TRY(hipStreamSynchronize(num->stream));
            HIP_TRY(hipFree(num->work));
            num->work = nullptr;
            num->work_cols = 0;
        }
        if (hipMalloc(&num->work, sizeof(double) * (size_t)n * nrhs) != hipSuccess) return ERR_OOM;
        num->work_cols = nrhs;
    }
    KArgs a;
    a.sn_first = P->sn_first;
    a.sn_w = P->sn_w;
    a.sn_ld = P->sn_ld;
    a.sn_off = P->sn_off;
    a.rowptr = P->rowptr;
    a.rows = P->rows;
    a.rowpair = P->rowpair;
    a.pair_tgt = P->pair_tgt;
    a.pair_seg = P->pair_seg;
    a.pair_rel = P->pair_rel;
    a.rel = P->rel;
    const int64_t total = n * nrhs;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, st, b, ldb, P->perm, num->work, n, nrhs);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1];
        hipLaunchKernelGGL(k_fwd, dim3(n1 - n0), dim3(256), 0, st, P->level_sn + n0, a,
                           num->arena, num->work, n, nrhs);
    }
    for (int32_t l = nl - 1; l >= 0; --l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1];
        hipLaunchKernelGGL(k_bwd, dim3(n1 - n0), dim3(256), 0, st, P->level_sn + n0, a,
                           num->arena, num->work, n, nrhs);
    }
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, st, num->work, P->perm, x, ldx, n, nrhs);
    HIP_TRY(hipGetLastError());
    return OK;
}

}  // namespace spc
