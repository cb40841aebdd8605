// Small supernodes (width <= 16, at most 64 rows below the diagonal block)
// one wavefront each, with no workgroup barrier: the F task (diagonal
// factorization and panel solve) and the U + A tasks (update and
// relative-index scatter) of Section III-A fused in one pass over the
// supernode, and both solves of Section II-A fused per supernode.  Nested
// dissection leaves most supernodes this small (for a batch of 2D problems,
// nearly all of them); one workgroup per supernode and per task, as the
// large-supernode kernels use, would spend its time on launch and barriers.
//
// Factorization of supernode s (w columns, m = w + r rows), staged in LDS:
//   for k < w:  L(k, k) = sqrt(A(k, k)); L(i, k) = A(i, k) / L(k, k) for i > k;
//               A(i, j) -= L(i, k) L(j, k) for k < j <= min(i, w - 1)
// (the column form of the diagonal factorization and of L21 = A21 L11^-T
// together), then the inverse of L11 for the solves, then for every pair of
// rows i >= c below the block, (L21 L21^T)(i, c) is subtracted from the
// target that owns row c, at the row given by the relative index of i.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "runtime.hpp"

namespace spc {

namespace {

constexpr int kSmallLd = kSmallW + kSmallR;  // LDS column stride of the staged block
constexpr float kSmallTau = 1e-3f;           // FP32 pivot ratio that calls for FP64

__device__ __forceinline__ void rsqrt_sqrt_s(double d, double& rs, double& sq) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * (1.5 - 0.5 * d * y * y);
    y = y * (1.5 - 0.5 * d * y * y);
    rs = y;
    sq = d * y;
}
__device__ __forceinline__ void rsqrt_sqrt_s(float d, float& rs, float& sq) {
    float y = __builtin_amdgcn_rsqf(d);
    y = y * (1.5f - 0.5f * d * y * y);
    rs = y;
    sq = d * y;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Factorization, inverse and scatter of one small supernode by one wave.
// Storage type S, compute type C.  kCheck (the FP32 pass): no status is
// recorded; a pivot at most kSmallTau times its starting diagonal entry
// makes the function return true before anything is written to global
// memory, so that the caller can run it again in FP64.
template <class S, class C, bool kCheck>
__device__ bool small_body(int s, const KArgs& a, S* __restrict__ arena, S* __restrict__ dinv,
                           int32_t* __restrict__ status, C* __restrict__ blk,
                           int64_t* __restrict__ colbase, int64_t* __restrict__ relbase,
                           int lane) {
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int m = (int)(a.rowptr[s + 1] - rp), r = m - w;
    S* __restrict__ base = arena + a.sn_off[s];
    // the block into LDS, eight columns at a time with every load in flight
    for (int j0 = 0; j0 < w; j0 += 8) {
        constexpr int kChunks = (kSmallLd + 63) / 64;
        C v[8][kChunks];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
#pragma unroll
            for (int q = 0; q < kChunks; ++q) {
                const int i = lane + 64 * q, j = j0 + jj;
                v[jj][q] = (j < w && i < m && i >= j) ? (C)base[i + (int64_t)j * ld] : C(0);
            }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
#pragma unroll
            for (int q = 0; q < kChunks; ++q) {
                const int i = lane + 64 * q, j = j0 + jj;
                if (j < w && i < m) blk[j * kSmallLd + i] = v[jj][q];
            }
    }
    // targets of the rows below (their columns in the update)
    if (lane < r) {
        const int64_t at = rp + w + lane;
        const int p = a.rowpair[at];
        const int t = a.pair_tgt[p];
        colbase[lane] = a.sn_off[t] + (int64_t)(a.rows[at] - a.sn_first[t]) * a.sn_ld[t];
        relbase[lane] = a.pair_rel[p] - a.pair_seg[p];
    }
    __builtin_amdgcn_wave_barrier();
    bool bad = false;
    for (int k = 0; k < w; ++k) {
        const C d = blk[k * kSmallLd + k];
        if (kCheck) {
            bad |= !(d > (C)kSmallTau * (C)base[k + (int64_t)k * ld]);
        } else if (!(d > C(0)) && lane == 0) {
            atomicMin(status, first + k + 1);
        }
        C rs, l;
        rsqrt_sqrt_s(d, rs, l);
        __builtin_amdgcn_wave_barrier();
        for (int i = k + 1 + lane; i < m; i += 64) blk[k * kSmallLd + i] *= rs;
        if (lane == 0) blk[k * kSmallLd + k] = l;
        __builtin_amdgcn_wave_barrier();
        for (int i = k + 1 + lane; i < m; i += 64) {
            const C lik = blk[k * kSmallLd + i];
            const int jend = min(w, i + 1);
            for (int j = k + 1; j < jend; ++j) blk[j * kSmallLd + i] -= lik * blk[k * kSmallLd + j];
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (kCheck && bad) return true;
    // inverse of L11, column c by lane c, row major into the compact w x w block
    if (lane < w) {
        S* __restrict__ inv = dinv + a.inv_off[s];
        C x[kSmallW];
#pragma unroll
        for (int q = 0; q < kSmallW; ++q) {
            if (q < w) {
                C acc = q == lane ? C(1) : C(0);
#pragma unroll
                for (int k = 0; k < q; ++k) acc -= blk[k * kSmallLd + q] * x[k];
                x[q] = acc / blk[q * kSmallLd + q];
                inv[q * w + lane] = (S)x[q];
            } else {
                x[q] = C(0);
            }
        }
    }
    for (int j = 0; j < w; ++j)
        for (int i = j + lane; i < m; i += 64) base[i + (int64_t)j * ld] = (S)blk[j * kSmallLd + i];
    // update + scatter: lane i takes row i below the block and every column
    // c <= i, in groups of kGroup columns whose relative indices are all
    // loaded before the group's products and atomics
    if (lane < r) {
        constexpr int kGroup = 8;
        C li[kSmallW];
#pragma unroll
        for (int k = 0; k < kSmallW; ++k) li[k] = k < w ? blk[k * kSmallLd + w + lane] : C(0);
        for (int c0 = 0; c0 <= lane; c0 += kGroup) {
            int32_t rv[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int c = c0 + u;
                rv[u] = c <= lane ? a.rel[relbase[c] + lane] : 0;
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int c = c0 + u;
                if (c <= lane) {
                    C v = C(0);
#pragma unroll
                    for (int k = 0; k < kSmallW; ++k)
                        if (k < w) v += li[k] * blk[k * kSmallLd + w + c];
                    unsafeAtomicAdd(arena + colbase[c] + rv[u], (S)(-v));
                }
            }
        }
    }
    return false;
}

__device__ __forceinline__ void small_factor(int s, const KArgs& a, double* arena, double* dinv,
                                             int32_t* status, int32_t*, double* lds,
                                             int64_t* cb, int64_t* rb, int lane) {
    small_body<double, double, false>(s, a, arena, dinv, status, lds, cb, rb, lane);
}
__device__ __forceinline__ void small_factor(int s, const KArgs& a, float* arena, float* dinv,
                                             int32_t* status, int32_t* fallbacks, double* lds,
                                             int64_t* cb, int64_t* rb, int lane) {
    if (small_body<float, float, true>(s, a, arena, dinv, status, (float*)lds, cb, rb, lane)) {
        __builtin_amdgcn_wave_barrier();
        small_body<float, double, false>(s, a, arena, dinv, status, lds, cb, rb, lane);
        if (lane == 0) atomicAdd(fallbacks, 1);
    }
}

// One wave per small supernode of list[0 .. count).  A wave past the end
// returns at once: the kernel has no workgroup barrier.  LDS (dynamic) holds
// per wave the block's first maxw columns (stride kSmallLd, FP64) and maxr
// column lookups: sized to the widest and tallest small supernode of the
// level, so that levels of tiny supernodes keep many waves per CU.
template <class R>
__global__ __launch_bounds__(256) void k_small(const int32_t* __restrict__ list, int count,
                                               KArgs a, R* __restrict__ arena,
                                               R* __restrict__ dinv, int32_t* __restrict__ status,
                                               int maxw, int maxr) {
    extern __shared__ double sm_small[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* blk = sm_small + (size_t)wave * kSmallLd * maxw;
    int64_t* cb = (int64_t*)(sm_small + (size_t)4 * kSmallLd * maxw) + (size_t)wave * 2 * maxr;
    const int idx = blockIdx.x * 4 + wave;
    if (idx >= count) return;
    small_factor(list[idx], a, arena, dinv, status, status + 1, blk, cb, cb + maxr, lane);
}

size_t small_lds(int maxw, int maxr) {
    return (size_t)4 * kSmallLd * maxw * sizeof(double) + (size_t)4 * 2 * maxr * sizeof(int64_t);
}

// Forward solve of one small supernode per wave, every right-hand side
// (WB: a bound on the level's small widths, so registers follow the level):
//   y_s = inv(L11) y_s;  y[rows below] -= L21 y_s  (atomic: siblings share ancestors)
template <class R, int WB>
__global__ __launch_bounds__(256) void k_small_fwd(const int32_t* __restrict__ list, int count,
                                                   KArgs a, const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, int64_t n, int nrhs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wave;
    if (idx >= count) return;
    const int s = list[idx];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ L = arena + a.sn_off[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];
    R li[WB], iv[WB];
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        li[k] = (lane < r && k < w) ? L[w + lane + (int64_t)k * ld] : R(0);
        iv[k] = (lane < w && k < w) ? inv[lane * w + k] : R(0);
    }
    const int32_t row = lane < r ? a.rows[rp + w + lane] : 0;
    for (int c = 0; c < nrhs; ++c) {
        R* __restrict__ yc = y + (int64_t)c * n;
        const R b = lane < w ? yc[first + lane] : R(0);
        R ys = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) ys += iv[k] * __shfl(b, k, 64);
        if (lane < w) yc[first + lane] = ys;
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) acc += li[k] * __shfl(ys, k, 64);
        if (lane < r) unsafeAtomicAdd(yc + row, -acc);
    }
}

// Backward solve of one small supernode per wave, every right-hand side
// (WB as for the forward solve):
//   t = L21^T y[rows below] (wave sums);  y_s = inv(L11)^T (y_s - t)
template <class R, int WB>
__global__ __launch_bounds__(256) void k_small_bwd(const int32_t* __restrict__ list, int count,
                                                   KArgs a, const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, int64_t n, int nrhs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wave;
    if (idx >= count) return;
    const int s = list[idx];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const R* __restrict__ L = arena + a.sn_off[s];
    const R* __restrict__ inv = dinv + a.inv_off[s];
    R li[WB], ivt[WB];
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        li[k] = (lane < r && k < w) ? L[w + lane + (int64_t)k * ld] : R(0);
        ivt[k] = (lane < w && k < w) ? inv[k * w + lane] : R(0);
    }
    const int32_t row = lane < r ? a.rows[rp + w + lane] : 0;
    for (int c = 0; c < nrhs; ++c) {
        R* __restrict__ yc = y + (int64_t)c * n;
        const R yb = lane < r ? yc[row] : R(0);
        R u = lane < w ? yc[first + lane] : R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) {
            if (k < w) {
                const R t = wave_sum(li[k] * yb);
                if (lane == k) u -= t;
            }
        }
        R out = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) out += ivt[k] * __shfl(u, k, 64);
        if (lane < w) yc[first + lane] = out;
    }
}

unsigned waves_grid(int count) { return (unsigned)std::max(1, (count + 3) / 4); }

}  // namespace

void launch_small_factor(spc_numeric* num, const KArgs& a, const int32_t* list, int count,
                         int maxw, int maxr, hipStream_t st) {
    if (count <= 0) return;
    maxw = std::max(1, std::min(maxw, kSmallW));
    maxr = std::max(1, std::min(maxr, kSmallR));
    const size_t lds = small_lds(maxw, maxr);
    if (num->prec == 1)
        hipLaunchKernelGGL(k_small<float>, dim3(waves_grid(count)), dim3(256), lds, st, list,
                           count, a, (float*)num->arena, (float*)num->dinv, num->status_dev, maxw,
                           maxr);
    else
        hipLaunchKernelGGL(k_small<double>, dim3(waves_grid(count)), dim3(256), lds, st, list,
                           count, a, (double*)num->arena, (double*)num->dinv, num->status_dev,
                           maxw, maxr);
}

void launch_small_solve(spc_numeric* num, const KArgs& a, const int32_t* list, int count,
                        int maxw, void* y, int64_t n, int nrhs, bool forward, hipStream_t st) {
    if (count <= 0) return;
    const dim3 g(waves_grid(count)), b(256);
    auto go = [&](auto kf, auto kb, auto* yt) {
        using T = std::remove_pointer_t<decltype(yt)>;
        if (forward)
            hipLaunchKernelGGL(kf, g, b, 0, st, list, count, a, (const T*)num->arena,
                               (const T*)num->dinv, yt, n, nrhs);
        else
            hipLaunchKernelGGL(kb, g, b, 0, st, list, count, a, (const T*)num->arena,
                               (const T*)num->dinv, yt, n, nrhs);
    };
    if (num->prec == 1) {
        float* yf = (float*)y;
        if (maxw <= 4) go(k_small_fwd<float, 4>, k_small_bwd<float, 4>, yf);
        else if (maxw <= 8) go(k_small_fwd<float, 8>, k_small_bwd<float, 8>, yf);
        else go(k_small_fwd<float, kSmallW>, k_small_bwd<float, kSmallW>, yf);
    } else {
        double* yd = (double*)y;
        if (maxw <= 4) go(k_small_fwd<double, 4>, k_small_bwd<double, 4>, yd);
        else if (maxw <= 8) go(k_small_fwd<double, 8>, k_small_bwd<double, 8>, yd);
        else go(k_small_fwd<double, kSmallW>, k_small_bwd<double, kSmallW>, yd);
    }
}

}  // namespace spc
