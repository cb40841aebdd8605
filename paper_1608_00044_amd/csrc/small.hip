// Small supernodes (width <= 16, at most 64 rows below the diagonal block),
// one group of 16, 32 or 64 lanes each (several per wavefront when every
// small supernode of the level has at most 16 or 32 rows), with no workgroup
// barrier: the F task (diagonal
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

// Factorization, inverse and scatter of one small supernode by G lanes of a
// wave (gl: the lane's place among them; G = 64 takes any small supernode,
// G = 16 or 32 only those with at most G rows, several per wave).  The block
// sits in LDS with column stride LDG rows.  Storage type S, compute type C.
// kCheck (the FP32 pass): no status is recorded; a pivot at most kSmallTau
// times its starting diagonal entry makes the function return true before
// anything is written to global memory, so that the caller can run it again
// in FP64.
// Deterministic order (det.scratch set): a column whose pair is exclusive
// (no other source of the level updates its target) is added to the target
// directly; the other columns go to the supernode's block in the level's
// scratch (column c, row i >= c of the r x r lower triangle at
// c (2r - c + 1) / 2 + i - c), which the apply kernel adds in source order.
template <class S>
struct SmallDet {
    const uint8_t* excl;
    const int64_t* scr_off;
    S* scratch;
};

template <class S, class C, bool kCheck, int G, int LDG>
__device__ bool small_body(int s, const KArgs& a, S* __restrict__ arena, S* __restrict__ dinv,
                           int32_t* __restrict__ status, C* __restrict__ blk,
                           int64_t* __restrict__ colbase, int64_t* __restrict__ relbase,
                           int gl, const SmallDet<S>& det) {
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    const int64_t rp = a.rowptr[s];
    const int m = (int)(a.rowptr[s + 1] - rp), r = m - w;
    S* __restrict__ base = arena + a.sn_off[s];
    // the block into LDS, eight columns at a time with every load in flight
    for (int j0 = 0; j0 < w; j0 += 8) {
        constexpr int kChunks = (LDG + G - 1) / G;
        C v[8][kChunks];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
#pragma unroll
            for (int q = 0; q < kChunks; ++q) {
                const int i = gl + G * q, j = j0 + jj;
                v[jj][q] = (j < w && i < m && i >= j) ? (C)base[i + (int64_t)j * ld] : C(0);
            }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
#pragma unroll
            for (int q = 0; q < kChunks; ++q) {
                const int i = gl + G * q, j = j0 + jj;
                if (j < w && i < m) blk[j * LDG + i] = v[jj][q];
            }
    }
    // targets of the rows below (their columns in the update)
    if (gl < r) {
        const int64_t at = rp + w + gl;
        const int p = a.rowpair[at];
        const int t = a.pair_tgt[p];
        const int64_t cb = a.sn_off[t] + (int64_t)(a.rows[at] - a.sn_first[t]) * a.sn_ld[t];
        // deterministic order: a shared target's column is marked by ~cb (< 0)
        colbase[gl] = (det.scratch && !det.excl[p]) ? ~cb : cb;
        relbase[gl] = a.pair_rel[p] - a.pair_seg[p];
    }
    __builtin_amdgcn_wave_barrier();
    bool bad = false;
    for (int k = 0; k < w; ++k) {
        const C d = blk[k * LDG + k];
        if (kCheck) {
            bad |= !(d > (C)kSmallTau * (C)base[k + (int64_t)k * ld]);
        } else if (!(d > C(0)) && gl == 0) {
            atomicMin(status, first + k + 1);
        }
        C rs, l;
        rsqrt_sqrt_s(d, rs, l);
        __builtin_amdgcn_wave_barrier();
        for (int i = k + 1 + gl; i < m; i += G) blk[k * LDG + i] *= rs;
        if (gl == 0) blk[k * LDG + k] = l;
        __builtin_amdgcn_wave_barrier();
        for (int i = k + 1 + gl; i < m; i += G) {
            const C lik = blk[k * LDG + i];
            const int jend = min(w, i + 1);
            for (int j = k + 1; j < jend; ++j) blk[j * LDG + i] -= lik * blk[k * LDG + j];
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (kCheck && bad) return true;
    // inverse of L11, column c by lane c, row major into the compact w x w block
    if (gl < w) {
        S* __restrict__ inv = dinv + a.inv_off[s];
        C x[kSmallW];
#pragma unroll
        for (int q = 0; q < kSmallW; ++q) {
            if (q < w) {
                C acc = q == gl ? C(1) : C(0);
#pragma unroll
                for (int k = 0; k < q; ++k) acc -= blk[k * LDG + q] * x[k];
                x[q] = acc / blk[q * LDG + q];
                inv[q * w + gl] = (S)x[q];
            } else {
                x[q] = C(0);
            }
        }
    }
    for (int j = 0; j < w; ++j)
        for (int i = j + gl; i < m; i += G) base[i + (int64_t)j * ld] = (S)blk[j * LDG + i];
    // update + scatter: lane i takes row i below the block and every column
    // c <= i, in groups of kGroup columns whose relative indices are all
    // loaded before the group's products and atomics
    if (gl < r) {
        constexpr int kGroup = 8;
        C li[kSmallW];
#pragma unroll
        for (int k = 0; k < kSmallW; ++k) li[k] = k < w ? blk[k * LDG + w + gl] : C(0);
        for (int c0 = 0; c0 <= gl; c0 += kGroup) {
            int32_t rv[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int c = c0 + u;
                rv[u] = c <= gl ? a.rel[relbase[c] + gl] : 0;
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int c = c0 + u;
                if (c <= gl) {
                    C v = C(0);
#pragma unroll
                    for (int k = 0; k < kSmallW; ++k)
                        if (k < w) v += li[k] * blk[k * LDG + w + c];
                    const int64_t cb = colbase[c];
                    if (!det.scratch) {
                        unsafeAtomicAdd(arena + cb + rv[u], (S)(-v));
                    } else if (cb >= 0) {  // the only source of the level for this target
                        S* q = arena + cb + rv[u];
                        *q = *q + (S)(-v);
                    } else {
                        const int64_t at = (int64_t)c * (2 * r - c + 1) / 2 + (gl - c);
                        det.scratch[det.scr_off[s] + at] = (S)(-v);
                    }
                }
            }
        }
    }
    return false;
}

template <int G, int LDG>
__device__ __forceinline__ void small_factor(int s, const KArgs& a, double* arena, double* dinv,
                                             int32_t* status, int32_t*, double* lds,
                                             int64_t* cb, int64_t* rb, int gl,
                                             const SmallDet<double>& det) {
    small_body<double, double, false, G, LDG>(s, a, arena, dinv, status, lds, cb, rb, gl, det);
}
template <int G, int LDG>
__device__ __forceinline__ void small_factor(int s, const KArgs& a, float* arena, float* dinv,
                                             int32_t* status, int32_t* fallbacks, double* lds,
                                             int64_t* cb, int64_t* rb, int gl,
                                             const SmallDet<float>& det) {
    if (small_body<float, float, true, G, LDG>(s, a, arena, dinv, status, (float*)lds, cb, rb,
                                               gl, det)) {
        __builtin_amdgcn_wave_barrier();
        small_body<float, double, false, G, LDG>(s, a, arena, dinv, status, lds, cb, rb, gl, det);
        if (gl == 0) atomicAdd(fallbacks, 1);
    }
}

// G lanes per small supernode of list[0 .. count), 64 / G supernodes per
// wave.  A group past the end returns at once: the kernel has no workgroup
// barrier.  LDS (dynamic) holds per group the block's first maxw columns
// (stride LDG rows, FP64) and maxr column lookups, sized to the widest and
// tallest small supernode of the level, so that levels of tiny supernodes
// keep many waves per CU.
template <class R, int G, int LDG>
__global__ __launch_bounds__(256) void k_small(const int32_t* __restrict__ list, int count,
                                               KArgs a, R* __restrict__ arena,
                                               R* __restrict__ dinv, int32_t* __restrict__ status,
                                               int maxw, int maxr, SmallDet<R> det) {
    extern __shared__ double sm_small[];
    constexpr int kGroups = 4 * (64 / G);  // groups per workgroup
    const int lane = threadIdx.x & 63;
    const int grp = threadIdx.x / G, gl = lane % G;
    double* blk = sm_small + (size_t)grp * LDG * maxw;
    int64_t* cb = (int64_t*)(sm_small + (size_t)kGroups * LDG * maxw) + (size_t)grp * 2 * maxr;
    const int idx = blockIdx.x * kGroups + grp;
    if (idx >= count) return;
    small_factor<G, LDG>(list[idx], a, arena, dinv, status, status + 1, blk, cb, cb + maxr, gl,
                         det);
}

// Deterministic order, apply pass: one wave per item (a shared target t and
// a block of 64 of its rows, rho0 .. rho0 + 63).  Lane L owns target row
// rho0 + L: for every entry of the item, sources in increasing order, it
// adds the scratch values of the source row landing on its target row, one
// column after another; so each target entry is updated by one lane, in
// program order (plain read-modify-writes, no atomics).
template <class R>
__global__ __launch_bounds__(256) void k_apply(const int32_t* __restrict__ app_t,
                                               const int32_t* __restrict__ app_rb,
                                               const int64_t* __restrict__ app_p0,
                                               const AppEnt* __restrict__ ent,
                                               const int32_t* __restrict__ pair_src,
                                               const int32_t* __restrict__ pair_end,
                                               const int64_t* __restrict__ scr_off,
                                               const R* __restrict__ scratch, KArgs a,
                                               R* __restrict__ arena, int64_t count) {
    __shared__ int own_s[4][kTile];
    __shared__ int64_t cb_s[4][kMaxWidth];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + wave;
    if (k >= count) return;  // no workgroup barrier below
    int* own = own_s[wave];
    int64_t* cbs = cb_s[wave];
    const int t = app_t[k], rho0 = app_rb[k] * kTile;
    const int64_t toff = a.sn_off[t] + rho0 + lane;
    const int tfirst = a.sn_first[t], tld = a.sn_ld[t];
    for (int64_t q = app_p0[k]; q < app_p0[k + 1]; ++q) {
        const AppEnt en = ent[q];
        const int p = en.p;
        const int s = pair_src[p];
        const int w = a.sn_w[s];
        const int64_t rp = a.rowptr[s];
        const int r = (int)(a.rowptr[s + 1] - rp) - w;
        const int b = a.pair_seg[p], e = pair_end[p];
        const int64_t relb = a.pair_rel[p] - b;
        const R* __restrict__ blk = scratch + scr_off[s];
        own[lane] = -1;
        __builtin_amdgcn_wave_barrier();
        for (int i = en.ilo + lane; i < en.ihi; i += 64) own[a.rel[relb + i] - rho0] = i;
        for (int c = b + lane; c < e; c += 64)
            cbs[c - b] = (int64_t)(a.rows[rp + w + c] - tfirst) * tld;
        __builtin_amdgcn_wave_barrier();
        const int i = own[lane];
        if (i >= 0) {
            const int c1 = min(e, i + 1);
            for (int c0 = b; c0 < c1; c0 += 8) {  // eight columns' loads in flight
                R v[8], old[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = c0 + u;
                    v[u] = c < c1 ? blk[(int64_t)c * (2 * r - c + 1) / 2 + (i - c)] : R(0);
                    old[u] = c < c1 ? arena[toff + cbs[c - b]] : R(0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (c0 + u < c1) arena[toff + cbs[c0 + u - b]] = old[u] + v[u];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int G, int LDG>
size_t small_lds(int maxw, int maxr) {
    constexpr int kGroups = 4 * (64 / G);
    return (size_t)kGroups * LDG * maxw * sizeof(double) +
           (size_t)kGroups * 2 * maxr * sizeof(int64_t);
}

// Sum over the G lanes of a lane group (G a power of two, groups aligned).
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Forward solve of one small supernode per G lanes, every right-hand side
// (WB: a bound on the level's small widths, so registers follow the level):
//   y_s = inv(L11) y_s;  y[rows below] -= L21 y_s, in place for a row that no
//   other source of the level updates, else into the row's contribution slot
//   (reduced after the level in source order).  recs: the level's small
//   supernodes, one record each.
template <class R, int WB, int G>
__global__ __launch_bounds__(256) void k_small_fwd(const SmallRec* __restrict__ recs, int count,
                                                   KArgs a, const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, int64_t n, int nrhs,
                                                   SolveBufs<R> sb) {
    const int lane = threadIdx.x & 63, gl = lane % G;
    const int idx = blockIdx.x * (256 / G) + (int)threadIdx.x / G;
    if (idx >= count) return;
    const SmallRec rec = recs[idx];
    const int w = rec.w, ld = rec.ld, first = rec.first, r = rec.r;
    const int64_t rp = rec.rp;
    const R* __restrict__ L = arena + rec.off;
    const R* __restrict__ inv = dinv + rec.inv;
    R li[WB], iv[WB];
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        li[k] = (gl < r && k < w) ? L[w + gl + (int64_t)k * ld] : R(0);
        iv[k] = (gl < w && k < w) ? inv[gl * w + k] : R(0);
    }
    const int32_t row = gl < r ? a.rows[rp + w + gl] : 0;
    const bool shared = gl < r && sb.shared[rp + w + gl];
    for (int c = 0; c < nrhs; ++c) {
        R* __restrict__ yc = y + (int64_t)c * n;
        R* __restrict__ cbc = sb.cb + (int64_t)c * sb.nslots;
        const R b = gl < w ? yc[first + gl] : R(0);
        // a row below that no other source of the level updates has this
        // supernode as its one writer here, and lies outside its columns:
        // its old value can be loaded with b, before y_s is stored
        const R yold = (gl < r && !shared) ? yc[row] : R(0);
        R ys = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) ys += iv[k] * __shfl(b, k, G);
        if (gl < w) yc[first + gl] = ys;
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) acc += li[k] * __shfl(ys, k, G);
        if (gl < r) {
            if (shared) cbc[rp + w + gl] = acc;
            else yc[row] = yold - acc;
        }
    }
}

// Backward solve of one small supernode per G lanes, every right-hand side
// (WB as for the forward solve):
//   t = L21^T y[rows below] (group sums);  y_s = inv(L11)^T (y_s - t)
template <class R, int WB, int G>
__global__ __launch_bounds__(256) void k_small_bwd(const SmallRec* __restrict__ recs, int count,
                                                   KArgs a, const R* __restrict__ arena,
                                                   const R* __restrict__ dinv,
                                                   R* __restrict__ y, int64_t n, int nrhs) {
    const int lane = threadIdx.x & 63, gl = lane % G;
    const int idx = blockIdx.x * (256 / G) + (int)threadIdx.x / G;
    if (idx >= count) return;
    const SmallRec rec = recs[idx];
    const int w = rec.w, ld = rec.ld, first = rec.first, r = rec.r;
    const int64_t rp = rec.rp;
    const R* __restrict__ L = arena + rec.off;
    const R* __restrict__ inv = dinv + rec.inv;
    R li[WB], ivt[WB];
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        li[k] = (gl < r && k < w) ? L[w + gl + (int64_t)k * ld] : R(0);
        ivt[k] = (gl < w && k < w) ? inv[k * w + gl] : R(0);
    }
    const int32_t row = gl < r ? a.rows[rp + w + gl] : 0;
    for (int c = 0; c < nrhs; ++c) {
        R* __restrict__ yc = y + (int64_t)c * n;
        const R yb = gl < r ? yc[row] : R(0);
        R u = gl < w ? yc[first + gl] : R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) {
            if (k < w) {
                const R t = group_sum<G>(li[k] * yb);
                if (gl == k) u -= t;
            }
        }
        R out = R(0);
#pragma unroll
        for (int k = 0; k < WB; ++k) out += ivt[k] * __shfl(u, k, G);
        if (gl < w) yc[first + gl] = out;
    }
}

}  // namespace

void launch_small_factor(spc_numeric* num, const KArgs& a, const int32_t* list, int count,
                         int maxw, int maxr, int maxm, hipStream_t st) {
    if (count <= 0) return;
    maxw = std::max(1, std::min(maxw, kSmallW));
    maxr = std::max(1, std::min(maxr, kSmallR));
    const DevicePlan* P = num->plan;
    auto go = [&](auto kern, size_t lds, int per_block, auto* arena) {
        using T = std::remove_pointer_t<decltype(arena)>;
        const unsigned g = (unsigned)std::max(1, (count + per_block - 1) / per_block);
        SmallDet<T> det{nullptr, nullptr, nullptr};
        if (num->det) det = SmallDet<T>{P->pair_excl, P->scr_off, (T*)num->det_scratch};
        hipLaunchKernelGGL(kern, dim3(g), dim3(256), lds, st, list, count, a, arena,
                           (T*)num->dinv, num->status_dev, maxw, maxr, det);
    };
    // several supernodes per wave when every one of the level has few rows
    if (num->prec == 1) {
        float* ar = (float*)num->arena;
        if (maxm <= 16) go(k_small<float, 16, 16>, small_lds<16, 16>(maxw, maxr), 16, ar);
        else if (maxm <= 32) go(k_small<float, 32, 32>, small_lds<32, 32>(maxw, maxr), 8, ar);
        else go(k_small<float, 64, kSmallLd>, small_lds<64, kSmallLd>(maxw, maxr), 4, ar);
    } else {
        double* ar = (double*)num->arena;
        if (maxm <= 16) go(k_small<double, 16, 16>, small_lds<16, 16>(maxw, maxr), 16, ar);
        else if (maxm <= 32) go(k_small<double, 32, 32>, small_lds<32, 32>(maxw, maxr), 8, ar);
        else go(k_small<double, 64, kSmallLd>, small_lds<64, kSmallLd>(maxw, maxr), 4, ar);
    }
}

void launch_small_apply(spc_numeric* num, int64_t i0, int64_t i1, hipStream_t st) {
    const DevicePlan* P = num->plan;
    const KArgs a = kargs(P);
    const int64_t count = i1 - i0;
    if (count <= 0) return;
    const dim3 g((unsigned)((count + 3) / 4)), b(256);
    if (num->prec == 1)
        hipLaunchKernelGGL(k_apply<float>, g, b, 0, st, P->app_t + i0, P->app_rb + i0,
                           P->app_p0 + i0, (const AppEnt*)P->app_ent, (const int32_t*)P->pair_src,
                           (const int32_t*)P->pair_end, (const int64_t*)P->scr_off,
                           (const float*)num->det_scratch, a, (float*)num->arena, count);
    else
        hipLaunchKernelGGL(k_apply<double>, g, b, 0, st, P->app_t + i0, P->app_rb + i0,
                           P->app_p0 + i0, (const AppEnt*)P->app_ent, (const int32_t*)P->pair_src,
                           (const int32_t*)P->pair_end, (const int64_t*)P->scr_off,
                           (const double*)num->det_scratch, a, (double*)num->arena, count);
}

void launch_small_solve(spc_numeric* num, const KArgs& a, const SmallRec* recs, int count,
                        int maxw, int maxm, void* y, void* cb, int64_t n, int nrhs, bool forward,
                        hipStream_t st) {
    if (count <= 0) return;
    const DevicePlan* P = num->plan;
    auto go = [&](auto kf, auto kb, int per_block, auto* yt) {
        using T = std::remove_pointer_t<decltype(yt)>;
        const dim3 g((unsigned)std::max(1, (count + per_block - 1) / per_block)), b(256);
        const SolveBufs<T> sb{(T*)cb, P->nslots, P->slot_shared};
        if (forward)
            hipLaunchKernelGGL(kf, g, b, 0, st, recs, count, a, (const T*)num->arena,
                               (const T*)num->dinv, yt, n, nrhs, sb);
        else
            hipLaunchKernelGGL(kb, g, b, 0, st, recs, count, a, (const T*)num->arena,
                               (const T*)num->dinv, yt, n, nrhs);
    };
    // the width bound sizes the registers; lanes per supernode follow the
    // level's tallest small supernode
    auto pick = [&](auto* yt) {
        using T = std::remove_pointer_t<decltype(yt)>;
        if (maxm <= 16) {
            if (maxw <= 4) go(k_small_fwd<T, 4, 16>, k_small_bwd<T, 4, 16>, 16, yt);
            else if (maxw <= 8) go(k_small_fwd<T, 8, 16>, k_small_bwd<T, 8, 16>, 16, yt);
            else go(k_small_fwd<T, kSmallW, 16>, k_small_bwd<T, kSmallW, 16>, 16, yt);
        } else if (maxm <= 32) {
            if (maxw <= 4) go(k_small_fwd<T, 4, 32>, k_small_bwd<T, 4, 32>, 8, yt);
            else if (maxw <= 8) go(k_small_fwd<T, 8, 32>, k_small_bwd<T, 8, 32>, 8, yt);
            else go(k_small_fwd<T, kSmallW, 32>, k_small_bwd<T, kSmallW, 32>, 8, yt);
        } else {
            if (maxw <= 4) go(k_small_fwd<T, 4, 64>, k_small_bwd<T, 4, 64>, 4, yt);
            else if (maxw <= 8) go(k_small_fwd<T, 8, 64>, k_small_bwd<T, 8, 64>, 4, yt);
            else go(k_small_fwd<T, kSmallW, 64>, k_small_bwd<T, kSmallW, 64>, 4, yt);
        }
    };
    if (num->prec == 1) pick((float*)y);
    else pick((double*)y);
}

}  // namespace spc
