// Numeric supernodal Cholesky on gfx950: plan upload, value load, and the
// per-level task kernels.
//
// Tasks (Section III-A of arXiv:1608.00044), per supernode s of width w with
// r rows below its diagonal block, stored as a column-major (w + r) x w block:
//   F  (k_potrf, k_trsm):  L11 = chol(A11) in LDS, then L21 = A21 L11^{-T}
//                          row by row;
//   U  (k_update):         the lower triangle of L21 L21^T in 64 x 64 tiles on
//                          FP64 matrix cores (v_mfma_f64_16x16x4);
//   A  (k_update epilogue): each tile entry is subtracted from the target
//                          supernode that owns its column, at the row given by
//                          the precomputed relative index (an atomic add, since
//                          sibling supernodes of one level may hit the same target).
// Dependencies (Section II-C) are met by running the supernodal elimination
// tree level by level: every supernode of level l only receives updates from
// descendants, which all sit on lower levels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "runtime.hpp"

namespace spc {

typedef double v4d __attribute__((ext_vector_type(4)));

#define HIP_TRY(x)                               \
    do {                                         \
        if ((x) != hipSuccess) return ERR_HIP;   \
    } while (0)

// ---------------------------------------------------------------------------
// plan upload
// ---------------------------------------------------------------------------

namespace {

struct Layout {
    size_t total = 0;
    template <class T>
    size_t add(size_t count) {
        size_t at = (total + 255) & ~size_t(255);
        total = at + count * sizeof(T);
        return at;
    }
};

struct PlanOffsets {
    size_t sn_first, sn_w, sn_ld, sn_off, rowptr, rows, rowpair, slot, perm, pair_tgt, pair_seg,
        pair_rel, rel, level_sn, rowblk, tiles;
    size_t total;
};

void count_work(const Symbolic& S, std::vector<int64_t>& rb_ptr, std::vector<int64_t>& tl_ptr) {
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    rb_ptr.assign((size_t)nl + 1, 0);
    tl_ptr.assign((size_t)nl + 1, 0);
    for (int32_t l = 0; l < nl; ++l) {
        int64_t rb = 0, tl = 0;
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            const int64_t r = S.nbelow(S.level_sn[q]);
            const int64_t nb = (r + kTile - 1) / kTile;
            rb += nb;
            tl += nb * (nb + 1) / 2;
        }
        rb_ptr[l + 1] = rb_ptr[l] + rb;
        tl_ptr[l + 1] = tl_ptr[l] + tl;
    }
}

PlanOffsets plan_layout(const Symbolic& S, const std::vector<int64_t>& rb_ptr,
                        const std::vector<int64_t>& tl_ptr) {
    Layout L;
    PlanOffsets o;
    const size_t ns = (size_t)S.nsup;
    o.sn_first = L.add<int32_t>(ns);
    o.sn_w = L.add<int32_t>(ns);
    o.sn_ld = L.add<int32_t>(ns);
    o.sn_off = L.add<int64_t>(ns);
    o.rowptr = L.add<int64_t>(ns + 1);
    o.rows = L.add<int32_t>(S.rows.size());
    o.rowpair = L.add<int32_t>(S.rows.size());
    o.slot = L.add<int64_t>(S.slot.size());
    o.perm = L.add<int32_t>(S.perm.size());
    o.pair_tgt = L.add<int32_t>(S.pairs.size());
    o.pair_seg = L.add<int32_t>(S.pairs.size());
    o.pair_rel = L.add<int64_t>(S.pairs.size());
    o.rel = L.add<int32_t>(S.rel.size());
    o.level_sn = L.add<int32_t>(S.level_sn.size());
    o.rowblk = L.add<RowBlock>((size_t)rb_ptr.back());
    o.tiles = L.add<UpdTile>((size_t)tl_ptr.back());
    o.total = L.total;
    return o;
}

}  // namespace

size_t plan_bytes(const Symbolic& S) {
    std::vector<int64_t> a, b;
    count_work(S, a, b);
    return plan_layout(S, a, b).total;
}

int32_t get_plan(spc_symbolic* sym, DevicePlan** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(sym->mu);
    for (DevicePlan* p : sym->plans)
        if (p->device == dev) { *out = p; return OK; }
    const Symbolic& S = sym->S;
    if (S.max_r >= 32767 * kTile) return ERR_ARG;  // tile coordinates are 16-bit
    DevicePlan* P = new DevicePlan();
    P->device = dev;
    count_work(S, P->rowblk_ptr, P->tile_ptr);
    PlanOffsets o = plan_layout(S, P->rowblk_ptr, P->tile_ptr);
    std::vector<char> h(o.total ? o.total : 1, 0);
    auto put = [&](size_t at, const void* src, size_t bytes) {
        if (bytes) std::memcpy(h.data() + at, src, bytes);
    };
    const size_t ns = (size_t)S.nsup;
    std::vector<int32_t> w(ns), first(ns);
    for (size_t s = 0; s < ns; ++s) { first[s] = S.sn_ptr[s]; w[s] = S.width((int64_t)s); }
    put(o.sn_first, first.data(), ns * 4);
    put(o.sn_w, w.data(), ns * 4);
    put(o.sn_ld, S.ld.data(), ns * 4);
    put(o.sn_off, S.off.data(), ns * 8);
    put(o.rowptr, S.rowptr.data(), (ns + 1) * 8);
    put(o.rows, S.rows.data(), S.rows.size() * 4);
    {
        std::vector<int32_t> rp(S.rows.size(), -1);
        for (size_t p = 0; p < S.pairs.size(); ++p) {
            const Pair& pr = S.pairs[p];
            const int64_t base = S.rowptr[pr.src] + S.width(pr.src);
            for (int32_t i = pr.seg_begin; i < pr.seg_end; ++i) rp[base + i] = (int32_t)p;
        }
        put(o.rowpair, rp.data(), rp.size() * 4);
    }
    put(o.slot, S.slot.data(), S.slot.size() * 8);
    put(o.perm, S.perm.data(), S.perm.size() * 4);
    {
        const size_t np = S.pairs.size();
        std::vector<int32_t> tg(np), sg(np);
        std::vector<int64_t> ro(np);
        for (size_t p = 0; p < np; ++p) {
            tg[p] = S.pairs[p].tgt;
            sg[p] = S.pairs[p].seg_begin;
            ro[p] = S.pairs[p].rel_off;
        }
        put(o.pair_tgt, tg.data(), np * 4);
        put(o.pair_seg, sg.data(), np * 4);
        put(o.pair_rel, ro.data(), np * 8);
    }
    put(o.rel, S.rel.data(), S.rel.size() * 4);
    put(o.level_sn, S.level_sn.data(), S.level_sn.size() * 4);
    {
        const int32_t nl = (int32_t)S.level_ptr.size() - 1;
        std::vector<RowBlock> rb((size_t)P->rowblk_ptr.back());
        std::vector<UpdTile> tl((size_t)P->tile_ptr.back());
        P->level_maxw.assign((size_t)nl, 0);
        size_t a = 0, b = 0;
        for (int32_t l = 0; l < nl; ++l) {
            for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
                const int32_t s = S.level_sn[q];
                P->level_maxw[l] = std::max(P->level_maxw[l], S.width(s));
                const int32_t nb = (S.nbelow(s) + kTile - 1) / kTile;  // < 32768 (checked)
                for (int32_t i = 0; i < nb; ++i) rb[a++] = RowBlock{s, i};
                for (int32_t i = 0; i < nb; ++i)
                    for (int32_t j = 0; j <= i; ++j) tl[b++] = UpdTile{s, (int16_t)i, (int16_t)j};
            }
        }
        put(o.rowblk, rb.data(), rb.size() * sizeof(RowBlock));
        put(o.tiles, tl.data(), tl.size() * sizeof(UpdTile));
    }
    void* d = nullptr;
    if (hipMalloc(&d, o.total ? o.total : 256) != hipSuccess) { delete P; return ERR_OOM; }
    if (hipMemcpy(d, h.data(), o.total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        delete P;
        return ERR_HIP;
    }
    char* base = (char*)d;
    P->block = d;
    P->bytes = o.total;
    P->sn_first = (int32_t*)(base + o.sn_first);
    P->sn_w = (int32_t*)(base + o.sn_w);
    P->sn_ld = (int32_t*)(base + o.sn_ld);
    P->sn_off = (int64_t*)(base + o.sn_off);
    P->rowptr = (int64_t*)(base + o.rowptr);
    P->rows = (int32_t*)(base + o.rows);
    P->rowpair = (int32_t*)(base + o.rowpair);
    P->slot = (int64_t*)(base + o.slot);
    P->perm = (int32_t*)(base + o.perm);
    P->pair_tgt = (int32_t*)(base + o.pair_tgt);
    P->pair_seg = (int32_t*)(base + o.pair_seg);
    P->pair_rel = (int64_t*)(base + o.pair_rel);
    P->rel = (int32_t*)(base + o.rel);
    P->level_sn = (int32_t*)(base + o.level_sn);
    P->rowblk = (RowBlock*)(base + o.rowblk);
    P->tiles = (UpdTile*)(base + o.tiles);
    sym->plans.push_back(P);
    *out = P;
    return OK;
}

void free_plan(DevicePlan* p) {
    if (!p) return;
    if (p->block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        (void)hipFree(p->block);
        (void)hipSetDevice(cur);
    }
    delete p;
}

static KArgs kargs(const DevicePlan* P) {
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
    return a;
}

// ---------------------------------------------------------------------------
// value load
// ---------------------------------------------------------------------------

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
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
__global__ void k_load(const double* __restrict__ values, const int64_t* __restrict__ slot,
                       double* __restrict__ arena, int64_t nnz) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        arena[slot[k]] = values[k];
}

// ---------------------------------------------------------------------------
// F: diagonal block factorization (POTRF)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int tri_idx(int i, int j, int w) {
    // packed lower triangle, column major: column j starts after sum_{c<j} (w - c)
    return j * w - (j * (j - 1)) / 2 + (i - j);
}

// One workgroup per supernode of the level.  The w x w diagonal block is held
// as a packed lower triangle in LDS and factored right-looking: pivot, scale
// the column, rank-1 update of the trailing triangle (Algorithm 1 on the
// block).  A pivot that is not positive records its global column with
// atomicMin on *status (the smallest failing column wins).
__global__ __launch_bounds__(256) void k_potrf(const int32_t* __restrict__ level_sn, KArgs a,
                                               double* __restrict__ arena,
                                               int32_t* __restrict__ status) {
    extern __shared__ double T[];
    __shared__ double piv;
    const int s = level_sn[blockIdx.x];
    const int w = a.sn_w[s], ld = a.sn_ld[s], first = a.sn_first[s];
    double* __restrict__ base = arena + a.sn_off[s];
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += blockDim.x) {
        const int i = e % w, j = e / w;
        if (i >= j) T[tri_idx(i, j, w)] = base[i + (int64_t)j * ld];
    }
    __syncthreads();
    for (int k = 0; k < w; ++k) {
        if (tid == 0) {
            double d = T[tri_idx(k, k, w)];
            if (!(d > 0.0)) atomicMin(status, first + k + 1);
            double p = sqrt(d);
            T[tri_idx(k, k, w)] = p;
            piv = p;
        }
        __syncthreads();
        const double inv = 1.0 / piv;
        for (int i = k + 1 + tid; i < w; i += blockDim.x) T[tri_idx(i, k, w)] *= inv;
        __syncthreads();
        const int m = w - k - 1;
        for (int e = tid; e < m * m; e += blockDim.x) {
            const int ii = e % m, jj = e / m;
            if (ii >= jj) {
                const int i = k + 1 + ii, j = k + 1 + jj;
                T[tri_idx(i, j, w)] -= T[tri_idx(i, k, w)] * T[tri_idx(j, k, w)];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < w * w; e += blockDim.x) {
        const int i = e % w, j = e / w;
        if (i >= j) base[i + (int64_t)j * ld] = T[tri_idx(i, j, w)];
    }
}

// ---------------------------------------------------------------------------
// F: panel solve (TRSM) L21 = A21 L11^{-T}
// ---------------------------------------------------------------------------

// One 64-thread workgroup per 64-row block of a panel; each lane solves one
// row x L11^T = a by forward substitution, with its row staged in LDS.
__global__ __launch_bounds__(64) void k_trsm(const RowBlock* __restrict__ work, KArgs a,
                                             double* __restrict__ arena) {
    extern __shared__ double X[];  // [w][64]
    const RowBlock wb = work[blockIdx.x];
    const int s = wb.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int r = (int)(a.rowptr[s + 1] - a.rowptr[s]) - w;
    const double* __restrict__ L = arena + a.sn_off[s];
    double* __restrict__ P = arena + a.sn_off[s] + w;
    const int t = threadIdx.x;
    const int row = wb.rb * kTile + t;
    const bool ok = row < r;
    for (int k = 0; k < w; ++k) X[k * kTile + t] = ok ? P[row + (int64_t)k * ld] : 0.0;
    for (int j = 0; j < w; ++j) {
        double acc = X[j * kTile + t];
        const double* __restrict__ Lj = L + j;
        for (int k = 0; k < j; ++k) acc -= X[k * kTile + t] * Lj[(int64_t)k * ld];
        X[j * kTile + t] = acc / Lj[(int64_t)j * ld];
    }
    if (ok)
        for (int k = 0; k < w; ++k) P[row + (int64_t)k * ld] = X[k * kTile + t];
}

// ---------------------------------------------------------------------------
// U + A: update tiles on FP64 MFMA with relative-index scatter
// ---------------------------------------------------------------------------

constexpr int kCtPad = kTile + 1;

// 256 threads = 4 waves in a 2 x 2 grid, each wave a 32 x 32 quarter of the
// 64 x 64 tile as 2 x 2 blocks of v_mfma_f64_16x16x4.  Operand lanes: lane l
// holds element (row l % 16, k l / 16) of each 16 x 4 slice; the A and B
// operands are both rows of the same column-major panel.  The result goes to
// LDS, then every entry (i, c), i >= c, is subtracted from the target that
// owns the column's row: target block + rel[i] + (row(c) - first(t)) * ld(t).
__global__ __launch_bounds__(256) void k_update(const UpdTile* __restrict__ tiles, KArgs a,
                                                double* __restrict__ arena) {
    __shared__ double Ct[kTile * kCtPad];  // column-major: Ct[c * kCtPad + i]
    __shared__ int64_t colbase[kTile];
    __shared__ int64_t relbase[kTile];
    const UpdTile tile = tiles[blockIdx.x];
    const int s = tile.s;
    const int w = a.sn_w[s], ld = a.sn_ld[s];
    const int64_t rp = a.rowptr[s];
    const int r = (int)(a.rowptr[s + 1] - rp) - w;
    const double* __restrict__ P = arena + a.sn_off[s] + w;
    const int i0 = tile.bi * kTile, c0 = tile.bj * kTile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const bool diag = tile.bi == tile.bj;
    const bool skip = diag && wr < wc;  // strictly upper quarter of a diagonal tile

    v4d acc[2][2];
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n) acc[m][n] = v4d{0.0, 0.0, 0.0, 0.0};
    if (!skip) {
        const int ra0 = i0 + wr * 32 + lr, ra1 = ra0 + 16;
        const int rb0 = c0 + wc * 32 + lr, rb1 = rb0 + 16;
        const bool va0 = ra0 < r, va1 = ra1 < r, vb0 = rb0 < r, vb1 = rb1 < r;
        for (int k0 = 0; k0 < w; k0 += 4) {
            const int k = k0 + lk;
            const bool vk = k < w;
            const double* __restrict__ col = P + (int64_t)k * ld;
            const double a0 = (vk && va0) ? col[ra0] : 0.0;
            const double a1 = (vk && va1) ? col[ra1] : 0.0;
            const double b0 = (vk && vb0) ? col[rb0] : 0.0;
            const double b1 = (vk && vb1) ? col[rb1] : 0.0;
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    // accumulator layout (v_mfma_f64_16x16x4): register q of lane l holds D[4q + l/16][l%16]
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n)
            for (int q = 0; q < 4; ++q) {
                const int i = wr * 32 + m * 16 + 4 * q + lk;
                const int c = wc * 32 + n * 16 + lr;
                Ct[c * kCtPad + i] = acc[m][n][q];
            }
    if (tid < kTile) {
        const int gc = c0 + tid;
        if (gc < r) {
            const int64_t at = rp + w + gc;
            const int p = a.rowpair[at];
            const int t = a.pair_tgt[p];
            colbase[tid] = a.sn_off[t] + (int64_t)(a.rows[at] - a.sn_first[t]) * a.sn_ld[t];
            relbase[tid] = a.pair_rel[p] - a.pair_seg[p];
        }
    }
    __syncthreads();
    for (int e = tid; e < kTile * kTile; e += blockDim.x) {
        const int i = e & (kTile - 1), c = e >> 6;
        const int gi = i0 + i, gc = c0 + c;
        if (gi < r && gc < r && gi >= gc) {
            const int64_t dst = colbase[c] + a.rel[relbase[c] + gi];
            unsafeAtomicAdd(arena + dst, -Ct[c * kCtPad + i]);
        }
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

int32_t run_factor(spc_numeric* num, const double* values, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    const DevicePlan* P = num->plan;
    const KArgs a = kargs(P);
    num->stream = st;
    num->factored = false;
    num->marks.clear();
    num->next_event = 0;
    int ev = mark_begin(num, st);
    if (S.arena > 0)
        hipLaunchKernelGGL(k_fill, dim3(grid_for(S.arena, 256)), dim3(256), 0, st, num->arena,
                           S.arena, 0.0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, num->status_dev, (int64_t)1,
                       (int32_t)INT32_MAX);
    if (S.nnz_a > 0)
        hipLaunchKernelGGL(k_load, dim3(grid_for(S.nnz_a, 256)), dim3(256), 0, st, values,
                           P->slot, num->arena, S.nnz_a);
    mark_end(num, st, 0, ev);
    const int32_t nl = (int32_t)S.level_ptr.size() - 1;
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t n0 = S.level_ptr[l], n1 = S.level_ptr[l + 1];
        const int wmax = P->level_maxw[l];
        const size_t lds_tri = (size_t)wmax * (wmax + 1) / 2 * sizeof(double);
        ev = mark_begin(num, st);
        hipLaunchKernelGGL(k_potrf, dim3(n1 - n0), dim3(256), lds_tri, st, P->level_sn + n0, a,
                           num->arena, num->status_dev);
        mark_end(num, st, 1, ev);
        const int64_t rb0 = P->rowblk_ptr[l], rb1 = P->rowblk_ptr[l + 1];
        if (rb1 > rb0) {
            ev = mark_begin(num, st);
            hipLaunchKernelGGL(k_trsm, dim3((unsigned)(rb1 - rb0)), dim3(kTile),
                               (size_t)wmax * kTile * sizeof(double), st, P->rowblk + rb0, a,
                               num->arena);
            mark_end(num, st, 2, ev);
        }
        const int64_t t0 = P->tile_ptr[l], t1 = P->tile_ptr[l + 1];
        if (t1 > t0) {
            ev = mark_begin(num, st);
            hipLaunchKernelGGL(k_update, dim3((unsigned)(t1 - t0)), dim3(256), 0, st,
                               P->tiles + t0, a, num->arena);
            mark_end(num, st, 3, ev);
        }
    }
    HIP_TRY(hipGetLastError());
    num->factored = true;
    return OK;
}

int32_t configure_kernels() {
    static int done = 0;
    static int32_t result = OK;
    if (done) return result;
    done = 1;
    const int lds_max = (int)(((size_t)kMaxWidth * (kMaxWidth + 1) / 2) * sizeof(double));
    if (hipFuncSetAttribute((const void*)k_potrf, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_max) != hipSuccess)
        result = ERR_HIP;
    if (hipFuncSetAttribute((const void*)k_trsm, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxWidth * kTile * (int)sizeof(double)) != hipSuccess)
        result = ERR_HIP;
    return result;
}

}  // namespace spc
