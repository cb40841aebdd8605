// Iterative refinement in FP64 around the supernodal factor: the mixed-
// precision form of the solve.  The factor (FP32 or FP64) gives corrections;
// the residual r = b - A x, its norms and the update x += d stay in FP64:
//
//   x = 0
//   repeat:  r = b - A x                        (FP64, full CSR of A)
//            eta_c = ||r_c|| / (||A|| ||x_c|| + ||b_c||)   (inf-norms, per column)
//            stop when every eta_c <= tol
//            d = (L L^T)^{-1} P (r / ||r||)    (gather, scaled, in the factor's type;
//                                              level sweeps of the solve)
//            x += ||r|| P^T d                  (FP64)
//
// Scaling r by its norm before the rounding to FP32 keeps every correction
// solve in the normal range of FP32.  eta is the normwise backward error of
// Rigal and Gaches in the infinity norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/spchol.h"
#include "runtime.hpp"

namespace spc {

#define HIP_TRY(x)                               \
    do {                                         \
        if ((x) != hipSuccess) return ERR_HIP;   \
    } while (0)

namespace {

// Groups of 64 rows walked by one wave of the row kernels.
constexpr int kRowsPerWave = 16;
// Right-hand sides per pass of the residual kernel.
constexpr int kResidCols = 8;

int grid_of(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

// One thread per element.
unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }
// Row kernels: each wave covers kRowsPerWave x 64 consecutive rows.
unsigned row_blocks(int64_t n) {
    const int64_t per_block = 4 * 64 * (int64_t)kRowsPerWave;
    return (unsigned)std::max<int64_t>(1, (n + per_block - 1) / per_block);
}

// Non-negative doubles order like their bit patterns as unsigned integers.
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Per-matrix maxima over rows.  Every wave walks kRowsPerWave consecutive
// groups of 64 rows and carries a wave-uniform (matrix, max) pair: a group
// whose rows all lie in one matrix is reduced across the wave and merged
// into the pair (flushed with one atomic when the matrix changes); a group
// that straddles matrices issues one atomic per lane.  One matrix costs one
// atomic per wave, not per row.

struct SegMax {
    int seg = -1;
    double m = 0.0;
    __device__ __forceinline__ void add(double* out, int segi, double v) {
        const int s0 = __shfl(segi, 0, 64);
        if (__all(segi == s0 || segi < 0) && s0 >= 0) {
            for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
            if (s0 != seg) {
                flush(out);
                seg = s0;
                m = v;
            } else {
                m = fmax(m, v);
            }
        } else if (segi >= 0) {
            atomic_max_nonneg(out + segi, v);
        }
    }
    __device__ __forceinline__ void flush(double* out) {
        if (seg >= 0 && (threadIdx.x & 63) == 0) atomic_max_nonneg(out + seg, m);
    }
};

// Row handled by this lane in step u of its wave's range.
__device__ __forceinline__ int64_t row_of(int u) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    return (wave * kRowsPerWave + u) * 64 + (threadIdx.x & 63);
}

__device__ __forceinline__ int seg_of(const int32_t* seg, int64_t i, int64_t n) {
    return i < n ? (seg ? seg[i] : 0) : -1;
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// x[:, c] = 0 for the caller's column-major x with leading dimension ldx.
__global__ void k_zero_cols(double* __restrict__ x, int64_t ldx, int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        x[i + c * ldx] = 0.0;
    }
}

// a_val[q] = values[a_src[q]]: the caller's lower-CSC values into the full CSR.
__global__ void k_gather_vals(const double* __restrict__ values, const int64_t* __restrict__ src,
                              double* __restrict__ aval, int64_t nnz) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x)
        aval[q] = values[src[q]];
}

// Sparse row kernels: a group of kLpr consecutive lanes takes one row (lane j
// of the group reads entries ptr[i] + j, + kLpr, ... so the group's loads of
// val and col are contiguous), the partial sums meet by shuffles, and each
// wave walks kRowGroups groups of 64 / kLpr consecutive rows.
// The single-column residual of matrices with short rows (at most six
// entries on average, the 2D stencils) uses groups of kLprShort lanes.
constexpr int kLpr = 8;
constexpr int kLprShort = 4;
constexpr int kRowGroups = 16;
template <int L = kLpr>
unsigned sparse_blocks(int64_t n) {
    const int64_t per_block = 4 * (64 / L) * (int64_t)kRowGroups;
    return (unsigned)std::max<int64_t>(1, (n + per_block - 1) / per_block);
}
// Row of this lane's group in step u, and the lane's place in the group.
template <int L = kLpr>
__device__ __forceinline__ int64_t sparse_row(int u) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    return (wave * kRowGroups + u) * (64 / L) + ((threadIdx.x & 63) / L);
}
template <int L = kLpr>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ||A_k||_inf = max over the rows of matrix k of the absolute row sum.
__global__ __launch_bounds__(256) void k_anorm(const int64_t* __restrict__ ptr,
                                               const double* __restrict__ val,
                                               const int32_t* __restrict__ seg, int64_t n,
                                               double* __restrict__ out) {
    const int j = threadIdx.x % kLpr;
    SegMax sm;
    for (int u = 0; u < kRowGroups; ++u) {
        const int64_t i = sparse_row(u);
        double s = 0.0;
        if (i < n)
            for (int64_t q = ptr[i] + j; q < ptr[i + 1]; q += kLpr) s += fabs(val[q]);
        s = group_sum(s);
        sm.add(out, seg_of(seg, i, n), s);
    }
    sm.flush(out);
}

// ||v_{k,c}||_inf per matrix k and column c (blockIdx.y); out[c * nseg + k].
__global__ __launch_bounds__(256) void k_colmax(const double* __restrict__ v, int64_t ld, int64_t n,
                                                const int32_t* __restrict__ seg, int64_t nseg,
                                                double* __restrict__ out) {
    const int c = blockIdx.y;
    SegMax sm;
    for (int u = 0; u < kRowsPerWave; ++u) {
        const int64_t i = row_of(u);
        sm.add(out + c * nseg, seg_of(seg, i, n), i < n ? fabs(v[i + c * ld]) : 0.0);
    }
    sm.flush(out + c * nseg);
}

// xt[k NR + c] = x[k + (c0 + c) ldx] (zero past nrhs): the NR columns of x
// interleaved, so that the residual's gather of row k of x is one
// contiguous read instead of NR reads NR cache lines apart.
template <int NR>
__global__ void k_interleave(const double* __restrict__ x, int64_t ldx, double* __restrict__ xt,
                             int64_t n, int c0, int nrhs) {
    const int64_t total = n * NR;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / NR;
        const int c = (int)(e % NR);
        xt[e] = c0 + c < nrhs ? x[k + (int64_t)(c0 + c) * ldx] : 0.0;
    }
}

// r_c = b_c - A x_c and ||r_{k,c}||_inf for the columns c0 .. c0 + NR - 1
// (those below nrhs) in one pass over A: each entry of A is read once and
// multiplies NR gathered entries of x (NR > 1: from the interleaved copy xt,
// row k at xt + k NR).
template <int NR, int L = kLpr>
__global__ __launch_bounds__(256) void k_resid(const int64_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ val,
                                               const double* __restrict__ b, int64_t ldb,
                                               const double* __restrict__ x, int64_t ldx,
                                               double* __restrict__ r, int64_t n, int c0,
                                               int nrhs, const int32_t* __restrict__ seg,
                                               int64_t nseg, double* __restrict__ rnorm) {
    const int j = threadIdx.x % L;
    const int nc = min(NR, nrhs - c0);
    SegMax sm[NR];
    for (int u = 0; u < kRowGroups; ++u) {
        const int64_t i = sparse_row<L>(u);
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = 0.0;
        if (i < n) {
            for (int64_t q = ptr[i] + j; q < ptr[i + 1]; q += L) {
                const double v = val[q];
                const int64_t k = col[q];
                if (NR == 1) {
                    acc[0] += v * x[k + (int64_t)c0 * ldx];
                } else {
                    const double* __restrict__ xk = x + k * NR;
#pragma unroll
                    for (int c = 0; c < NR; ++c) acc[c] += v * xk[c];
                }
            }
        }
        const int si = seg_of(seg, i, n);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (c >= nc) break;  // uniform
            const double s = group_sum<L>(acc[c]);
            double ri = 0.0;
            if (i < n) {
                ri = b[i + (int64_t)(c0 + c) * ldb] - s;
                if (j == 0) r[i + (int64_t)(c0 + c) * n] = ri;
            }
            sm[c].add(rnorm + (int64_t)(c0 + c) * nseg, si, fabs(ri));
        }
    }
#pragma unroll
    for (int c = 0; c < NR; ++c)
        if (c < nc) sm[c].flush(rnorm + (int64_t)(c0 + c) * nseg);
}

// eta and the scale 1 / ||r|| of the next correction (0 when r = 0), per
// (column, matrix) entry e = c * nseg + k.
__global__ void k_eta(const double* __restrict__ rn, const double* __restrict__ xn,
                      const double* __restrict__ bn, const double* __restrict__ anorm,
                      int64_t nseg, double* __restrict__ eta, double* __restrict__ scale,
                      int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const double den = anorm[e % nseg] * xn[e] + bn[e];
    eta[e] = den > 0.0 ? rn[e] / den : (rn[e] > 0.0 ? 1.0 : 0.0);
    scale[e] = rn[e] > 0.0 ? 1.0 / rn[e] : 0.0;
}

// y = P (r / ||r||) rounded to the factor's type (each matrix scaled by its own norm).
template <class R>
__global__ void k_gather_scaled(const double* __restrict__ r, const int32_t* __restrict__ perm,
                                const int32_t* __restrict__ seg, int64_t nseg,
                                const double* __restrict__ scale, R* __restrict__ y, int64_t n,
                                int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        const int32_t o = perm[i];
        y[e] = (R)(r[o + c * n] * scale[c * nseg + (seg ? seg[o] : 0)]);
    }
}

// x += ||r|| P^T y in FP64.
template <class R>
__global__ void k_scatter_add(const R* __restrict__ y, const int32_t* __restrict__ perm,
                              const int32_t* __restrict__ seg, int64_t nseg,
                              const double* __restrict__ rn, double* __restrict__ x, int64_t ldx,
                              int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        const int32_t o = perm[i];
        x[o + c * ldx] += (double)y[e] * rn[c * nseg + (seg ? seg[o] : 0)];
    }
}

// One correction with factor f (num itself, or its FP64 fallback factor),
// the batch segments and norms of num.
template <class R>
void correction(spc_numeric* num, spc_numeric* f, int32_t nrhs, const double* r,
                const double* scale, const double* rn, double* x, int64_t ldx, hipStream_t st,
                int32_t* rc) {
    const int64_t n = num->sym->S.n;
    const int32_t* perm = f->plan->perm;
    const int g = grid_of(n * nrhs);
    hipLaunchKernelGGL(k_gather_scaled<R>, dim3(g), dim3(256), 0, st, r, perm,
                       (const int32_t*)num->a_seg, num->nseg, scale, (R*)f->work, n, nrhs);
    *rc = run_sweeps(f, nrhs, st);
    if (*rc != OK) return;
    hipLaunchKernelGGL(k_scatter_add<R>, dim3(g), dim3(256), 0, st, (const R*)f->work, perm,
                       (const int32_t*)num->a_seg, num->nseg, rn, x, ldx, n, nrhs);
}

// A's values in the caller's order, from the refinement copy (every input
// entry appears once or, off the diagonal, twice with the same value).
__global__ void k_values_from_csr(const double* __restrict__ val, const int64_t* __restrict__ src,
                                  double* __restrict__ out, int64_t nnzf) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzf;
         e += (int64_t)gridDim.x * blockDim.x)
        out[src[e]] = val[e];
}

// The FP64 factor of num's matrix for stalled refinement: allocated on first
// use, factored from the refinement copy of A once per factorization of num.
int32_t fallback_factor(spc_numeric* num, int32_t nrhs, hipStream_t st) {
    if (!num->fb) {
        int32_t rc = numeric_create_prec(num->sym, 0, &num->fb);
        if (rc != OK) return rc;
        const int64_t nnz = num->sym->S.nnz_a;
        if (hipMalloc(&num->fb_values, sizeof(double) * (size_t)std::max<int64_t>(nnz, 1)) !=
            hipSuccess)
            return ERR_OOM;
        num->fb_current = false;
    }
    int32_t rc = ensure_solve_work(num->fb, nrhs);
    if (rc != OK) return rc;
    if (!num->fb_current) {
        if (num->a_nnz > 0)
            hipLaunchKernelGGL(k_values_from_csr, dim3(grid_of(num->a_nnz)), dim3(256), 0, st,
                               (const double*)num->a_val, (const int64_t*)num->a_src,
                               num->fb_values, num->a_nnz);
        rc = run_factor(num->fb, num->fb_values, st);
        if (rc != OK) return rc;
        rc = spc_numeric_status(num->fb);
        if (rc != OK) return rc;
        num->fb_current = true;
    }
    return OK;
}

}  // namespace

// Full symmetric CSR of the input matrix A (original numbering), built on
// the host from the permuted lower pattern: entry q of C = lower(P A P^T) in
// row i, column j is A(perm[i], perm[j]); each stored entry appears in row
// perm[i] and, off the diagonal, in row perm[j].  a_src maps every CSR entry
// to the caller's value index.
static int32_t build_refine_matrix(spc_numeric* num) {
    const Symbolic& S = num->sym->S;
    const int64_t n = S.n, nnz = S.nnz_a;
    std::vector<int64_t> inv_amap((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) inv_amap[(size_t)S.amap[k]] = k;
    std::vector<int64_t> ptr((size_t)n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t q = S.Cp[j]; q < S.Cp[j + 1]; ++q) {
            const int64_t i = S.Ci[q];
            ptr[(size_t)S.perm[i] + 1]++;
            if (i != j) ptr[(size_t)S.perm[j] + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    const int64_t nnzf = ptr[n];
    num->a_nnz = nnzf;
    std::vector<int32_t> col((size_t)std::max<int64_t>(nnzf, 1));
    std::vector<int64_t> src((size_t)std::max<int64_t>(nnzf, 1));
    std::vector<int64_t> next(ptr.begin(), ptr.end() - 1);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t q = S.Cp[j]; q < S.Cp[j + 1]; ++q) {
            const int64_t i = S.Ci[q];
            const int32_t oi = S.perm[i], oj = S.perm[j];
            int64_t at = next[oi]++;
            col[at] = oj;
            src[at] = inv_amap[q];
            if (i != j) {
                at = next[oj]++;
                col[at] = oi;
                src[at] = inv_amap[q];
            }
        }
    const size_t b_ptr = sizeof(int64_t) * (size_t)(n + 1);
    const size_t b_nz = (size_t)std::max<int64_t>(nnzf, 1);
    if (hipMalloc(&num->a_ptr, b_ptr) != hipSuccess) return ERR_OOM;
    if (hipMalloc(&num->a_col, sizeof(int32_t) * b_nz) != hipSuccess) return ERR_OOM;
    if (hipMalloc(&num->a_src, sizeof(int64_t) * b_nz) != hipSuccess) return ERR_OOM;
    if (hipMalloc(&num->a_val, sizeof(double) * b_nz) != hipSuccess) return ERR_OOM;
    num->nseg = std::max<int64_t>(1, (int64_t)S.batch_ptr.size() - 1);
    if (hipMalloc(&num->a_norm, sizeof(double) * (size_t)num->nseg) != hipSuccess) return ERR_OOM;
    if (num->nseg > 1) {
        std::vector<int32_t> seg((size_t)n);
        for (int64_t k = 0; k + 1 < (int64_t)S.batch_ptr.size(); ++k)
            for (int64_t i = S.batch_ptr[k]; i < S.batch_ptr[k + 1]; ++i) seg[i] = (int32_t)k;
        if (hipMalloc(&num->a_seg, sizeof(int32_t) * (size_t)n) != hipSuccess) return ERR_OOM;
        HIP_TRY(hipMemcpy(num->a_seg, seg.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(num->a_ptr, ptr.data(), b_ptr, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(num->a_col, col.data(), sizeof(int32_t) * b_nz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(num->a_src, src.data(), sizeof(int64_t) * b_nz, hipMemcpyHostToDevice));
    return OK;
}

int32_t load_refine_matrix(spc_numeric* num, const double* values, hipStream_t st) {
    const Symbolic& S = num->sym->S;
    if (!num->a_ptr) {
        const int32_t r = build_refine_matrix(num);
        if (r != OK) return r;
    }
    const int64_t nnzf = num->a_nnz;
    if (nnzf > 0)
        hipLaunchKernelGGL(k_gather_vals, dim3(grid_of(nnzf)), dim3(256), 0, st, values,
                           (const int64_t*)num->a_src, num->a_val, nnzf);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_of(num->nseg)), dim3(256), 0, st, num->a_norm,
                       num->nseg, 0.0);
    if (S.n > 0)
        hipLaunchKernelGGL(k_anorm, dim3(sparse_blocks(S.n)), dim3(256), 0, st,
                           (const int64_t*)num->a_ptr, (const double*)num->a_val,
                           (const int32_t*)num->a_seg, S.n, num->a_norm);
    HIP_TRY(hipGetLastError());
    return OK;
}

void free_refine(spc_numeric* num) {
    (void)hipFree(num->a_ptr);
    (void)hipFree(num->a_col);
    (void)hipFree(num->a_src);
    (void)hipFree(num->a_val);
    (void)hipFree(num->a_norm);
    (void)hipFree(num->a_seg);
    (void)hipFree(num->ir_work);
    if (num->ir_host) (void)hipHostFree(num->ir_host);
    num->a_ptr = nullptr;
    num->a_col = nullptr;
    num->a_src = nullptr;
    num->a_val = nullptr;
    num->a_norm = nullptr;
    num->a_seg = nullptr;
    num->ir_work = nullptr;
    num->ir_host = nullptr;
    num->ir_cols = 0;
}

int32_t run_refine(spc_numeric* num, int32_t nrhs, const double* b, int64_t ldb, double* x,
                   int64_t ldx, double tol, int32_t max_iter, hipStream_t st, int32_t* iters,
                   double* berr) {
    const int64_t n = num->sym->S.n;
    const int64_t ns = num->nseg;
    const int64_t ne = ns * nrhs;  // (column, matrix) entries
    if (iters) *iters = 0;
    if (n == 0 || nrhs == 0) {
        for (int64_t e = 0; berr && e < ne; ++e) berr[e] = 0.0;
        return OK;
    }
    int32_t rc = ensure_solve_work(num, nrhs);
    if (rc != OK) return rc;
    if (num->ir_cols < nrhs) {
        (void)hipFree(num->ir_work);
        if (num->ir_host) (void)hipHostFree(num->ir_host);
        num->ir_work = nullptr;
        num->ir_host = nullptr;
        num->ir_cols = 0;
        if (hipMalloc(&num->ir_work, sizeof(double) * (((size_t)n + 5 * (size_t)ns) * nrhs +
                                                       (size_t)n * kResidCols)) != hipSuccess)
            return ERR_OOM;
        if (hipHostMalloc(&num->ir_host, sizeof(double) * (size_t)ns * nrhs,
                          hipHostMallocDefault) != hipSuccess)
            return ERR_OOM;
        num->ir_cols = nrhs;
    }
    double* r = num->ir_work;
    double* bn = r + (size_t)n * nrhs;
    double* xn = bn + ne;
    double* rn = xn + ne;
    double* eta = rn + ne;
    double* scale = eta + ne;
    double* xt = scale + ne;  // n x kResidCols, x's columns interleaved for the residual
    const int32_t* seg = num->a_seg;
    const dim3 grid_rows(row_blocks(n), nrhs);
    // stall: consecutive steps whose worst eta did not halve; two of them on
    // an FP32 factor switch the corrections to the FP64 factor, on an FP64
    // factor they end the refinement
    int stall = 0;
    double prev_worst = 0.0;
    bool on_fb = false;
    hipLaunchKernelGGL(k_zero_cols, dim3(grid_of(n * nrhs)), dim3(256), 0, st, x, ldx, n, nrhs);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_of(ne)), dim3(256), 0, st, bn, ne, 0.0);
    hipLaunchKernelGGL(k_colmax, grid_rows, dim3(256), 0, st, b, ldb, n, seg, ns, bn);
    for (int32_t it = 0;; ++it) {
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_of(2 * ne)), dim3(256), 0, st, xn, 2 * ne, 0.0);
        for (int32_t c0 = 0; c0 < nrhs; c0 += kResidCols) {
            if (nrhs - c0 == 1) {
                const bool short_rows = num->a_nnz <= 6 * n;
                auto kern = short_rows ? k_resid<1, kLprShort> : k_resid<1>;
                const unsigned g = short_rows ? sparse_blocks<kLprShort>(n) : sparse_blocks(n);
                hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, st, (const int64_t*)num->a_ptr,
                                   (const int32_t*)num->a_col, (const double*)num->a_val, b, ldb,
                                   (const double*)x, ldx, r, n, (int)c0, (int)nrhs, seg, ns, rn);
            } else {
                hipLaunchKernelGGL(k_interleave<kResidCols>, dim3(grid_of(n * kResidCols)),
                                   dim3(256), 0, st, (const double*)x, ldx, xt, n, (int)c0,
                                   (int)nrhs);
                hipLaunchKernelGGL(k_resid<kResidCols>, dim3(sparse_blocks(n)), dim3(256), 0, st,
                                   (const int64_t*)num->a_ptr, (const int32_t*)num->a_col,
                                   (const double*)num->a_val, b, ldb, (const double*)xt,
                                   (int64_t)kResidCols, r, n, (int)c0, (int)nrhs, seg, ns, rn);
            }
        }
        hipLaunchKernelGGL(k_colmax, grid_rows, dim3(256), 0, st, (const double*)x, ldx, n, seg,
                           ns, xn);
        hipLaunchKernelGGL(k_eta, dim3(blocks_of(ne)), dim3(256), 0, st, (const double*)rn,
                           (const double*)xn, (const double*)bn, (const double*)num->a_norm, ns,
                           eta, scale, ne);
        HIP_TRY(hipMemcpyAsync(num->ir_host, eta, sizeof(double) * ne, hipMemcpyDeviceToHost,
                               st));
        HIP_TRY(hipStreamSynchronize(st));
        bool done = true;
        double worst = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            const double v = num->ir_host[e];
            if (berr) berr[e] = v;
            if (!(v <= tol)) done = false;
            worst = (v > worst || v != v) ? v : worst;
        }
        if (iters) *iters = it;
        if (done) return OK;
        if (it >= max_iter) return ERR_NOT_CONVERGED;
        if (it > 0) stall = (worst > 0.5 * prev_worst || worst != worst) ? stall + 1 : 0;
        prev_worst = worst;
        if (stall >= 2) {
            if (num->prec != 1 || on_fb) return ERR_NOT_CONVERGED;
            rc = fallback_factor(num, nrhs, st);
            if (rc != OK) return rc;
            on_fb = true;
            stall = 0;
            num->refine_fallbacks++;
        }
        if (on_fb)
            correction<double>(num, num->fb, nrhs, r, scale, rn, x, ldx, st, &rc);
        else if (num->prec == 1)
            correction<float>(num, num, nrhs, r, scale, rn, x, ldx, st, &rc);
        else
            correction<double>(num, num, nrhs, r, scale, rn, x, ldx, st, &rc);
        if (rc != OK) return rc;
        HIP_TRY(hipGetLastError());
    }
}

}  // namespace spc
