// Measurement helpers, not part of the factorization: what the device's
// matrix cores and HBM deliver to kernels that do nothing else, for stating
// the factorization's kernels against a measured ceiling beside the
// published peaks.
//   k_mfma_peak: every wave keeps 8 independent accumulators and issues
//                16 x 16 x 4 matrix-core products from registers (2048 flops
//                each), 8 waves per SIMD;
//   k_copy:      a streaming copy in 16-byte vectors (read + write).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/spchol.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kAcc = 8;

__global__ __launch_bounds__(256) void k_mfma_peak_f64(double* out, int iters, double seed) {
    const int lane = threadIdx.x & 63;
    double a = seed + lane, b = seed - lane;
    v4d acc[kAcc];
#pragma unroll
    for (int q = 0; q < kAcc; ++q) acc[q] = v4d{0.0, 0.0, 0.0, (double)q};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < kAcc; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kAcc; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    if (s == 12345.678) out[0] = s;  // keeps the products live
}

__global__ __launch_bounds__(256) void k_mfma_peak_f32(float* out, int iters, float seed) {
    const int lane = threadIdx.x & 63;
    float a = seed + lane, b = seed - lane;
    v4f acc[kAcc];
#pragma unroll
    for (int q = 0; q < kAcc; ++q) acc[q] = v4f{0.f, 0.f, 0.f, (float)q};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < kAcc; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kAcc; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    if (s == 12345.678f) out[0] = s;
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

extern "C" spc_status spc_measure_ceilings(spc_ceilings* out) {
    if (!out) return SPC_ERR_ARG;
    *out = spc_ceilings{};
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return SPC_ERR_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void* buf = nullptr;
    spc_status st = SPC_OK;
    const int iters = 4096;
    const unsigned blocks = (unsigned)std::max(1, ncu) * 8;  // 8 waves per SIMD
    const double flops = (double)blocks * 4 * iters * kAcc * 2048.0;
    const int64_t copy_bytes = int64_t(512) << 20;
    float ms = 0.f;
    auto timed = [&](auto launch) -> float {
        launch();  // warm-up
        if (hipEventRecord(e0, nullptr) != hipSuccess) return -1.f;
        launch();
        if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return -1.f;
        float t = 0.f;
        return hipEventElapsedTime(&t, e0, e1) == hipSuccess ? t : -1.f;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMalloc(&buf, 2 * (size_t)copy_bytes) != hipSuccess) {
        st = SPC_ERR_HIP;
        goto done;
    }
    ms = timed([&] {
        hipLaunchKernelGGL(k_mfma_peak_f64, dim3(blocks), dim3(256), 0, nullptr, (double*)buf,
                           iters, 1.0);
    });
    if (ms <= 0.f) { st = SPC_ERR_HIP; goto done; }
    out->fp64_mfma_tflops = flops / (ms * 1e-3) / 1e12;
    ms = timed([&] {
        hipLaunchKernelGGL(k_mfma_peak_f32, dim3(blocks), dim3(256), 0, nullptr, (float*)buf,
                           iters, 1.0f);
    });
    if (ms <= 0.f) { st = SPC_ERR_HIP; goto done; }
    out->fp32_mfma_tflops = flops / (ms * 1e-3) / 1e12;
    ms = timed([&] {
        const int64_t n4 = copy_bytes / 16;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)std::max(1, ncu) * 16), dim3(256), 0, nullptr,
                           (const float4*)buf, (float4*)((char*)buf + copy_bytes), n4);
    });
    if (ms <= 0.f) { st = SPC_ERR_HIP; goto done; }
    out->copy_gbs = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
done:
    if (buf) (void)hipFree(buf);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
}
