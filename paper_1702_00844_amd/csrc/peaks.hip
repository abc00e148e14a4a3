// Achievable instruction peaks of the device, for roofline reports: every
// wave issues independent matrix-core (or FMA) instructions from registers
// only, 8 waves per SIMD, and the rate is timed with HIP events.  This is the
// ceiling the correlator's kernels can approach on this device and clock,
// next to the published peaks.
#include "common.h"

namespace xc {
namespace peaks {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void f32_16(float *out, int iters, float seed) {
    v4f acc[8];
    for (int i = 0; i < 8; i++) acc[i] = v4f{0, 0, 0, 0};
    const float a = seed * threadIdx.x, b = seed + threadIdx.x;
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 8; i++) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 8; i++) s += acc[i][0] + acc[i][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void f32_32(float *out, int iters, float seed) {
    v16f acc[4];
    for (int i = 0; i < 4; i++) acc[i] = v16f{};
    const float a = seed * threadIdx.x, b = seed + threadIdx.x;
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 4; i++) s += acc[i][0] + acc[i][15];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void i8_32(float *out, int iters, float seed) {
    v16i acc[4];
    for (int i = 0; i < 4; i++) acc[i] = v16i{};
    const v4i a = {(int)threadIdx.x, 1, 2, 3}, b = {3, (int)seed, 1, 0};
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[i], 0, 0, 0);
    int s = 0;
    for (int i = 0; i < 4; i++) s += acc[i][0] + acc[i][15];
    out[blockIdx.x * 256 + threadIdx.x] = (float)s;
}
__global__ __launch_bounds__(256) void f16_32(float *out, int iters, float seed) {
    v16f acc[4];
    for (int i = 0; i < 4; i++) acc[i] = v16f{};
    v8h a, b;
    for (int e = 0; e < 8; e++) {
        a[e] = (_Float16)(seed * e);
        b[e] = (_Float16)(threadIdx.x * 0.001f);
    }
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 4; i++) s += acc[i][0] + acc[i][15];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void bf16_32(float *out, int iters, float seed) {
    v16f acc[4];
    for (int i = 0; i < 4; i++) acc[i] = v16f{};
    v8bf a, b;
    for (int e = 0; e < 8; e++) {
        a[e] = (__bf16)(seed * e);
        b[e] = (__bf16)(threadIdx.x * 0.001f);
    }
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < 4; i++) s += acc[i][0] + acc[i][15];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void fma32(float *out, int iters, float seed) {
    float acc[32];
    for (int i = 0; i < 32; i++) acc[i] = seed * i;
    const float a = seed * threadIdx.x, b = 1.0f - seed;
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int i = 0; i < 32; i++) acc[i] = fmaf(acc[i], b, a);
    float s = 0;
    for (int i = 0; i < 32; i++) s += acc[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
// Stream copy of n float4 (HBM read + write).
__global__ __launch_bounds__(256) void copy4(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 256;
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace peaks
}  // namespace xc

using namespace xc;

extern "C" {

xc_status xc_measure_peak(int32_t which, double *value) {
    if (!value) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (which < XC_PEAK_F32_MFMA16 || which > XC_PEAK_HBM_COPY)
        return set_error(XC_ERR_INVALID_ARG, "unknown peak %d", which);
    const int cus = device_cu_count();
    const int blocks = cus * 8;   // 8 workgroups of 4 waves per CU
    float *out = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float));
    if (e != hipSuccess) return set_error(XC_ERR_OUT_OF_MEMORY, "hipMalloc: %s", hipGetErrorString(e));
    void *src = nullptr, *dst = nullptr;
    const size_t copy_bytes = (size_t)1 << 30;
    if (which == XC_PEAK_HBM_COPY) {
        e = hipMalloc(&src, copy_bytes);
        if (e == hipSuccess) e = hipMalloc(&dst, copy_bytes);
        if (e == hipSuccess) e = hipMemset(src, 0, copy_bytes);
        if (e != hipSuccess) {
            (void)hipFree(out);
            if (src) (void)hipFree(src);
            if (dst) (void)hipFree(dst);
            return set_error(XC_ERR_OUT_OF_MEMORY, "hipMalloc: %s", hipGetErrorString(e));
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto launch = [&](int iters) {
        switch (which) {
        case XC_PEAK_F32_MFMA16: hipLaunchKernelGGL(peaks::f32_16, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        case XC_PEAK_F32_MFMA32: hipLaunchKernelGGL(peaks::f32_32, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        case XC_PEAK_I8_MFMA: hipLaunchKernelGGL(peaks::i8_32, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        case XC_PEAK_F16_MFMA: hipLaunchKernelGGL(peaks::f16_32, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        case XC_PEAK_BF16_MFMA: hipLaunchKernelGGL(peaks::bf16_32, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        case XC_PEAK_F32_FMA: hipLaunchKernelGGL(peaks::fma32, dim3(blocks), dim3(256), 0, 0, out, iters, 0.5f); break;
        default:
            for (int k = 0; k < iters; ++k)
                hipLaunchKernelGGL(peaks::copy4, dim3(cus * 16), dim3(256), 0, 0, static_cast<const float4 *>(src),
                                   static_cast<float4 *>(dst), copy_bytes / 16);
        }
    };
    const int iters = which == XC_PEAK_HBM_COPY ? 10 : 4000;
    launch(which == XC_PEAK_HBM_COPY ? 1 : 10);   // warm-up
    (void)hipEventRecord(e0, 0);
    launch(iters);
    (void)hipEventRecord(e1, 0);
    e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (e != hipSuccess) return hip_error(e, "peak measurement");
    const double waves = (double)blocks * 4.0;
    double work = 0;   // flops (or bytes) of the timed region
    switch (which) {
    case XC_PEAK_F32_MFMA16: work = waves * iters * 8.0 * 16 * 16 * 4 * 2; break;
    case XC_PEAK_F32_MFMA32: work = waves * iters * 4.0 * 32 * 32 * 2 * 2; break;
    case XC_PEAK_I8_MFMA: work = waves * iters * 4.0 * 32 * 32 * 32 * 2; break;
    case XC_PEAK_F16_MFMA:
    case XC_PEAK_BF16_MFMA: work = waves * iters * 4.0 * 32 * 32 * 16 * 2; break;
    case XC_PEAK_F32_FMA: work = waves * iters * 32.0 * 2 * 64; break;
    default: work = 2.0 * (double)copy_bytes * iters; break;
    }
    *value = work / (ms * 1e-3) / (which == XC_PEAK_HBM_COPY ? 1e9 : 1e12);
    return XC_OK;
}

}  // extern "C"
