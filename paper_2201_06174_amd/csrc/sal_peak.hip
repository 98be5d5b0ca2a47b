// sal_peak.hip -- microbenchmarks of the device's own matrix-core, vector-ALU and HBM rates
// (the measured denominators of the roofline fractions; no step of the method uses them).
#include <hip/hip_runtime.h>

#include "../../include/sal_peak.h"
#include "sal_internal.h"

namespace sal {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kPeakThreads = 256;
constexpr int kMfmaChains = 4;
constexpr int kValuChains = 8;
constexpr int64_t kMaxIters = 16384;
constexpr int64_t kMaxBlocks = int64_t(1) << 20;

// Four independent accumulator chains per wave keep the matrix core of each SIMD issuing back to
// back; with every operand 1 each product adds K to each accumulator.  FP32: 16x16x4 (4
// accumulators per lane, K = 4; four chains sustained the published rate, eight only about 80 %
// of it).  BF16 and FP16: the 32x32x16 form (16 accumulators, K = 16), which has the rate of the
// 16x16x32 form the feature kernels use and whose accumulators the compiler keeps in place across
// iterations (around 16x16x32 chains it copies them between registers every iteration).
template <int KIND>
__global__ __launch_bounds__(kPeakThreads) void k_peak_mfma(int64_t iters, float* out) {
    float sum = 0.f;
    if constexpr (KIND == SAL_PEAK_MFMA_F32) {
        f4 acc[kMfmaChains];
#pragma unroll
        for (int c = 0; c < kMfmaChains; c++) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        const float a = 1.f;
        for (int64_t i = 0; i < iters; i++)
#pragma unroll
            for (int c = 0; c < kMfmaChains; c++) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < kMfmaChains; c++) sum += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else {
        f16v acc[kMfmaChains];
#pragma unroll
        for (int c = 0; c < kMfmaChains; c++) acc[c] = f16v{};
        if constexpr (KIND == SAL_PEAK_MFMA_BF16) {
            bf8 a;
#pragma unroll
            for (int e = 0; e < 8; e++) a[e] = (__bf16)1.f;
            for (int64_t i = 0; i < iters; i++)
#pragma unroll
                for (int c = 0; c < kMfmaChains; c++)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, acc[c], 0, 0, 0);
        } else {
            h8 a;
#pragma unroll
            for (int e = 0; e < 8; e++) a[e] = (_Float16)1.f;
            for (int64_t i = 0; i < iters; i++)
#pragma unroll
                for (int c = 0; c < kMfmaChains; c++)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, a, acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < kMfmaChains; c++)
#pragma unroll
            for (int j = 0; j < 16; j++) sum += acc[c][j];
    }
    out[(int64_t)blockIdx.x * kPeakThreads + threadIdx.x] = sum;
}

// a and b arrive as kernel arguments (both 1), so each step stays one v_fma_f32
__global__ __launch_bounds__(kPeakThreads) void k_peak_valu(int64_t iters, float a, float b, float* out) {
    float acc[kValuChains];
#pragma unroll
    for (int c = 0; c < kValuChains; c++) acc[c] = 0.f;
#pragma unroll 4
    for (int64_t i = 0; i < iters; i++)
#pragma unroll
        for (int c = 0; c < kValuChains; c++) acc[c] = fmaf(acc[c], a, b);
    float sum = 0.f;
#pragma unroll
    for (int c = 0; c < kValuChains; c++) sum += acc[c];
    out[(int64_t)blockIdx.x * kPeakThreads + threadIdx.x] = sum;
}

__global__ __launch_bounds__(kPeakThreads) void k_peak_read(const float4* src, int64_t words, float* out) {
    const int64_t tid = (int64_t)blockIdx.x * kPeakThreads + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kPeakThreads;
    float sum = 0.f;
    for (int64_t i = tid; i < words; i += stride) {
        const float4 v = src[i];
        sum += (v.x + v.y) + (v.z + v.w);
    }
    out[tid] = sum;
}

__global__ __launch_bounds__(kPeakThreads) void k_peak_copy(const float4* src, float4* dst, int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * kPeakThreads;
    for (int64_t i = (int64_t)blockIdx.x * kPeakThreads + threadIdx.x; i < words; i += stride) dst[i] = src[i];
}

// flops of one loop iteration of one wave
int64_t wave_iteration_flops(int kind) {
    switch (kind) {
        case SAL_PEAK_MFMA_F32: return kMfmaChains * (16 * 16 * 4 * 2);
        case SAL_PEAK_MFMA_BF16:
        case SAL_PEAK_MFMA_F16: return kMfmaChains * (32 * 32 * 16 * 2);
        default: return 64 * kValuChains * 2;
    }
}

}  // namespace
}  // namespace sal

using namespace sal;

extern "C" {

int64_t sal_peak_compute_flops(int kind, int64_t iters, int64_t blocks) {
    if (kind < SAL_PEAK_MFMA_F32 || kind > SAL_PEAK_VALU_F32 || iters < 1 || iters > kMaxIters || blocks < 1 ||
        blocks > kMaxBlocks)
        return 0;
    return blocks * (kPeakThreads / 64) * iters * wave_iteration_flops(kind);
}

sal_status sal_peak_compute(int kind, int64_t iters, int64_t blocks, float* out, sal_stream stream) {
    if (kind < SAL_PEAK_MFMA_F32 || kind > SAL_PEAK_VALU_F32) return fail(SAL_ERR_ARG, "unknown peak kind");
    if (iters < 1 || iters > kMaxIters) return fail(SAL_ERR_ARG, "iters must be 1..16384");
    if (blocks < 1 || blocks > kMaxBlocks) return fail(SAL_ERR_ARG, "blocks must be 1..2^20");
    if (!out) return fail(SAL_ERR_ARG, "out is NULL");
    const dim3 grid((unsigned)blocks), block(kPeakThreads);
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case SAL_PEAK_MFMA_F32: hipLaunchKernelGGL(k_peak_mfma<SAL_PEAK_MFMA_F32>, grid, block, 0, st, iters, out); break;
        case SAL_PEAK_MFMA_BF16: hipLaunchKernelGGL(k_peak_mfma<SAL_PEAK_MFMA_BF16>, grid, block, 0, st, iters, out); break;
        case SAL_PEAK_MFMA_F16: hipLaunchKernelGGL(k_peak_mfma<SAL_PEAK_MFMA_F16>, grid, block, 0, st, iters, out); break;
        default: hipLaunchKernelGGL(k_peak_valu, grid, block, 0, st, iters, 1.f, 1.f, out); break;
    }
    return check_hip(hipGetLastError(), "launch peak compute kernel");
}

sal_status sal_peak_stream(int kind, const void* src, void* dst, int64_t bytes, float* out, int64_t blocks,
                           sal_stream stream) {
    if (kind != 0 && kind != 1) return fail(SAL_ERR_ARG, "stream kind must be 0 (read) or 1 (copy)");
    if (bytes < 16 || bytes % 16) return fail(SAL_ERR_ARG, "bytes must be a positive multiple of 16");
    if (blocks < 1 || blocks > kMaxBlocks) return fail(SAL_ERR_ARG, "blocks must be 1..2^20");
    if (!src || ((uintptr_t)src & 15)) return fail(SAL_ERR_ARG, "src must be a 16-byte aligned device pointer");
    if (kind == 0 && !out) return fail(SAL_ERR_ARG, "out is NULL");
    if (kind == 1) {
        if (!dst || ((uintptr_t)dst & 15)) return fail(SAL_ERR_ARG, "dst must be a 16-byte aligned device pointer");
        const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
        if (s0 < d0 + (uintptr_t)bytes && d0 < s0 + (uintptr_t)bytes) return fail(SAL_ERR_ARG, "src and dst overlap");
    }
    const dim3 grid((unsigned)blocks), block(kPeakThreads);
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0)
        hipLaunchKernelGGL(k_peak_read, grid, block, 0, st, (const float4*)src, bytes / 16, out);
    else
        hipLaunchKernelGGL(k_peak_copy, grid, block, 0, st, (const float4*)src, (float4*)dst, bytes / 16);
    return check_hip(hipGetLastError(), "launch peak stream kernel");
}

}  // extern "C"
