// MFMA-only throughput kernels (include/mm_peak.h): each wave keeps CH
// independent accumulator chains busy, so with enough chains the matrix cores
// never wait on a dependency; no memory traffic inside the loop.  The binary64
// chains read distinct operand registers (shared ones measured a third slower).
#include <hip/hip_runtime.h>

#include "../../include/mm_peak.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int CH>
__global__ __launch_bounds__(256) void peak_f64(float *out, int iters) {
    d4 acc[CH];
    double a[CH], b[CH];   // each chain reads its own operand registers, as a GEMM's blocks do
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        acc[i] = d4{0, 0, 0, 0};
        a[i] = threadIdx.x * 1e-3 + i;
        b[i] = 1.0 + blockIdx.x * 1e-9 + i * 1e-6;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[(i + 1) % CH], acc[i], 0, 0, 0);
    }
    double s = 0;
#pragma unroll
    for (int i = 0; i < CH; ++i) s += acc[i][0] + acc[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

template <int CH>
__global__ __launch_bounds__(256) void peak_f32(float *out, int iters) {
    f4 acc[CH];
    const float a = threadIdx.x * 1e-3f, b = 1.0f;
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
    }
    float s = 0;
#pragma unroll
    for (int i = 0; i < CH; ++i) s += acc[i][0] + acc[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void peak_bf16(float *out, int iters) {
    f4 acc[CH];
    bf8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(threadIdx.x * 1e-3f);
        b[e] = (__bf16)1.0f;
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
    }
    float s = 0;
#pragma unroll
    for (int i = 0; i < CH; ++i) s += acc[i][0] + acc[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int CH>
void launch(int32_t dtype, int32_t blocks, int32_t iters, float *out, hipStream_t st) {
    if (dtype == 0) hipLaunchKernelGGL(peak_f64<CH>, dim3(blocks), dim3(256), 0, st, out, iters);
    else if (dtype == 1) hipLaunchKernelGGL(peak_f32<CH>, dim3(blocks), dim3(256), 0, st, out, iters);
    else hipLaunchKernelGGL(peak_bf16<CH>, dim3(blocks), dim3(256), 0, st, out, iters);
}

// Waves 0-3 of each 512-thread workgroup run 8 chains of bf16 MFMAs, waves
// 4-7 chains of FP32 fused multiply-adds; with two workgroups per CU every
// SIMD holds matrix waves and vector waves.  ROLE 0 runs both kinds, 1 only
// the matrix waves, 2 only the vector waves (the others exit at once).
template <int ROLE>
__global__ __launch_bounds__(512) void overlap_kernel(float *out, int iters) {
    const bool matrix = (threadIdx.x >> 6) < 4;
    float s = 0;
    if (matrix && ROLE != 2) {
        bf8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(threadIdx.x * 1e-3f + e);
            b[e] = (__bf16)(e * 0.5f);
        }
        f4 acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = f4{0, 0, 0, 0};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][3];
    }
    if (!matrix && ROLE != 1) {
        float x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = threadIdx.x * 0.01f + j;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int j = 0; j < 16; ++j) x[j] = __builtin_fmaf(x[j], 0.999f, 0.25f);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) s += x[j];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int32_t mm_peak_overlap(int32_t role, int32_t blocks, int32_t iters, float *out, void *stream) {
    if (blocks < 1 || iters < 1 || !out || role < 0 || role > 2) return -1;
    hipStream_t st = (hipStream_t)stream;
    if (role == 0) hipLaunchKernelGGL(overlap_kernel<0>, dim3(blocks), dim3(512), 0, st, out, iters);
    else if (role == 1) hipLaunchKernelGGL(overlap_kernel<1>, dim3(blocks), dim3(512), 0, st, out, iters);
    else hipLaunchKernelGGL(overlap_kernel<2>, dim3(blocks), dim3(512), 0, st, out, iters);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

extern "C" int32_t mm_peak_mfma(int32_t dtype, int32_t chains, int32_t blocks, int32_t iters, float *out,
                                void *stream) {
    if (blocks < 1 || iters < 1 || !out || dtype < 0 || dtype > 2) return -1;
    if (chains != 8 && chains != 16 && chains != 32) return -1;
    hipStream_t st = (hipStream_t)stream;
    if (chains == 8) launch<8>(dtype, blocks, iters, out, st);
    else if (chains == 16) launch<16>(dtype, blocks, iters, out, st);
    else launch<32>(dtype, blocks, iters, out, st);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
