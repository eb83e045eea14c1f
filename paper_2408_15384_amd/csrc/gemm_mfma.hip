// Single-problem binary64 and FP32 GEMM kernels built from the workgroup tile
// in gemm_tile.h, with their tile variants.
#include "mm_internal.h"
#include "gemm_tile.h"
#include "variants.h"

namespace mm {

template <typename TG, typename T>
__global__ __launch_bounds__(TG::NT, (TG::NWAVES <= 4 ? 2 : 1)) void gemm_kernel(const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                                      int64_t ldb, T *__restrict__ C, int64_t ldc, int64_t M,
                                                      int64_t N, int64_t K, int64_t tiles_m, int64_t tiles_n,
                                                      int group_m, int vec_ok) {
    __shared__ __attribute__((aligned(16))) T smem[TG::LDS_ELEMS];
    int64_t tm, tn;
    tile_order(blockIdx.x, tiles_m, tiles_n, group_m, &tm, &tn);
    TG::run(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, vec_ok != 0, smem);
}

template <typename TG, typename T>
static hipError_t launch_tile(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B, int64_t ldb,
                              T *C, int64_t ldc, hipStream_t stream) {
    const int64_t tiles_m = (M + TG::BM - 1) / TG::BM;
    const int64_t tiles_n = (N + TG::BN - 1) / TG::BN;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const int vec = TG::VEC;
    const int vec_ok = (lda % vec == 0) && (ldb % vec == 0) && ((uintptr_t)A % 16 == 0) &&
                       ((uintptr_t)B % 16 == 0);
    static const int group = tile_group_rows((const void *)&gemm_kernel<TG, T>, TG::NT, TG::BM, TG::BN);
    hipLaunchKernelGGL((gemm_kernel<TG, T>), dim3((unsigned)blocks), dim3(TG::NT), 0, stream, A, lda, B, ldb, C,
                       ldc, M, N, K, tiles_m, tiles_n, group, vec_ok);
    return hipGetLastError();
}

// ---------------------------------------------------------------- variants
#define MM_COUNT(id, bm, bn, bk, wm, wn, st) +1
#define MM_CFG(id, bm, bn, bk, wm, wn, st) case id: return TileCfg{bm, bn, bk};

int f64_variant_count() { return 0 MM_F64_VARIANTS(MM_COUNT); }
int f32_variant_count() { return 0 MM_F32_VARIANTS(MM_COUNT); }
TileCfg f64_variant(int v) {
    switch (v) { MM_F64_VARIANTS(MM_CFG) default: return TileCfg{0, 0, 0}; }
}
TileCfg f32_variant(int v) {
    switch (v) { MM_F32_VARIANTS(MM_CFG) default: return TileCfg{0, 0, 0}; }
}

#define MM_LAUNCH_F64(id, bm, bn, bk, wm, wn, st) \
    case id: return launch_tile<TileSel<double, bm, bn, bk, wm, wn, st>::type, double>(M, N, K, A, lda, B, ldb, C, ldc, stream);
#define MM_LAUNCH_F32(id, bm, bn, bk, wm, wn, st) \
    case id: return launch_tile<TileSel<float, bm, bn, bk, wm, wn, st>::type, float>(M, N, K, A, lda, B, ldb, C, ldc, stream);

hipError_t launch_gemm_f64(int variant, int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t stream) {
    switch (variant) {
        MM_F64_VARIANTS(MM_LAUNCH_F64)
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_f32(int variant, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                           const float *B, int64_t ldb, float *C, int64_t ldc, hipStream_t stream) {
    switch (variant) {
        MM_F32_VARIANTS(MM_LAUNCH_F32)
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- transpose
// 64 x 64 tiles through LDS: reads along rows of X, writes along rows of X^T.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ X, int64_t ldx, int64_t rows,
                                                        int64_t cols, T *__restrict__ Y, int64_t ldy) {
    __shared__ T tile[64][65];
    const int64_t tiles_c = (cols + 63) / 64;
    const int64_t r0 = (blockIdx.x / tiles_c) * 64, c0 = (blockIdx.x % tiles_c) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = X[r * ldx + c];
    }
    __syncthreads();
    for (int j = ty; j < 64; j += 4) {
        const int64_t c = c0 + j, r = r0 + tx;
        if (c < cols && r < rows) Y[c * ldy + r] = tile[tx][j];
    }
}

hipError_t launch_transpose(const void *X, int64_t ldx, int64_t rows, int64_t cols, void *Y, int64_t ldy,
                            int elem_bytes, hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t blocks = ((rows + 63) / 64) * ((cols + 63) / 64);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(transpose_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, (const double *)X,
                           ldx, rows, cols, (double *)Y, ldy);
    else
        hipLaunchKernelGGL(transpose_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, (const float *)X,
                           ldx, rows, cols, (float *)Y, ldy);
    return hipGetLastError();
}

// ---------------------------------------------------------------- zero fill
// C := 0 for K == 0 (the empty sum).  A kernel rather than a memset so the
// call can sit inside a captured graph.
template <typename T>
__global__ void fill_zero_kernel(T *C, int64_t M, int64_t N, int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / N, c = i % N;
        C[r * ldc + c] = T(0);
    }
}

hipError_t launch_fill_zero(void *C, int64_t M, int64_t N, int64_t ldc, int elem_bytes, hipStream_t stream) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int64_t blocks = (M * N + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(fill_zero_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, (double *)C, M,
                           N, ldc);
    else
        hipLaunchKernelGGL(fill_zero_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, (float *)C, M, N,
                           ldc);
    return hipGetLastError();
}

}  // namespace mm
