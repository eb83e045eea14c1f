// Split-precision product of FP32 matrices on the bfloat16 matrix cores.
//
// Split pass: an FP32 value x is written as bfloat16 planes, plane 0 = bf16(x)
// and each further plane = bf16 of what the previous planes leave over; the
// leftover is formed in FP32, where it is exact.  Conversions use the gfx950
// packed convert (round to nearest even).
//
// Split GEMM: the tile in split_tile.h over the planes, one workgroup per tile.
#include "mm_internal.h"
#include "gemm_tile.h"   // tile_order
#include "split_tile.h"
#include "variants.h"

namespace mm {


// ------------------------------------------------------------------ split pass
// Element offset of (row r, column c) of plane p: separate planes (plane p at
// p * plane_stride, rows of ldp), or interleaved (rows of nplanes * ldp; each
// 32-column block of plane 0, then the same block of plane 1 ...).  The 8
// columns c0 .. c0+7 (c0 a multiple of 8) are contiguous either way.
__device__ __forceinline__ int64_t plane_offset(int interleave, int nplanes, int64_t plane_stride, int64_t ldp, int p,
                                                int64_t r, int64_t c) {
    return interleave ? r * nplanes * ldp + (c >> 5) * (32 * nplanes) + p * 32 + (c & 31)
                      : p * plane_stride + r * ldp + c;
}

// Row-major planes with rows of ldp >= cols elements (columns cols..ldp-1
// written as zero): each thread splits 8 consecutive elements of one row,
// read as two 16-byte loads when they are all inside the row (the memory
// system runs in unaligned mode, so element alignment suffices) and written
// as one 16-byte store per plane.
__global__ void split_rows_kernel(const float *__restrict__ X, int64_t ldx, int64_t rows, int64_t cols, int nplanes,
                                  uint16_t *__restrict__ planes, int64_t plane_stride, int64_t ldp, int interleave) {
    const int64_t chunks_per_row = (ldp + 7) / 8;
    const int64_t total = rows * chunks_per_row;
    const bool vec_store = ldp % 8 == 0 && plane_stride % 8 == 0 && (uintptr_t)planes % 16 == 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / chunks_per_row;
        const int64_t c0 = (t % chunks_per_row) * 8;
        const gptr<const float> src = (gptr<const float>)(X + r * ldx + c0);
        float v[8];
        if (c0 + 8 <= cols) {
            const f32x4 lo = load_f32x4_ea(src), hi = load_f32x4_ea(src + 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = lo[e];
                v[4 + e] = hi[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (c0 + e < cols) ? src[e] : 0.f;
        }
        const int n = ldp - c0 < 8 ? (int)(ldp - c0) : 8;
        for (int p = 0; p < nplanes; ++p)
            split_store_chunk(v, (gptr<uint16_t>)(planes + plane_offset(interleave, nplanes, plane_stride, ldp, p, r, c0)),
                              n, vec_store);
    }
}

// Transposed planes (rows of X^T hold ldp >= rows elements, the tail written
// as zero): 64 x 64 tiles through LDS so that the FP32 reads run along rows of
// X and the bfloat16 writes along rows of X^T, 8 values (16 bytes) per thread
// and plane.
__global__ __launch_bounds__(256) void split_transpose_kernel(const float *__restrict__ X, int64_t ldx, int64_t rows,
                                                              int64_t cols, int nplanes, uint16_t *__restrict__ planes,
                                                              int64_t plane_stride, int64_t ldp, int interleave) {
    __shared__ float tile[64][65];
    const int64_t tiles_c = (cols + 63) / 64;
    const int64_t r0 = (blockIdx.x / tiles_c) * 64;
    const int64_t c0 = (blockIdx.x % tiles_c) * 64;
    // 16 threads read one 64-float row segment as 16-byte loads, 4 rows per
    // pass of the 256 threads
    const int cq = (threadIdx.x & 15) * 4, rq = threadIdx.x >> 4;
    for (int i = rq; i < 64; i += 16) {
        const int64_t r = r0 + i, c = c0 + cq;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (r < rows) {
            const gptr<const float> src = (gptr<const float>)(X + r * ldx + c);
            if (c + 4 <= cols) {
                const f32x4 q = load_f32x4_ea(src);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = q[e];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c + e < cols) v[e] = src[e];
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[i][cq + e] = v[e];
    }
    __syncthreads();
    const bool vec_store = ldp % 8 == 0 && plane_stride % 8 == 0 && (uintptr_t)planes % 16 == 0;
    // output row c of X^T, entries r .. r+7: 8 consecutive threads cover 64 r
    for (int k = threadIdx.x; k < 64 * 8; k += 256) {
        const int cl = k >> 3, rl = (k & 7) * 8;
        const int64_t c = c0 + cl, r = r0 + rl;
        if (c >= cols || r >= ldp) continue;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = tile[rl + e][cl];
        const int n = ldp - r < 8 ? (int)(ldp - r) : 8;
        for (int p = 0; p < nplanes; ++p)
            split_store_chunk(v, (gptr<uint16_t>)(planes + plane_offset(interleave, nplanes, plane_stride, ldp, p, c, r)),
                              n, vec_store);
    }
}

hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, int nplanes, int transpose,
                        uint16_t *planes, int64_t plane_stride, int64_t ldp, int interleave, hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (interleave && ldp % 32 != 0) return hipErrorInvalidValue;
    if (transpose) {
        // 64-row tiles cover ldp: ldp <= round_up(rows, 64)
        const int64_t blocks = ((rows + 63) / 64) * ((cols + 63) / 64);
        if (blocks > 0x7fffffffLL || ldp < rows || ldp > (rows + 63) / 64 * 64) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(split_transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, ldx, rows, cols,
                           nplanes, planes, plane_stride, ldp, interleave);
    } else {
        if (ldp < cols) return hipErrorInvalidConfiguration;
        int64_t blocks = (rows * ((ldp + 7) / 8) + 255) / 256;
        if (blocks > 1 << 20) blocks = 1 << 20;
        hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, ldx, rows, cols,
                           nplanes, planes, plane_stride, ldp, interleave);
    }
    return hipGetLastError();
}

int64_t split_padded_k(int64_t K) { return (K + 31) / 32 * 32; }

hipError_t launch_split_product(int variant, int nprod, int opa, int opb, int64_t M, int64_t N, int64_t K,
                                const float *A, int64_t lda, const float *B, int64_t ldb, void *C, int64_t ldc,
                                int c_is_f64, void *ws, hipStream_t st) {
    if (split_variant_fused(variant)) {
        // the fused tile reads row-major FP32 operands; transposed ones take
        // the plane pass (which transposes) and a plane-reading tile
        if (!opa && !opb) return launch_split_fused(variant, nprod, M, N, K, A, lda, B, ldb, C, ldc, c_is_f64, st);
        variant = default_unfused_split_variant(nprod == 3 ? MM_SPLIT_BF16_3 : MM_SPLIT_BF16_6, M, N, K);
    }
    const int np = nprod == 3 ? 2 : 3;
    const int64_t Kp = split_padded_k(K);
    const int il = split_planes_interleaved(variant, nprod);
    uint16_t *Ap = (uint16_t *)ws;
    uint16_t *Bt = (uint16_t *)((char *)ws + split_b_offset_bytes(M, K, nprod));
    // A planes are M x Kp: rows of A as stored (N), or the transpose of K x M (T)
    hipError_t e = opa ? launch_split(K, M, A, lda, np, 1, Ap, M * Kp, Kp, il, st)
                       : launch_split(M, K, A, lda, np, 0, Ap, M * Kp, Kp, il, st);
    // B planes are N x Kp: the transpose of K x N (N), or rows of B as stored (T)
    if (e == hipSuccess)
        e = opb ? launch_split(N, K, B, ldb, np, 0, Bt, N * Kp, Kp, il, st)
                : launch_split(K, N, B, ldb, np, 1, Bt, N * Kp, Kp, il, st);
    if (e == hipSuccess) e = launch_gemm_split(variant, nprod, M, N, Kp, Ap, Bt, C, ldc, c_is_f64, st);
    return e;
}

// Planes of the product use rows of split_padded_k(K) elements (zero tail):
// every 8-element fragment is one aligned 16-byte access and every 32-wide K
// step is whole.
size_t split_b_offset_bytes(int64_t M, int64_t K, int nprod) {
    const int np = nprod == 3 ? 2 : 3;
    // B planes start 256-byte aligned behind the A planes
    return ((size_t)np * M * split_padded_k(K) * 2 + 255) & ~(size_t)255;
}

size_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int nprod) {
    const int np = nprod == 3 ? 2 : 3;
    return split_b_offset_bytes(M, K, nprod) + (size_t)np * N * split_padded_k(K) * 2;
}


template <typename ST>
__global__ __launch_bounds__(ST::NT, (ST::NWAVES >= 8 ? 2 : 1)) void split_gemm_kernel(const uint16_t *__restrict__ Ap, int64_t pa_stride,
                                                            const uint16_t *__restrict__ Bt, int64_t pb_stride,
                                                            void *C, int64_t ldc, int c_is_f64, int64_t M, int64_t N,
                                                            int64_t K, int64_t tiles_m, int64_t tiles_n, int group_m,
                                                            int vec_ok) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[ST::LDS_ELEMS];
    int64_t tm, tn;
    tile_order(blockIdx.x, tiles_m, tiles_n, group_m, &tm, &tn);
    ST::run(Ap, pa_stride, Bt, pb_stride, C, ldc, c_is_f64, M, N, K, tm, tn, vec_ok != 0, smem);
}

template <typename ST>
__global__ __launch_bounds__(ST::NT, SplitWaves<ST>::value) void split_fused_kernel(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ B, int64_t ldb, void *C, int64_t ldc,
    int c_is_f64, int64_t M, int64_t N, int64_t K, int64_t tiles_m, int64_t tiles_n, int group_m) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[ST::LDS_ELEMS];
    int64_t tm, tn;
    tile_order(blockIdx.x, tiles_m, tiles_n, group_m, &tm, &tn);
    ST::run_fused(A, lda, B, ldb, C, ldc, c_is_f64, M, N, K, tm, tn, smem);
}

template <typename ST>
static hipError_t launch_fused_tile(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                                    int64_t ldb, void *C, int64_t ldc, int c_is_f64, hipStream_t stream) {
    if constexpr (!ST::FUSED) {
        return hipErrorInvalidValue;
    } else {
        const int64_t tiles_m = (M + ST::BM - 1) / ST::BM;
        const int64_t tiles_n = (N + ST::BN - 1) / ST::BN;
        const int64_t blocks = tiles_m * tiles_n;
        if (blocks <= 0) return hipSuccess;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        static const int group = tile_group_rows((const void *)&split_fused_kernel<ST>, ST::NT, ST::BM, ST::BN);
        hipLaunchKernelGGL((split_fused_kernel<ST>), dim3((unsigned)blocks), dim3(ST::NT), 0, stream, A, lda, B, ldb,
                           C, ldc, c_is_f64, M, N, K, tiles_m, tiles_n, group);
        return hipGetLastError();
    }
}

template <typename ST>
static hipError_t launch_split_tile(int64_t M, int64_t N, int64_t K, const uint16_t *Ap, const uint16_t *Bt, void *C,
                                    int64_t ldc, int c_is_f64, hipStream_t stream) {
    if constexpr (ST::FUSED) {
        return hipErrorInvalidValue;   // fused tiles take FP32 operands
    } else {
        const int64_t tiles_m = (M + ST::BM - 1) / ST::BM;
        const int64_t tiles_n = (N + ST::BN - 1) / ST::BN;
        const int64_t blocks = tiles_m * tiles_n;
        if (blocks <= 0) return hipSuccess;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        const int vec_ok = (K % 8 == 0) && ((uintptr_t)Ap % 16 == 0) && ((uintptr_t)Bt % 16 == 0);
        static const int group = tile_group_rows((const void *)&split_gemm_kernel<ST>, ST::NT, ST::BM, ST::BN);
        hipLaunchKernelGGL((split_gemm_kernel<ST>), dim3((unsigned)blocks), dim3(ST::NT), 0, stream, Ap, M * K, Bt,
                           N * K, C, ldc, c_is_f64, M, N, K, tiles_m, tiles_n, group, vec_ok);
        return hipGetLastError();
    }
}

#define MM_S_FUSED(id, bm, bn, bk, wm, wn, st) case id: return (st) >= 20;
bool split_variant_fused(int v) {
    switch (v) { MM_SPLIT_VARIANTS(MM_S_FUSED) default: return false; }
}

#define MM_S_DIRECT(id, bm, bn, bk, wm, wn, st) case id: return (st) >= 10 && (st) < 20;
bool split_planes_interleaved(int v, int nprod) {
    if (nprod != 3) return false;
    switch (v) { MM_SPLIT_VARIANTS(MM_S_DIRECT) default: return false; }
}

#define MM_S_FLAUNCH(id, bm, bn, bk, wm, wn, st)                                                                  \
    case id:                                                                                                       \
        return nprod == 3 ? launch_fused_tile<SplitTileSel<3, bm, bn, bk, wm, wn, st>::type>(M, N, K, A, lda, B,     \
                                                                                             ldb, C, ldc, c_is_f64,  \
                                                                                             stream)                 \
                          : launch_fused_tile<SplitTileSel<6, bm, bn, bk, wm, wn, st>::type>(M, N, K, A, lda, B,     \
                                                                                             ldb, C, ldc, c_is_f64,  \
                                                                                             stream);

hipError_t launch_split_fused(int variant, int nprod, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                              const float *B, int64_t ldb, void *C, int64_t ldc, int c_is_f64, hipStream_t stream) {
    switch (variant) {
        MM_SPLIT_VARIANTS(MM_S_FLAUNCH)
        default: return hipErrorInvalidValue;
    }
}

#define MM_S_COUNT(id, bm, bn, bk, wm, wn, st) +1
#define MM_S_CFG(id, bm, bn, bk, wm, wn, st) case id: return TileCfg{bm, bn, bk};
int split_variant_count() { return 0 MM_SPLIT_VARIANTS(MM_S_COUNT); }
TileCfg split_variant(int v) {
    switch (v) { MM_SPLIT_VARIANTS(MM_S_CFG) default: return TileCfg{0, 0, 0}; }
}

#define MM_S_LAUNCH(id, bm, bn, bk, wm, wn, st)                                                                   \
    case id:                                                                                                       \
        return nprod == 3                                                                                          \
                   ? launch_split_tile<SplitTileSel<3, bm, bn, bk, wm, wn, st, true>::type>(M, N, K, Ap, Bt, C, ldc, \
                                                                                       c_is_f64, stream)            \
                   : launch_split_tile<SplitTileSel<6, bm, bn, bk, wm, wn, st>::type>(M, N, K, Ap, Bt, C, ldc,       \
                                                                                       c_is_f64, stream);

hipError_t launch_gemm_split(int variant, int nprod, int64_t M, int64_t N, int64_t K, const uint16_t *Ap,
                             const uint16_t *Bt, void *C, int64_t ldc, int c_is_f64, hipStream_t stream) {
    switch (variant) {
        MM_SPLIT_VARIANTS(MM_S_LAUNCH)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mm
