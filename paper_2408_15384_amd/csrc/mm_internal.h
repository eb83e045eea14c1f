// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include "../../include/mm.h"

namespace mm {

// Thread-local error text behind mm_last_error().
void set_error(const std::string &msg);
mm_status fail(mm_status s, const std::string &msg);
mm_status hip_fail(hipError_t e, const char *what);

#define MM_HIP(call)                                                   \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ::mm::hip_fail(_e, #call);        \
    } while (0)

// Per-device facts, filled once.
struct DeviceInfo {
    int device = -1;
    int cus = 0;
    std::string arch;
    bool ok = false;
};
mm_status device_info(DeviceInfo *out);

// ---------------------------------------------------------------- kernels
// Tile variants of the dense MFMA kernels.  Variant ids index these tables.
struct TileCfg { int bm, bn, bk; };

int f64_variant_count();
TileCfg f64_variant(int v);
int f32_variant_count();
TileCfg f32_variant(int v);
int split_variant_count();
TileCfg split_variant(int v);

// Plain MFMA GEMM (row-major NN), launches on `stream`.
hipError_t launch_gemm_f64(int variant, int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t stream);
hipError_t launch_gemm_f32(int variant, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                           const float *B, int64_t ldb, float *C, int64_t ldc, hipStream_t stream);

// Split pass: FP32 -> nplanes bfloat16 planes (optionally transposed).
hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, int nplanes, int transpose,
                        uint16_t *planes, int64_t plane_stride, hipStream_t stream);

// Split GEMM on planes: A planes M x K row-major (stride M*K), B planes stored
// transposed N x K (stride N*K); C FP32 or binary64.
hipError_t launch_gemm_split(int variant, int nprod, int64_t M, int64_t N, int64_t K, const uint16_t *Ap,
                             const uint16_t *Bt, void *C, int64_t ldc, int c_is_f64, hipStream_t stream);

size_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int nprod);
// Byte offset of the B planes inside the split workspace.
size_t split_b_offset_bytes(int64_t M, int64_t K, int nprod);

// Residual probe.
size_t residual_workspace_bytes(int64_t M, int64_t N, int64_t K);
hipError_t launch_residual(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                           int64_t ldb, const void *C, int64_t ldc, int in_dtype, int c_dtype, const double *x,
                           double *out, void *ws, hipStream_t stream);

// Zero-fill of an M x N matrix (K == 0 products).
hipError_t launch_fill_zero(void *C, int64_t M, int64_t N, int64_t ldc, int elem_bytes, hipStream_t stream);

// ---------------------------------------------------------------- grouped
// Device descriptor of one grouped problem.
struct GroupedDesc {
    int64_t M, N, K;
    const void *A; int64_t lda;
    const void *B; int64_t ldb;
    void *C; int64_t ldc;
    int64_t tile_begin;   // exclusive prefix sum of tile counts
    int32_t tiles_n;      // tiles along N
    int32_t pad;
};

hipError_t launch_grouped(mm_method method, int variant, const GroupedDesc *descs, int32_t count,
                          int64_t total_tiles, int grid, hipStream_t stream);
int grouped_tile_bm(mm_method method, int variant);
int grouped_tile_bn(mm_method method, int variant);

// Autotune cache lookup (pure function of key + loaded cache).
int select_variant(mm_method method, int64_t M, int64_t N, int64_t K);

}  // namespace mm
