// C ABI of libmm: argument checks, error reporting and dispatch to the
// kernels.  Every export catches everything; no exception crosses the ABI.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mm_internal.h"

namespace mm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

mm_status fail(mm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

mm_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? MM_E_NOMEM : MM_E_DEVICE;
}

mm_status device_info(DeviceInfo *out) {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    MM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    DeviceInfo &d = cache[dev];
    if (!d.ok) {
        hipDeviceProp_t prop;
        MM_HIP(hipGetDeviceProperties(&prop, dev));
        d.device = dev;
        d.cus = prop.multiProcessorCount;
        d.arch = prop.gcnArchName;
        d.ok = true;
    }
    *out = d;
    return MM_OK;
}

void retain_default_pool() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(mu);
    for (int d : done)
        if (d == dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        // best effort: without it the pool only returns memory more eagerly
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    done.push_back(dev);
}

mm_status check_arch() {
    DeviceInfo d;
    mm_status s = device_info(&d);
    if (s != MM_OK) return s;
    retain_default_pool();
    if (d.arch.compare(0, 6, "gfx950") != 0)
        return fail(MM_E_UNSUPPORTED, "libmm kernels are built for gfx950; device is " + d.arch);
    return MM_OK;
}

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

// Bytes spanned by a rows x cols row-major matrix with leading dimension ld.
static size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t elem) {
    if (rows <= 0 || cols <= 0) return 0;
    return ((size_t)(rows - 1) * (size_t)ld + (size_t)cols) * elem;
}

// Largest dimension accepted, and the largest element offset a stored matrix
// may span: byte extents then fit in 64 bits for every element size.
constexpr int64_t kMaxDim = (int64_t)1 << 40;

static bool extent_overflows(int64_t rows, int64_t cols, int64_t ld) {
    if (rows <= 0 || cols <= 0) return false;
    return (__int128)(rows - 1) * ld + cols > ((__int128)1 << 62);
}

mm_status check_split_k(int64_t K) {
    if (K > kSplitMaxK) return fail(MM_E_UNSUPPORTED, "split methods take K <= 2^26 - 32");
    return MM_OK;
}

mm_status check_gemm_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                          int64_t ldb, const void *C, int64_t ldc, size_t ab_elem, size_t c_elem) {
    if (M < 0 || N < 0 || K < 0) return fail(MM_E_INVAL, "negative dimension");
    if (M > kMaxDim || N > kMaxDim || K > kMaxDim) return fail(MM_E_INVAL, "dimension too large");
    if (lda < (K > 1 ? K : 1)) return fail(MM_E_INVAL, "lda < max(K,1)");
    if (ldb < (N > 1 ? N : 1)) return fail(MM_E_INVAL, "ldb < max(N,1)");
    if (ldc < (N > 1 ? N : 1)) return fail(MM_E_INVAL, "ldc < max(N,1)");
    if (M == 0 || N == 0) return MM_OK;
    if (!C) return fail(MM_E_INVAL, "C is NULL");
    if (K > 0 && (!A || !B)) return fail(MM_E_INVAL, "A or B is NULL");
    if (extent_overflows(M, N, ldc) || extent_overflows(M, K, lda) || extent_overflows(K, N, ldb))
        return fail(MM_E_INVAL, "matrix extent overflows");
    const size_t cb = span_bytes(M, N, ldc, c_elem);
    if (K > 0 && (overlaps(C, cb, A, span_bytes(M, K, lda, ab_elem)) || overlaps(C, cb, B, span_bytes(K, N, ldb, ab_elem))))
        return fail(MM_E_INVAL, "C overlaps A or B");
    return MM_OK;
}

}  // namespace mm

using namespace mm;

#define MM_GUARD_BEGIN try {
#define MM_GUARD_END                                                        \
    }                                                                       \
    catch (const std::bad_alloc &) {                                        \
        return fail(MM_E_NOMEM, "host allocation failed");                  \
    }                                                                       \
    catch (const std::exception &ex) {                                      \
        return fail(MM_E_DEVICE, std::string("internal error: ") + ex.what()); \
    }                                                                       \
    catch (...) {                                                           \
        return fail(MM_E_DEVICE, "internal error");                         \
    }

extern "C" {

const char *mm_version(void) { return "libmm 0.1 gfx950"; }

const char *mm_status_string(mm_status s) {
    switch (s) {
        case MM_OK: return "ok";
        case MM_E_INVAL: return "invalid argument";
        case MM_E_NOMEM: return "out of memory";
        case MM_E_DEVICE: return "device error";
        case MM_E_BUSY: return "busy";
        case MM_E_UNSUPPORTED: return "unsupported";
        case MM_E_TIMEOUT: return "timeout";
    }
    return "unknown status";
}

const char *mm_last_error(void) { return g_last_error.c_str(); }

mm_status mm_init(int device) {
    MM_GUARD_BEGIN
    MM_HIP(hipSetDevice(device));
    mm_status s = check_arch();
    if (s != MM_OK) return s;
    // device address of the no-allocation entry point's scratch
    MM_HIP(residual_scratch_init());
    return MM_OK;
    MM_GUARD_END
}

mm_status mm_gemm_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double *C, int64_t ldc, void *stream) {
    MM_GUARD_BEGIN
    mm_status s = check_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, 8, 8);
    if (s != MM_OK || M == 0 || N == 0) return s;
    if ((s = check_arch()) != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (K == 0) MM_HIP(launch_fill_zero(C, M, N, ldc, 8, st));
    else MM_HIP(launch_gemm_f64(select_variant(MM_F64, M, N, K), M, N, K, A, lda, B, ldb, C, ldc, st));
    return MM_OK;
    MM_GUARD_END
}

mm_status mm_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B, int64_t ldb,
                      float *C, int64_t ldc, void *stream) {
    MM_GUARD_BEGIN
    mm_status s = check_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, 4, 4);
    if (s != MM_OK || M == 0 || N == 0) return s;
    if ((s = check_arch()) != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (K == 0) MM_HIP(launch_fill_zero(C, M, N, ldc, 4, st));
    else MM_HIP(launch_gemm_f32(variant_for_operands(MM_F32, select_variant(MM_F32, M, N, K),
                                                     direct_operands(A, lda, B, ldb, N, 4)),
                                M, N, K, A, lda, B, ldb, C, ldc, st));
    return MM_OK;
    MM_GUARD_END
}

mm_status mm_split_bf16(int64_t rows, int64_t cols, const float *X, int64_t ldx, int32_t nplanes, int32_t transpose,
                        uint16_t *planes, int64_t plane_stride, void *stream) {
    MM_GUARD_BEGIN
    if (rows < 0 || cols < 0) return fail(MM_E_INVAL, "negative dimension");
    if (rows > kMaxDim || cols > kMaxDim) return fail(MM_E_INVAL, "dimension too large");
    if (nplanes < 1 || nplanes > 3) return fail(MM_E_INVAL, "nplanes must be 1, 2 or 3");
    if (ldx < (cols > 1 ? cols : 1)) return fail(MM_E_INVAL, "ldx < max(cols,1)");
    if (rows == 0 || cols == 0) return MM_OK;
    if (!X || !planes) return fail(MM_E_INVAL, "NULL pointer");
    if (extent_overflows(rows, cols, ldx) || (__int128)rows * cols > ((__int128)1 << 60) ||
        plane_stride > ((int64_t)1 << 60))
        return fail(MM_E_INVAL, "matrix extent overflows");
    if (plane_stride < rows * cols) return fail(MM_E_INVAL, "plane_stride < rows*cols");
    if (overlaps(X, span_bytes(rows, cols, ldx, 4), planes, (size_t)plane_stride * nplanes * 2))
        return fail(MM_E_INVAL, "planes overlap X");
    mm_status s = check_arch();
    if (s != MM_OK) return s;
    MM_HIP(launch_split(rows, cols, X, ldx, nplanes, transpose, planes, plane_stride, transpose ? rows : cols, 0,
                        (hipStream_t)stream));
    return MM_OK;
    MM_GUARD_END
}

size_t mm_split_workspace_bytes(int64_t M, int64_t N, int64_t K, int32_t nprod) {
    if (M <= 0 || N <= 0 || K <= 0 || (nprod != 3 && nprod != 6)) return 0;
    return split_workspace_bytes(M, N, K, nprod);
}

// Runs the split method with an explicit tile variant.
static mm_status run_split(int variant, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                           const float *B, int64_t ldb, void *C, int64_t ldc, int32_t c_is_f64, int32_t nprod,
                           void *workspace, size_t workspace_bytes, hipStream_t st) {
    if (mm_status s = check_split_k(K); s != MM_OK) return s;
    if (K == 0) {
        MM_HIP(launch_fill_zero(C, M, N, ldc, c_is_f64 ? 8 : 4, st));
        return MM_OK;
    }
    // fused variants split inside the product and need no plane workspace
    const size_t need = split_variant_fused(variant) ? 0 : split_workspace_bytes(M, N, K, nprod);
    void *ws = workspace;
    bool owned = false;
    if (need && !ws) {
        MM_HIP(hipMallocAsync(&ws, need, st));
        owned = true;
    } else if (need && workspace_bytes < need) {
        return fail(MM_E_INVAL, "workspace too small");
    }
    hipError_t e = launch_split_product(variant, nprod, 0, 0, M, N, K, A, lda, B, ldb, C, ldc, c_is_f64, ws, st);
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "split GEMM launch");
    return MM_OK;
}

mm_status mm_gemm_split_bf16(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                             int64_t ldb, void *C, int64_t ldc, int32_t c_is_f64, int32_t nprod, void *workspace,
                             size_t workspace_bytes, void *stream) {
    MM_GUARD_BEGIN
    if (nprod != 3 && nprod != 6) return fail(MM_E_INVAL, "nprod must be 3 or 6");
    mm_status s = check_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, 4, c_is_f64 ? 8 : 4);
    if (s != MM_OK || M == 0 || N == 0) return s;
    if ((s = check_split_k(K)) != MM_OK || (s = check_arch()) != MM_OK) return s;
    const mm_method m = nprod == 3 ? MM_SPLIT_BF16_3 : MM_SPLIT_BF16_6;
    return run_split(select_variant(m, M, N, K), M, N, K, A, lda, B, ldb, C, ldc, c_is_f64, nprod, workspace,
                     workspace_bytes, (hipStream_t)stream);
    MM_GUARD_END
}

size_t mm_gemm_ex_workspace_bytes(mm_method method, mm_op opa, mm_op opb, int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (method == MM_SPLIT_BF16_3 || method == MM_SPLIT_BF16_6)
        return split_workspace_bytes(M, N, K, method == MM_SPLIT_BF16_3 ? 3 : 6);
    const size_t e = method == MM_F64 ? 8 : 4;
    size_t b = 0;
    if (opa == MM_OP_T) b += ((size_t)M * K * e + 255) & ~(size_t)255;
    if (opb == MM_OP_T) b += (size_t)K * N * e;
    return b;
}

mm_status mm_gemm_ex(mm_method method, mm_op opa, mm_op opb, int64_t M, int64_t N, int64_t K, const void *A,
                     int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, void *workspace,
                     size_t workspace_bytes, void *stream) {
    MM_GUARD_BEGIN
    if ((opa != MM_OP_N && opa != MM_OP_T) || (opb != MM_OP_N && opb != MM_OP_T))
        return fail(MM_E_INVAL, "op must be MM_OP_N or MM_OP_T");
    if (method < MM_F64 || method > MM_SPLIT_BF16_6) return fail(MM_E_INVAL, "unknown method");
    const size_t e = method == MM_F64 ? 8 : 4;
    if (M < 0 || N < 0 || K < 0) return fail(MM_E_INVAL, "negative dimension");
    if (M > kMaxDim || N > kMaxDim || K > kMaxDim) return fail(MM_E_INVAL, "dimension too large");
    // stored shapes: A is (M x K) or (K x M), B is (K x N) or (N x K)
    const int64_t ar = opa ? K : M, ac = opa ? M : K, br = opb ? N : K, bc = opb ? K : N;
    if (lda < (ac > 1 ? ac : 1)) return fail(MM_E_INVAL, "lda smaller than a stored row of A");
    if (ldb < (bc > 1 ? bc : 1)) return fail(MM_E_INVAL, "ldb smaller than a stored row of B");
    if (ldc < (N > 1 ? N : 1)) return fail(MM_E_INVAL, "ldc < max(N,1)");
    if (M == 0 || N == 0) return MM_OK;
    if (!C) return fail(MM_E_INVAL, "C is NULL");
    if (K > 0 && (!A || !B)) return fail(MM_E_INVAL, "A or B is NULL");
    if (extent_overflows(M, N, ldc) || extent_overflows(ar, ac, lda) || extent_overflows(br, bc, ldb))
        return fail(MM_E_INVAL, "matrix extent overflows");
    const size_t cb = span_bytes(M, N, ldc, e);
    if (K > 0 && (overlaps(C, cb, A, span_bytes(ar, ac, lda, e)) || overlaps(C, cb, B, span_bytes(br, bc, ldb, e))))
        return fail(MM_E_INVAL, "C overlaps A or B");
    mm_status s = method >= MM_SPLIT_BF16_3 ? check_split_k(K) : MM_OK;
    if (s != MM_OK || (s = check_arch()) != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (K == 0) {
        MM_HIP(launch_fill_zero(C, M, N, ldc, (int)e, st));
        return MM_OK;
    }
    const size_t need = mm_gemm_ex_workspace_bytes(method, opa, opb, M, N, K);
    void *ws = workspace;
    bool owned = false;
    if (need && !ws) {
        MM_HIP(hipMallocAsync(&ws, need, st));
        owned = true;
    } else if (need && workspace_bytes < need) {
        return fail(MM_E_INVAL, "workspace too small");
    }
    hipError_t err = hipSuccess;
    if (method == MM_SPLIT_BF16_3 || method == MM_SPLIT_BF16_6) {
        const int nprod = method == MM_SPLIT_BF16_3 ? 3 : 6;
        err = launch_split_product(select_variant(method, M, N, K), nprod, opa, opb, M, N, K, (const float *)A, lda,
                                   (const float *)B, ldb, C, ldc, 0, ws, st);
    } else {
        // transposed operands are brought to row-major op(X) in the workspace
        const void *a = A, *b = B;
        int64_t la = lda, lb = ldb;
        char *p = (char *)ws;
        if (opa == MM_OP_T) {
            err = launch_transpose(A, lda, K, M, p, K, (int)e, st);
            a = p;
            la = K;
            p += ((size_t)M * K * e + 255) & ~(size_t)255;
        }
        if (err == hipSuccess && opb == MM_OP_T) {
            err = launch_transpose(B, ldb, N, K, p, N, (int)e, st);
            b = p;
            lb = N;
        }
        if (err == hipSuccess) {
            const int v = variant_for_operands(method, select_variant(method, M, N, K),
                                               direct_operands(a, la, b, lb, N, (int64_t)e));
            err = method == MM_F64 ? launch_gemm_f64(v, M, N, K, (const double *)a, la, (const double *)b, lb,
                                                     (double *)C, ldc, st)
                                   : launch_gemm_f32(v, M, N, K, (const float *)a, la, (const float *)b, lb,
                                                     (float *)C, ldc, st);
        }
    }
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, st);
        if (err == hipSuccess) err = e2;
    }
    if (err != hipSuccess) return hip_fail(err, "mm_gemm_ex launch");
    return MM_OK;
    MM_GUARD_END
}

size_t mm_strassen_workspace_bytes(int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0 || K <= 0 || M % 2 || N % 2 || K % 2) return 0;
    return strassen_workspace_bytes(M, N, K);
}

mm_status mm_gemm_strassen_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
                               int64_t ldb, double *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                               void *stream) {
    MM_GUARD_BEGIN
    mm_status s = check_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, 8, 8);
    if (s != MM_OK || M == 0 || N == 0) return s;
    if (M % 2 || N % 2 || K % 2) return fail(MM_E_UNSUPPORTED, "one Strassen level needs even M, N, K");
    if ((s = check_arch()) != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (K == 0) {
        MM_HIP(launch_fill_zero(C, M, N, ldc, 8, st));
        return MM_OK;
    }
    const size_t need = strassen_workspace_bytes(M, N, K);
    void *ws = workspace;
    bool owned = false;
    if (!ws) {
        MM_HIP(hipMallocAsync(&ws, need, st));
        owned = true;
    } else if (workspace_bytes < need) {
        return fail(MM_E_INVAL, "workspace too small");
    }
    hipError_t e = launch_strassen_f64(M, N, K, A, lda, B, ldb, C, ldc, ws, st);
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "Strassen launch");
    return MM_OK;
    MM_GUARD_END
}

size_t mm_residual_workspace_bytes(int64_t M, int64_t N, int64_t K) {
    if (M < 0 || N < 0 || K < 0) return 0;
    return residual_workspace_bytes(M, N, K);
}

// Argument checks of the residual probe (both entry points).
static mm_status check_residual_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                                     int64_t ldb, const void *C, int64_t ldc, int32_t in_dtype, int32_t c_dtype,
                                     const double *x, const double *out) {
    if ((in_dtype != 0 && in_dtype != 1) || (c_dtype != 0 && c_dtype != 1))
        return fail(MM_E_INVAL, "dtype must be 0 (binary64) or 1 (FP32)");
    if (M < 0 || N < 0 || K < 0) return fail(MM_E_INVAL, "negative dimension");
    if (M > kMaxDim || N > kMaxDim || K > kMaxDim) return fail(MM_E_INVAL, "dimension too large");
    if (lda < (K > 1 ? K : 1) || ldb < (N > 1 ? N : 1) || ldc < (N > 1 ? N : 1))
        return fail(MM_E_INVAL, "leading dimension too small");
    if (extent_overflows(M, N, ldc) || extent_overflows(M, K, lda) || extent_overflows(K, N, ldb))
        return fail(MM_E_INVAL, "matrix extent overflows");
    if (!out) return fail(MM_E_INVAL, "out is NULL");
    if ((M > 0 && K > 0 && !A) || (K > 0 && N > 0 && !B) || (M > 0 && N > 0 && !C) || (N > 0 && !x))
        return fail(MM_E_INVAL, "NULL operand");
    return check_arch();
}

mm_status mm_residual_f64(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B, int64_t ldb,
                          const void *C, int64_t ldc, int32_t in_dtype, int32_t c_dtype, const double *x, double *out,
                          void *workspace, size_t workspace_bytes, void *stream) {
    MM_GUARD_BEGIN
    mm_status s = check_residual_args(M, N, K, A, lda, B, ldb, C, ldc, in_dtype, c_dtype, x, out);
    if (s != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const size_t need = residual_workspace_bytes(M, N, K);
    void *ws = workspace;
    bool owned = false;
    if (!ws) {
        MM_HIP(hipMallocAsync(&ws, need, st));
        owned = true;
    } else if (workspace_bytes < need) {
        return fail(MM_E_INVAL, "workspace too small");
    }
    hipError_t e = launch_residual(M, N, K, A, lda, B, ldb, C, ldc, in_dtype, c_dtype, x, out, ws, st);
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    return MM_OK;
    MM_GUARD_END
}

size_t mm_residual_noalloc_max_bytes(void) { return kResidualScratchDoubles * sizeof(double); }

mm_status mm_residual_f64_noalloc(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                                  int64_t ldb, const void *C, int64_t ldc, int32_t in_dtype, int32_t c_dtype,
                                  const double *x, double *out, void *stream) {
    MM_GUARD_BEGIN
    mm_status s = check_residual_args(M, N, K, A, lda, B, ldb, C, ldc, in_dtype, c_dtype, x, out);
    if (s != MM_OK) return s;
    if (residual_workspace_bytes(M, N, K) > kResidualScratchDoubles * sizeof(double))
        return fail(MM_E_INVAL, "residual scratch needs 8*(K + 2M + 512) bytes; the fixed scratch holds 2 MiB "
                                "(use mm_residual_f64 with a workspace for larger shapes)");
    void *ws = nullptr;
    MM_HIP(residual_scratch(&ws));
    MM_HIP(launch_residual(M, N, K, A, lda, B, ldb, C, ldc, in_dtype, c_dtype, x, out, ws, (hipStream_t)stream));
    return MM_OK;
    MM_GUARD_END
}

int32_t mm_variant_count(mm_method method) {
    switch (method) {
        case MM_F64: return f64_variant_count();
        case MM_F32: return f32_variant_count();
        case MM_SPLIT_BF16_3:
        case MM_SPLIT_BF16_6: return split_variant_count();
    }
    return 0;
}

mm_status mm_variant_info(mm_method method, int32_t variant, int32_t *bm, int32_t *bn, int32_t *bk) {
    if (variant < 0 || variant >= mm_variant_count(method)) return fail(MM_E_INVAL, "no such variant");
    TileCfg c = method == MM_F64 ? f64_variant(variant) : method == MM_F32 ? f32_variant(variant) : split_variant(variant);
    if (bm) *bm = c.bm;
    if (bn) *bn = c.bn;
    if (bk) *bk = c.bk;
    return MM_OK;
}

int32_t mm_select_variant(mm_method method, int64_t M, int64_t N, int64_t K) {
    return select_variant(method, M, N, K);
}

mm_status mm_gemm_variant(mm_method method, int32_t variant, int64_t M, int64_t N, int64_t K, const void *A,
                          int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, void *workspace,
                          size_t workspace_bytes, void *stream) {
    MM_GUARD_BEGIN
    if (variant < 0 || variant >= mm_variant_count(method)) return fail(MM_E_INVAL, "no such variant");
    const size_t e = method == MM_F64 ? 8 : 4;
    mm_status s = check_gemm_args(M, N, K, A, lda, B, ldb, C, ldc, e, e);
    if (s != MM_OK || M == 0 || N == 0) return s;
    if (method >= MM_SPLIT_BF16_3 && (s = check_split_k(K)) != MM_OK) return s;
    if ((s = check_arch()) != MM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    switch (method) {
        case MM_F64:
            if (K == 0) MM_HIP(launch_fill_zero(C, M, N, ldc, 8, st));
            else MM_HIP(launch_gemm_f64(variant, M, N, K, (const double *)A, lda, (const double *)B, ldb, (double *)C, ldc, st));
            return MM_OK;
        case MM_F32:
            if (K == 0) MM_HIP(launch_fill_zero(C, M, N, ldc, 4, st));
            else MM_HIP(launch_gemm_f32(variant, M, N, K, (const float *)A, lda, (const float *)B, ldb, (float *)C, ldc, st));
            return MM_OK;
        case MM_SPLIT_BF16_3:
        case MM_SPLIT_BF16_6:
            return run_split(variant, M, N, K, (const float *)A, lda, (const float *)B, ldb, C, ldc, 0,
                             method == MM_SPLIT_BF16_3 ? 3 : 6, workspace, workspace_bytes, st);
    }
    return fail(MM_E_INVAL, "unknown method");
    MM_GUARD_END
}

}  // extern "C"
