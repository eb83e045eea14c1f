// Residual probe of a computed product (Freivalds): for a probe vector x,
// y = B.x, z = A.y, w = C.x, r = w - z, all in binary64, reduced to
// ||r||^2 and ||z||^2 in a fixed order (deterministic, no atomics).
#include <mutex>
#include <vector>

#include "mm_internal.h"

namespace mm {

static constexpr int kPartials = 256;

// out[i] = sum_j X[i][j] * v[j] for i < rows; one wave per row, lanes stride
// the row so loads are coalesced, then a fixed shuffle-tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void rowdot_kernel(const T *__restrict__ X, int64_t ldx, int64_t rows, int64_t cols,
                                                     const double *__restrict__ v, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t i = wave; i < rows; i += nwaves) {
        const T *row = X + i * ldx;
        double s = 0.0;
        for (int64_t j = lane; j < cols; j += 64) s += (double)row[j] * v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) out[i] = s;
    }
}

// partials[b] = (sum (w-z)^2, sum z^2) over a fixed grid-stride subset.
__global__ __launch_bounds__(256) void residual_partials_kernel(const double *__restrict__ w,
                                                                const double *__restrict__ z, int64_t m,
                                                                double *__restrict__ partials) {
    __shared__ double sr[256], sz[256];
    double r2 = 0.0, z2 = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)kPartials * 256) {
        const double d = w[i] - z[i];
        r2 += d * d;
        z2 += z[i] * z[i];
    }
    sr[threadIdx.x] = r2;
    sz[threadIdx.x] = z2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            sz[threadIdx.x] += sz[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sr[0];
        partials[2 * blockIdx.x + 1] = sz[0];
    }
}

__global__ __launch_bounds__(256) void residual_final_kernel(const double *__restrict__ partials,
                                                             double *__restrict__ out) {
    __shared__ double sr[256], sz[256];
    sr[threadIdx.x] = partials[2 * threadIdx.x];
    sz[threadIdx.x] = partials[2 * threadIdx.x + 1];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            sz[threadIdx.x] += sz[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sr[0];
        out[1] = sz[0];
    }
}

__global__ void zero_vec_kernel(double *v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 0.0;
}

size_t residual_workspace_bytes(int64_t M, int64_t N, int64_t K) {
    (void)N;
    return sizeof(double) * ((size_t)K + 2 * (size_t)M + 2 * kPartials);
}

template <typename T>
static void rowdot(const void *X, int64_t ldx, int64_t rows, int64_t cols, const double *v, double *out,
                   hipStream_t st) {
    if (rows <= 0) return;
    if (cols <= 0) {
        hipLaunchKernelGGL(zero_vec_kernel, dim3(64), dim3(256), 0, st, out, rows);
        return;
    }
    int64_t blocks = (rows + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((rowdot_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, (const T *)X, ldx, rows, cols,
                       v, out);
}

hipError_t launch_residual(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B, int64_t ldb,
                           const void *C, int64_t ldc, int in_dtype, int c_dtype, const double *x, double *out,
                           void *ws, hipStream_t st) {
    double *y = (double *)ws;
    double *z = y + K;
    double *w = z + M;
    double *partials = w + M;
    if (in_dtype == 0) {
        rowdot<double>(B, ldb, K, N, x, y, st);
        rowdot<double>(A, lda, M, K, y, z, st);
    } else {
        rowdot<float>(B, ldb, K, N, x, y, st);
        rowdot<float>(A, lda, M, K, y, z, st);
    }
    if (c_dtype == 0) rowdot<double>(C, ldc, M, N, x, w, st);
    else rowdot<float>(C, ldc, M, N, x, w, st);
    hipLaunchKernelGGL(residual_partials_kernel, dim3(kPartials), dim3(256), 0, st, w, z, M, partials);
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, st, partials, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ no-allocation form
// Fixed device scratch for mm_residual_f64_noalloc: y, z, w and the partial
// sums live here instead of in a caller workspace or a stream-ordered
// allocation.  Each device holds its own copy of the array (at its own
// address) for the life of the process.  The host must never use the array's
// name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept.
static __device__ __align__(256) double scratch[kResidualScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // index: device ordinal; nullptr until looked up
}  // namespace

hipError_t residual_scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
    return hipSuccess;
}

hipError_t residual_scratch(void **ptr) {
    hipError_t e = residual_scratch_init();
    if (e != hipSuccess) return e;
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace mm
