// One level of Strassen's scheme in Winograd's form on the binary64 MFMA
// GEMM: with A, B in 2 x 2 quadrants (M, N, K even),
//   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2
//   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
//   P6 = S2 T2, P7 = S3 T3
//   C11 = P1 + P2, C12 = ((P1 + P6) + P5) + P3, C21 = ((P1 + P6) + P7) - P4,
//   C22 = ((P1 + P6) + P7) + P5
// Seven half-size products (7/8 of the multiplications) plus three
// elementwise passes: S1..S4 in one pass over A, T1..T4 in one pass over B,
// the four quadrants of C in one pass over P1..P7.
#include "mm_internal.h"

namespace mm {

__global__ void strassen_pre_a(const double *__restrict__ A, int64_t lda, int64_t m, int64_t k,
                               double *__restrict__ S) {
    const int64_t total = m * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, c = i % k;
        const double a11 = A[r * lda + c], a12 = A[r * lda + k + c];
        const double a21 = A[(m + r) * lda + c], a22 = A[(m + r) * lda + k + c];
        const double s1 = a21 + a22;
        const double s2 = s1 - a11;
        S[i] = s1;
        S[total + i] = s2;
        S[2 * total + i] = a11 - a21;
        S[3 * total + i] = a12 - s2;
    }
}

__global__ void strassen_pre_b(const double *__restrict__ B, int64_t ldb, int64_t k, int64_t n,
                               double *__restrict__ T) {
    const int64_t total = k * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / n, c = i % n;
        const double b11 = B[r * ldb + c], b12 = B[r * ldb + n + c];
        const double b21 = B[(k + r) * ldb + c], b22 = B[(k + r) * ldb + n + c];
        const double t1 = b12 - b11;
        const double t2 = b22 - t1;
        T[i] = t1;
        T[total + i] = t2;
        T[2 * total + i] = b22 - b12;
        T[3 * total + i] = t2 - b21;
    }
}

__global__ void strassen_post(const double *__restrict__ P, int64_t m, int64_t n, double *__restrict__ C,
                              int64_t ldc) {
    const int64_t total = m * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / n, c = i % n;
        const double p1 = P[i], p2 = P[total + i], p3 = P[2 * total + i], p4 = P[3 * total + i];
        const double p5 = P[4 * total + i], p6 = P[5 * total + i], p7 = P[6 * total + i];
        const double u2 = p1 + p6;
        const double u3 = u2 + p7;
        const double u4 = u2 + p5;
        C[r * ldc + c] = p1 + p2;
        C[r * ldc + n + c] = u4 + p3;
        C[(m + r) * ldc + c] = u3 - p4;
        C[(m + r) * ldc + n + c] = u3 + p5;
    }
}

size_t strassen_workspace_bytes(int64_t M, int64_t N, int64_t K) {
    const int64_t m = M / 2, n = N / 2, k = K / 2;
    return sizeof(double) * (size_t)(4 * m * k + 4 * k * n + 7 * m * n);
}

static unsigned grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

hipError_t launch_strassen_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
                               int64_t ldb, double *C, int64_t ldc, void *ws, hipStream_t st) {
    const int64_t m = M / 2, n = N / 2, k = K / 2;
    double *S = (double *)ws;
    double *T = S + 4 * m * k;
    double *P = T + 4 * k * n;
    hipLaunchKernelGGL(strassen_pre_a, dim3(grid_for(m * k)), dim3(256), 0, st, A, lda, m, k, S);
    hipLaunchKernelGGL(strassen_pre_b, dim3(grid_for(k * n)), dim3(256), 0, st, B, ldb, k, n, T);
    hipError_t e = hipGetLastError();
    const int v = select_variant(MM_F64, m, n, k);
    const double *S1 = S, *S2 = S + m * k, *S3 = S + 2 * m * k, *S4 = S + 3 * m * k;
    const double *T1 = T, *T2 = T + k * n, *T3 = T + 2 * k * n, *T4 = T + 3 * k * n;
    const double *A11 = A, *A12 = A + k, *A22 = A + m * lda + k;
    const double *B11 = B, *B21 = B + k * ldb, *B22 = B + k * ldb + n;
    struct { const double *x; int64_t ldx; const double *y; int64_t ldy; } prod[7] = {
        {A11, lda, B11, ldb}, {A12, lda, B21, ldb}, {S4, k, B22, ldb}, {A22, lda, T4, n},
        {S1, k, T1, n},       {S2, k, T2, n},       {S3, k, T3, n}};
    for (int i = 0; i < 7 && e == hipSuccess; ++i)
        e = launch_gemm_f64(v, m, n, k, prod[i].x, prod[i].ldx, prod[i].y, prod[i].ldy, P + i * m * n, n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(strassen_post, dim3(grid_for(m * n)), dim3(256), 0, st, P, m, n, C, ldc);
    return hipGetLastError();
}

}  // namespace mm
