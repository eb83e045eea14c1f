/*
 * Reference CPU implementation of the dense product C = A.B.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU library.
 *
 * Definition followed (paper section III, the displayed sum): for an m x n
 * matrix A and an n x p matrix B, every entry of the m x p result is the
 * dot product of row i of A with column j of B,
 *     C[i][j] = sum over k of A[i][k] * B[k][j].
 * Storage is row-major as in C (section III, storage remark) with explicit
 * leading dimensions; indices are 0-based here where the paper's are 1-based.
 * The sum is the paper's plain loop (section VI), with OpenMP threads over
 * rows i (section III-A-1); orc_gemm walks it in i, k, j order, which leaves
 * every entry's sequence of operations unchanged (see there).
 *
 * Arithmetic is IEEE binary64.  Each entry starts from +0.0 and adds the
 * products in ascending k, each product and each sum rounded once (this file
 * must be compiled with -ffp-contract=off so no fused multiply-add is formed).
 * Rows are independent, so the result is bit-identical at any thread count.
 */
#include <stdint.h>
#include <omp.h>

static int orc_threads = 0; /* 0: OpenMP default */

void orc_set_threads(int n) { orc_threads = n; }

int orc_get_threads(void)
{
    return orc_threads > 0 ? orc_threads : omp_get_max_threads();
}

/* C (M x N, ldc) = A (M x K, lda) . B (K x N, ldb); all row-major binary64.
 *
 * The loops run i, k, j rather than the paper's i, j, k: row i of C is the
 * accumulator and each step k adds A[i][k] * B[k][j] to every entry j of it.
 * Every entry still receives exactly the operations of the plain loop --
 * start at +0.0, then for k = 0, 1, ..., K-1 one rounded product and one
 * rounded sum -- so the bits are those of the i, j, k order; only the walk
 * over memory changes (B is read along its rows instead of down a column).
 * C must not overlap A or B. */
void orc_gemm(int64_t M, int64_t N, int64_t K,
              const double *restrict A, int64_t lda,
              const double *restrict B, int64_t ldb,
              double *restrict C, int64_t ldc)
{
    int nt = orc_get_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t i = 0; i < M; ++i) {
        double *restrict c = C + i * ldc;
        for (int64_t j = 0; j < N; ++j)
            c[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double a = A[i * lda + k];
            const double *restrict b = B + k * ldb;
            for (int64_t j = 0; j < N; ++j)
                c[j] = c[j] + a * b[j];
        }
    }
}

/* The same definition evaluated only at the n listed (rows[t], cols[t])
 * positions: out[t] = C[rows[t]][cols[t]].  Used to check single entries of
 * products too large for the full loop. */
void orc_gemm_entries(int64_t K,
                      const double *A, int64_t lda,
                      const double *B, int64_t ldb,
                      int64_t n, const int64_t *rows, const int64_t *cols,
                      double *out)
{
    int nt = orc_get_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t t = 0; t < n; ++t) {
        const double *a = A + rows[t] * lda;
        const double *b = B + cols[t];
        double s = 0.0;
        for (int64_t k = 0; k < K; ++k)
            s = s + a[k] * b[k * ldb];
        out[t] = s;
    }
}
