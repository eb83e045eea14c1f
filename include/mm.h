/*
 * mm.h -- C ABI of libmm, dense matrix multiplication C = A.B on MI355X (gfx950).
 *
 * The operation is the textbook product of the paper's section III: for an
 * M x K matrix A and a K x N matrix B (the paper's m x n and n x p), every
 * entry of the M x N result is the dot product of a row of A with a column of
 * B, C[i][j] = sum_k A[i][k] * B[k][j].  Storage is row-major, as in C (the
 * storage remark of section III): element (r, c) of a matrix with leading
 * dimension ld sits at base[r * ld + c].  There is no alpha/beta: C is
 * overwritten with A.B.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Pointers named A, B, C, X, workspace are DEVICE pointers (memory of the
 *    current HIP device, e.g. from hipMalloc or a torch CUDA tensor).  Pointers
 *    to descriptors, configs and outputs such as id_out are HOST pointers
 *    unless stated otherwise.
 *  * Ownership: the caller owns every buffer it passes and must keep it alive
 *    until the enqueued work has finished.  The library never frees caller
 *    memory.  Objects the library creates (plans, servers) are released only by
 *    their *_destroy call.
 *  * Streams: `stream` is a hipStream_t passed as void*; NULL means the legacy
 *    default stream.  GEMM calls only enqueue work and return at once; device
 *    faults surface at the next synchronising call.
 *  * Errors: argument checks are synchronous and return a negative mm_status
 *    without enqueueing anything; mm_last_error() then describes the failure
 *    (thread-local).  No C++ exception crosses this interface.
 *  * Degenerate sizes: M == 0 or N == 0 is a no-op returning MM_OK; K == 0
 *    writes C := 0 (an empty sum).
 *  * Leading dimensions must satisfy lda >= max(K,1), ldb >= max(N,1),
 *    ldc >= max(N,1); C must not overlap A or B.
 *  * Every dimension is at most 2^40, and every stored matrix spans at most
 *    2^62 elements ((rows-1)*ld + cols); larger shapes return MM_E_INVAL.
 *  * Calls on distinct streams may run concurrently from any threads.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mm_status {
    MM_OK = 0,
    MM_E_INVAL = -1,        /* bad argument: sizes, leading dimensions, null or overlapping pointers */
    MM_E_NOMEM = -2,        /* device allocation failed, or a request larger than a server budget */
    MM_E_DEVICE = -3,       /* a HIP runtime call failed */
    MM_E_BUSY = -4,         /* server queue full */
    MM_E_UNSUPPORTED = -5,  /* valid but not implemented combination (e.g. wrong GPU architecture) */
    MM_E_TIMEOUT = -6       /* mm_serve_wait ran out of time; the request is still pending */
} mm_status;

/* How a product is computed. */
typedef enum mm_method {
    MM_F64 = 0,           /* binary64 operands, binary64 MFMA, binary64 accumulation */
    MM_F32 = 1,           /* FP32 operands, FP32 MFMA, FP32 accumulation */
    MM_SPLIT_BF16_3 = 2,  /* FP32 operands as 2 bfloat16 planes, 3 plane products */
    MM_SPLIT_BF16_6 = 3   /* FP32 operands as 3 bfloat16 planes, 6 plane products */
} mm_method;

/* Library version and the GPU architecture the kernels were built for. */
const char *mm_version(void);

/* Text for a status code; never NULL. */
const char *mm_status_string(mm_status s);

/* Description of the last failure on the calling thread ("" if none). */
const char *mm_last_error(void);

/* Check that the current device is a gfx950 and warm the library's per-device
 * state.  Returns MM_E_UNSUPPORTED on another architecture.  Optional: every
 * entry point initialises lazily. */
mm_status mm_init(int device);

/*
 * mm_gemm_f64 -- C = A.B in binary64 (section III's sum, every product and
 * partial sum in binary64 on the FP64 matrix cores).
 *   M, N, K   : A is M x K, B is K x N, C is M x N (row-major, leading dims lda, ldb, ldc)
 *   A, B      : device, read-only;  C : device, overwritten
 *   stream    : hipStream_t or NULL
 * Summation order differs from a serial loop; the result of each entry lies
 * within 4*K*2^-53*(|A||B|)_ij of the exact sum and is exact whenever every
 * partial sum is representable (e.g. small integers).  For a fixed shape the
 * result is deterministic (no atomics, no split-K).
 */
mm_status mm_gemm_f64(int64_t M, int64_t N, int64_t K,
                      const double *A, int64_t lda,
                      const double *B, int64_t ldb,
                      double *C, int64_t ldc, void *stream);

/* mm_gemm_f32 -- as mm_gemm_f64 with FP32 operands, FP32 MFMA and FP32
 * accumulation; per-entry error within 4*K*2^-24*(|A||B|)_ij. */
mm_status mm_gemm_f32(int64_t M, int64_t N, int64_t K,
                      const float *A, int64_t lda,
                      const float *B, int64_t ldb,
                      float *C, int64_t ldc, void *stream);

/*
 * mm_split_bf16 -- the split step on its own: writes the FP32 matrix X
 * (rows x cols, leading dim ldx) as `nplanes` bfloat16 planes, plane 0 =
 * bf16_rne(x), plane p = bf16_rne(x - plane_0 - ... - plane_{p-1}) with the
 * leftovers formed exactly in FP32.  Plane p of element (r, c) is stored at
 *   planes[p * plane_stride + r * cols + c]            (transpose == 0)
 *   planes[p * plane_stride + c * rows + r]            (transpose != 0)
 * as raw bfloat16 bits.  planes: device, caller-owned, at least
 * nplanes * plane_stride elements; plane_stride >= rows * cols.
 * nplanes in {1, 2, 3}.  Non-finite inputs and |x| at or above the largest
 * bfloat16 are outside the contract.
 */
mm_status mm_split_bf16(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                        int32_t nplanes, int32_t transpose,
                        uint16_t *planes, int64_t plane_stride, void *stream);

/* Bytes of device workspace mm_gemm_split_bf16 may need for this shape (the
 * planes of both operands): an upper bound, since the fused tile variants
 * split inside the product and use none. */
size_t mm_split_workspace_bytes(int64_t M, int64_t N, int64_t K, int32_t nprod);

/*
 * mm_gemm_split_bf16 -- C = A.B for FP32 operands on the bfloat16 matrix
 * cores.  A and B are split into bfloat16 planes (2 planes for nprod = 3,
 * 3 planes for nprod = 6, as mm_split_bf16), the plane products
 *   nprod = 3: hi.hi + hi.lo + lo.hi
 *   nprod = 6: h.h + h.m + m.h + h.l + m.m + l.h
 * are accumulated in FP32 in two accumulator sets (the leading h.h product and
 * the sum of the corrections), and each entry is recombined in binary64 as
 * (double)lead + (double)corr before being stored.  Depending on the tile
 * variant the planes are made by a split pass into the workspace or by the
 * product tile itself on the way into on-chip memory ("fused" variants); the
 * planes, and hence the result, are the same bits either way.
 *   C         : device; FP32 (c_is_f64 == 0) or binary64 (c_is_f64 != 0), ldc in elements
 *   workspace : device scratch of at least mm_split_workspace_bytes(M,N,K,nprod)
 *               bytes, or NULL to let the library allocate it stream-ordered
 *               when the chosen variant needs it; its layout is internal
 *               (for nprod = 3 the direct tiles keep the two planes
 *               interleaved per 32-element K block) and its contents scratch
 * Design error against the exact product: about 4e-6 normwise for nprod = 3 on
 * zero-mean data, below 1e-6 for nprod = 6.  nprod not in {3, 6} is MM_E_INVAL.
 * The binary64 residual check of the result is the separate call
 * mm_residual_f64 (it needs a caller-chosen probe vector x); enqueued on the
 * same stream right after this call it runs in stream order behind it.
 * K above 2^26 - 32 is MM_E_UNSUPPORTED for the split methods (here, in
 * mm_gemm_ex, grouped batches and served requests): the tiles address 16
 * plane rows of K elements (or 8 interleaved rows of 2K) with 32-bit byte
 * offsets.
 */
mm_status mm_gemm_split_bf16(int64_t M, int64_t N, int64_t K,
                             const float *A, int64_t lda,
                             const float *B, int64_t ldb,
                             void *C, int64_t ldc, int32_t c_is_f64,
                             int32_t nprod, void *workspace, size_t workspace_bytes,
                             void *stream);

/*
 * mm_residual_f64 -- the residual probe of a computed product (Freivalds):
 * for a caller-chosen probe vector x (binary64, length N, device) computes
 * y = B.x, z = A.y, w = C.x and r = w - z, all in binary64, and stores
 *   out[0] = ||r||_2^2,  out[1] = ||z||_2^2          (out: device, 2 doubles)
 * so sqrt(out[0]/out[1]) is the relative residual of C.  in_dtype selects the
 * element type of A and B and c_dtype that of C: 0 = binary64, 1 = FP32.
 * workspace: device, at least mm_residual_workspace_bytes(M, N, K) bytes, or
 * NULL for stream-ordered allocation by the library.  The reduction order is
 * fixed, so the result is deterministic.
 */
size_t mm_residual_workspace_bytes(int64_t M, int64_t N, int64_t K);
mm_status mm_residual_f64(int64_t M, int64_t N, int64_t K,
                          const void *A, int64_t lda, const void *B, int64_t ldb,
                          const void *C, int64_t ldc, int32_t in_dtype, int32_t c_dtype,
                          const double *x, double *out,
                          void *workspace, size_t workspace_bytes, void *stream);

/*
 * mm_residual_f64_noalloc -- mm_residual_f64 for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, meaning, kernels and result bits
 * as mm_residual_f64, without the workspace: its temporaries (8*(K + 2M + 512)
 * bytes) live in a fixed scratch array of the library, 2 MiB per device
 * (mm_residual_noalloc_max_bytes()), which each device holds from first use
 * until the process ends.  Shapes needing more return MM_E_INVAL.  The call
 * allocates nothing and only enqueues kernels on `stream`.  Every call on one
 * device shares that device's scratch: calls whose work overlaps on the device
 * (other streams, other threads) race and give wrong results, so the caller
 * serialises them (e.g. one stream).  Nothing in the scratch needs clearing
 * between calls.
 */
size_t mm_residual_noalloc_max_bytes(void);
mm_status mm_residual_f64_noalloc(int64_t M, int64_t N, int64_t K,
                                  const void *A, int64_t lda, const void *B, int64_t ldb,
                                  const void *C, int64_t ldc, int32_t in_dtype, int32_t c_dtype,
                                  const double *x, double *out, void *stream);

/*
 * mm_gemm_strassen_f64 -- C = A.B in binary64 by one level of Strassen's
 * scheme in Winograd's form (the sub-cubic method cited in the paper's
 * literature review): A and B are split in 2 x 2 quadrants and C is formed
 * from seven half-size binary64 products (mm_gemm_f64's kernels) and fifteen
 * quadrant additions, in the fixed order
 *   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
 *   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
 *   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
 *   P6 = S2 T2, P7 = S3 T3,
 *   C11 = P1 + P2, C12 = ((P1 + P6) + P5) + P3, C21 = ((P1 + P6) + P7) - P4,
 *   C22 = ((P1 + P6) + P7) + P5.
 * 7/8 of the multiplications of the definition; the error bound is normwise
 * rather than per entry (exact when every intermediate is representable, e.g.
 * small integers).  M, N and K must be even (otherwise MM_E_UNSUPPORTED).
 * workspace: device, >= mm_strassen_workspace_bytes(M, N, K) bytes
 * (8 * (M*K + K*N + 7*M*N/4)), or NULL for stream-ordered allocation.
 */
size_t mm_strassen_workspace_bytes(int64_t M, int64_t N, int64_t K);
mm_status mm_gemm_strassen_f64(int64_t M, int64_t N, int64_t K,
                               const double *A, int64_t lda, const double *B, int64_t ldb,
                               double *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                               void *stream);

/* ------------------------------------------------------------------------ */
/* Transposed operands.                                                      */
/* ------------------------------------------------------------------------ */

/* op(X) = X (MM_OP_N) or X^T (MM_OP_T). */
typedef enum mm_op { MM_OP_N = 0, MM_OP_T = 1 } mm_op;

/* Bytes of device workspace mm_gemm_ex needs (0 when none). */
size_t mm_gemm_ex_workspace_bytes(mm_method method, mm_op opa, mm_op opb, int64_t M, int64_t N, int64_t K);

/*
 * mm_gemm_ex -- C = op(A).op(B), the same product with either operand stored
 * transposed (the storage remark of section III: a column-major operand is
 * the row-major transpose).  All buffers row-major; op(A) is M x K and op(B)
 * is K x N, so A is M x K (lda >= K) for MM_OP_N and K x M (lda >= M) for
 * MM_OP_T; B is K x N (ldb >= N) for MM_OP_N and N x K (ldb >= K) for MM_OP_T.
 * C is M x N: binary64 for MM_F64, FP32 otherwise.  binary64/FP32: a
 * transposed operand is first transposed into the workspace, then the
 * product runs as mm_gemm_f64/f32 (same kernels, same result bits as on
 * explicitly transposed inputs).  Split methods: the split pass writes the
 * planes in the orientation the kernel reads, whatever the operand's storage.
 * workspace: device, >= mm_gemm_ex_workspace_bytes(...), or NULL to let the
 * library allocate it stream-ordered.  A whole column-major product
 * C = A.B (Fortran storage) is mm_gemm_* on the row-major transposes:
 * C^T = B^T.A^T, i.e. swap A with B and M with N.
 */
mm_status mm_gemm_ex(mm_method method, mm_op opa, mm_op opb, int64_t M, int64_t N, int64_t K,
                     const void *A, int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc,
                     void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Grouped products: many independent C_i = A_i.B_i of different shapes in   */
/* one persistent kernel launch.                                             */
/* ------------------------------------------------------------------------ */

/* One problem: device operands, row-major, same rules as mm_gemm_*.  The element
 * type follows the method: binary64 for MM_F64, FP32 otherwise (C is FP32 for
 * every FP32-input method). */
typedef struct mm_problem {
    int64_t M, N, K;
    const void *A; int64_t lda;
    const void *B; int64_t ldb;
    void *C;       int64_t ldc;
} mm_problem;

typedef struct mm_grouped_plan mm_grouped_plan;

/*
 * mm_gemm_grouped -- C_i = A_i.B_i for i < count (host array `probs`), all
 * with the same method, each result identical to what the single-problem
 * entry point with the same tile configuration returns.
 *   plan_inout: NULL runs once: descriptors (and split workspace) live in a
 *     stream-ordered allocation freed after the launch, and are uploaded
 *     through a small ring of library-owned pinned buffers, so the call
 *     enqueues work and returns without waiting for the stream (it waits at
 *     most for the upload of the eighth-latest such call on the device).  Not
 *     for use under stream capture: capture a plan instead.  Otherwise
 *     *plan_inout is a plan cache: if it is
 *     NULL a plan is built for these shapes (tile map, device descriptor
 *     buffers, split workspace, and a HIP graph of the whole sequence captured
 *     on a stream of the plan's own) and returned; if it is an existing plan
 *     whose shapes match, only the operand pointers are refreshed and the
 *     graph is replayed on `stream`.  A plan whose shapes differ is
 *     MM_E_INVAL.  A plan holds one set of device descriptors: its launches
 *     are ordered by the stream they are enqueued on, and a caller using one
 *     plan from several streams orders those streams itself.  A refresh
 *     copies descriptors and split jobs through the plan's own 4-deep pinned
 *     ring and does not wait for the stream (at most for the refresh four
 *     launches back).  A plan is owned by the caller and freed with
 *     mm_grouped_plan_destroy after its last launch finished.
 * count == 0 is a no-op.  Problems with M == 0 or N == 0 are skipped.
 */
mm_status mm_gemm_grouped(const mm_problem *probs, int32_t count, mm_method method,
                          mm_grouped_plan **plan_inout, void *stream);
mm_status mm_grouped_plan_destroy(mm_grouped_plan *plan);

/* Replay a plan's graph on `stream` with the operands it last ran with (no
 * descriptor refresh, one launch call).  The caller keeps those operands alive
 * and unchanged in place; their contents may change between replays. */
mm_status mm_grouped_plan_launch(mm_grouped_plan *plan, void *stream);

/* Tile configuration the plan chose (autotuned or default), its schedule, its
 * tile count, the workgroups of its grid (persistent grid; for schedule 3 one
 * per tile, the count rounded up to a multiple of 64 so that runs of 8
 * consecutive tiles go to one XCD) and whether it replays a graph.  Every
 * output is nullable. */
mm_status mm_grouped_plan_info(const mm_grouped_plan *plan, int32_t *variant_out, int32_t *schedule_out,
                               int64_t *tiles_out, int32_t *grid_out, int32_t *uses_graph_out);

/*
 * mm_gemm_grouped_config -- mm_gemm_grouped with an explicit tile variant (or
 * size-class pair, below) and schedule instead of the autotuned choice.
 * schedule: 0 = problems in the given order, a persistent grid takes tiles by
 * a fixed stride; 1 = heaviest problems (largest M*N*K) first, fixed stride;
 * 2 = heaviest first, the persistent grid pulls tiles from device work
 * counters (one per XCD, each XCD walking its own share of the tile map, for
 * the ring-fused split tiles; one for the others); 3 = heaviest first, one
 * workgroup per tile, dispatched by the hardware.  Every schedule gives the
 * same bits.  An existing plan must have been built with the same variant and
 * schedule.
 */
mm_status mm_gemm_grouped_config(const mm_problem *probs, int32_t count, mm_method method,
                                 int32_t variant, int32_t schedule,
                                 mm_grouped_plan **plan_inout, void *stream);

/*
 * Size-class pairs.  A grouped variant id MM_PAIR_BASE + p, for
 * p < mm_grouped_pair_count(method), runs each problem of the batch on one
 * of two tile variants of the same workgroup size (`small` and `large` of
 * mm_grouped_pair_info): on `small` when its tiles execute at most pct % of
 * the padded work (rows, columns and K rounded up to the tiles) of `large`'s,
 * else on `large`.  The choice is a function of (M, N, K) alone, so each
 * problem's result is identical to the single-problem result of the variant
 * it ran on.  Accepted wherever a grouped variant is: mm_gemm_grouped_config,
 * the grouped autotuner (which times every pair beside the single variants)
 * and the autotune cache.  Split pairs consist of ring-fused variants.
 * mm_grouped_pair_info: MM_E_INVAL for an unknown method or pair; outputs
 * nullable.
 */
#define MM_PAIR_BASE 64
int32_t mm_grouped_pair_count(mm_method method);
mm_status mm_grouped_pair_info(mm_method method, int32_t pair, int32_t *small_out, int32_t *large_out,
                               int32_t *pct_out);

/* ------------------------------------------------------------------------ */
/* Tile configurations and the autotuner.                                    */
/* ------------------------------------------------------------------------ */

/* Number of compiled tile variants for a method, and the tile sizes of one. */
int32_t mm_variant_count(mm_method method);
mm_status mm_variant_info(mm_method method, int32_t variant, int32_t *bm, int32_t *bn, int32_t *bk);

/* The variant the library will use for (method, M, N, K): the autotune cache
 * entry of the shape bucket if present, else a fixed cost model of the shape.
 * A pure function of its arguments and the loaded cache. */
int32_t mm_select_variant(mm_method method, int64_t M, int64_t N, int64_t K);

/* Run a single product with an explicit variant (for tuning and tests).
 * Operand element types follow `method`; workspace as mm_gemm_split_bf16. */
mm_status mm_gemm_variant(mm_method method, int32_t variant,
                          int64_t M, int64_t N, int64_t K,
                          const void *A, int64_t lda, const void *B, int64_t ldb,
                          void *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                          void *stream);

/*
 * mm_autotune -- time every variant of `method` on the caller's operands
 * (device, M x K / K x N / M x N as for mm_gemm_variant; C is overwritten) with
 * `warmup` untimed and `reps` timed launches each (HIP events, median), store
 * the fastest in the cache under the shape's bucket and return it in
 * *variant_out (and its median time in ms in *ms_out, nullable).  The bucket is
 * (method, ceil(log2 M), ceil(log2 N), ceil(log2 K)).  Runs synchronously on
 * `stream`.
 */
mm_status mm_autotune(mm_method method, int64_t M, int64_t N, int64_t K,
                      const void *A, int64_t lda, const void *B, int64_t ldb,
                      void *C, int64_t ldc, int32_t warmup, int32_t reps,
                      int32_t *variant_out, double *ms_out, void *stream);

/*
 * mm_grouped_autotune -- time every (variant, schedule) pair on this batch
 * (plans with graph replay; `warmup` untimed and `reps` timed replays each,
 * median), store the fastest under the batch's bucket (method, ceil(log2
 * count), ceil(log2 mean M*N), ceil(log2 mean K)) so later mm_gemm_grouped
 * calls on similar batches use it, and return it.  The problems' C are
 * overwritten.  Runs synchronously on `stream`.
 */
mm_status mm_grouped_autotune(const mm_problem *probs, int32_t count, mm_method method,
                              int32_t warmup, int32_t reps, int32_t *variant_out,
                              int32_t *schedule_out, double *ms_out, void *stream);

/* Persist / restore the autotune cache as JSON (keyed by architecture).  Loading
 * a file written for another architecture or library version is MM_E_INVAL
 * and leaves the cache unchanged. */
mm_status mm_autotune_save(const char *path);
mm_status mm_autotune_load(const char *path);
mm_status mm_autotune_clear(void);

/* ------------------------------------------------------------------------ */
/* Serving: a continuous-batching request loop.                              */
/* ------------------------------------------------------------------------ */

typedef struct mm_server mm_server;

typedef struct mm_serve_config {
    uint64_t budget_bytes;   /* admission budget: bytes of operands, results and split planes in flight */
    int32_t slots;           /* concurrent launch slots (one HIP stream each), 1..16 */
    int32_t max_batch;       /* most requests packed into one grouped launch, 1..4096 */
    int32_t queue_capacity;  /* most requests waiting for admission; submit beyond it is MM_E_BUSY */
    int32_t device;          /* HIP device ordinal */
    /* Test mode for hosts without a GPU: if > 0 no device is touched and no C
     * is written; each launch is modelled as taking sum(2MNK)/(dry_run_tflops
     * * 1e12) seconds.  0 for real serving. */
    double dry_run_tflops;
    /* Dry-run only: the request with this id (0 = none) completes with
     * MM_E_DEVICE, to exercise per-request failure reporting. */
    uint64_t dry_run_fail_id;
    /* Requests fall in two size classes by their own shape: "large" if
     * M*N >= large_mn (0: 1024*1024), else "small"; each class of each method
     * is launched as its own grouped launch with its own tile variant, so a
     * request always runs with the same kernel.  variants[m] / variants_large[m]
     * (index = mm_method) are the tile variants, e.g. from mm_grouped_autotune on
     * a sample of the expected requests; -1 = the library's choice. */
    int32_t variants[4];
    int32_t variants_large[4];
    int64_t large_mn;
} mm_serve_config;

typedef struct mm_serve_stats_t {
    uint64_t completed;       /* requests finished (ok or failed) */
    uint64_t failed;          /* requests finished with an error */
    double p50_ms, p99_ms;    /* nearest-rank latency percentiles, arrival -> completion */
    double mean_ms, max_ms;
    double useful_flop;       /* sum of 2*M*N*K over completed requests */
    double first_arrival_s;   /* server clock */
    double last_done_s;
    double tflops;            /* useful_flop / (last_done - first_arrival) / 1e12 */
    uint64_t peak_bytes;      /* largest admitted bytes in flight */
    uint64_t launches;        /* grouped launches issued */
    double mean_batch;        /* requests per launch */
} mm_serve_stats_t;

/*
 * mm_serve_create -- start a server: a scheduler thread that admits queued
 * requests in arrival order (the head of the queue is never overtaken) while
 * bytes in flight plus the request's bytes -- A, B and C at their element size
 * plus split workspace -- fit in budget_bytes and a slot is free, packs the admitted requests into grouped
 * launches (one per method present) on the free slot's stream, and retires
 * them when the slot's completion event fires.  Requests that arrive while
 * others run are admitted as soon as a slot and budget free up, so their work
 * overlaps on the device.  A request is charged its split planes only when its
 * class's tile variant reads planes (fused variants make none).  Each slot
 * keeps those planes in a grow-only workspace (it doubles when a batch needs
 * more; outgrown buffers are kept until mm_serve_destroy, since freeing would
 * wait for the whole device), which is not charged to the budget: the device
 * memory a server holds beyond its budget is at most about four times the
 * planes of the largest batch, per slot.
 */
mm_status mm_serve_create(const mm_serve_config *cfg, mm_server **out);

/*
 * mm_serve_submit -- enqueue C = A.B (device operands, caller-owned, valid
 * until mm_serve_wait returns for this id).  A and B must hold their values,
 * and C must be free to overwrite, when submit is called: the server's slot
 * streams do not wait for any caller stream, so work that writes A or B, or
 * still reads or writes C, on another stream must have finished first (e.g.
 * synchronise that stream before submitting).  method: MM_F64, MM_F32,
 * MM_SPLIT_BF16_3 or MM_SPLIT_BF16_6.  arrival_s is the request's arrival
 * time on the server clock (mm_serve_clock); latency is measured from it, so a
 * client replaying a schedule charges queueing before submission too; pass a
 * negative value for "now".  Thread-safe.  A request whose bytes exceed the
 * whole budget is MM_E_NOMEM at submit; a full queue is MM_E_BUSY.
 */
mm_status mm_serve_submit(mm_server *srv, const mm_problem *req, mm_method method,
                          double arrival_s, uint64_t *id_out);

/* Wait up to timeout_us (negative: forever) for request id.  On MM_OK the
 * request has finished: *req_status (nullable) is its own status and
 * *latency_ms (nullable) its latency, and the id is retired.  MM_E_TIMEOUT if
 * still pending (the id stays valid).  An id that was never issued or is
 * already retired is MM_E_INVAL; of several threads waiting on one id, the
 * first to wake collects it and the others return MM_E_INVAL. */
mm_status mm_serve_wait(mm_server *srv, uint64_t id, int64_t timeout_us,
                        mm_status *req_status, double *latency_ms);

/* Seconds since the server was created (monotonic clock). */
double mm_serve_clock(const mm_server *srv);

mm_status mm_serve_stats(mm_server *srv, mm_serve_stats_t *out);

/* Stop accepting requests, finish those in flight, free everything. */
mm_status mm_serve_destroy(mm_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
