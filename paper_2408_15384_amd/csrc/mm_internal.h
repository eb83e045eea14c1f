// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include <vector>
#include "../../include/mm.h"

namespace mm {

// Thread-local error text behind mm_last_error().
void set_error(const std::string &msg);
mm_status fail(mm_status s, const std::string &msg);
mm_status hip_fail(hipError_t e, const char *what);

// Synchronous argument checks shared by every product entry point.
// Split methods: plane rows (K rounded up to 32) stay below 2^26 elements, so
// the 32-bit per-lane offsets of a ring load over 16 plane rows fit.
constexpr int64_t kSplitMaxK = ((int64_t)1 << 26) - 32;
mm_status check_split_k(int64_t K);
// The current device is one the kernels were built for (gfx950).
mm_status check_arch();
mm_status check_gemm_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                          int64_t ldb, const void *C, int64_t ldc, size_t ab_elem, size_t c_elem);

#define MM_HIP(call)                                                   \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ::mm::hip_fail(_e, #call);        \
    } while (0)

// Tile rows per group of the single-product tile order (tile_order in
// gemm_tile.h) for `kernel`, launched with nt threads per BM x BN tile.  The R
// workgroups resident on one XCD at a time (its 32 CUs times the kernel's
// workgroups per CU) then cover about g tile rows by R/g tile columns; each K
// step they fetch g A slices and R/g B slices from beyond the L2, so over the
// product A is re-fetched once per window of columns and B once per window of
// rows.  For a square product the sum is least at g = sqrt(R * BN / BM).
inline int tile_group_rows(const void *kernel, int nt, int bm, int bn) {
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    const double r = __builtin_sqrt(32.0 * per_cu * bn / bm);
    return r < 1.0 ? 1 : (int)(r + 0.5);
}

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
// Fused split variants read the FP32 operands directly (no plane pass, no
// workspace); they take row-major operands only.
bool split_variant_fused(int v);
hipError_t launch_split_fused(int variant, int nprod, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                              const float *B, int64_t ldb, void *C, int64_t ldc, int c_is_f64, hipStream_t stream);
// The default plane-reading variant (for transposed operands).
int default_unfused_split_variant(mm_method method, int64_t M, int64_t N, int64_t K);

// Plain MFMA GEMM (row-major NN), launches on `stream`.
hipError_t launch_gemm_f64(int variant, int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t stream);
hipError_t launch_gemm_f32(int variant, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                           const float *B, int64_t ldb, float *C, int64_t ldc, hipStream_t stream);

// Split pass: FP32 -> nplanes bfloat16 planes (optionally transposed); output
// rows hold ldp elements (>= the row length), the tail written as zero.
// interleave != 0 (ldp a multiple of 32): one array of rows of nplanes * ldp
// elements, each 32-element block of a row followed by the same block of the
// next plane; plane_stride is then unused.
hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, int nplanes, int transpose,
                        uint16_t *planes, int64_t plane_stride, int64_t ldp, int interleave, hipStream_t stream);
// Row length of the planes the split GEMM reads: K rounded up to 32.
int64_t split_padded_k(int64_t K);

// Split GEMM on planes: A planes M x K row-major (stride M*K), B planes stored
// transposed N x K (stride N*K), K already padded (split_padded_k); C FP32 or
// binary64.  Planes interleaved (launch_split's layout) when
// split_planes_interleaved(variant, nprod).
hipError_t launch_gemm_split(int variant, int nprod, int64_t M, int64_t N, int64_t K, const uint16_t *Ap,
                             const uint16_t *Bt, void *C, int64_t ldc, int c_is_f64, hipStream_t stream);
// Whether the single-problem split tile of this variant reads interleaved
// planes (the direct tiles of the 2-plane method).
bool split_planes_interleaved(int variant, int nprod);

size_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int nprod);
// Byte offset of the B planes inside the split workspace.
size_t split_b_offset_bytes(int64_t M, int64_t K, int nprod);

// Residual probe.
size_t residual_workspace_bytes(int64_t M, int64_t N, int64_t K);
hipError_t launch_residual(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                           int64_t ldb, const void *C, int64_t ldc, int in_dtype, int c_dtype, const double *x,
                           double *out, void *ws, hipStream_t stream);
// Fixed per-device scratch of the no-allocation residual entry point:
// kResidualScratchDoubles binary64 values (2 MiB).  residual_scratch_init looks
// up the current device's address of the array once; residual_scratch returns
// it (looking it up on first use).
constexpr size_t kResidualScratchDoubles = (size_t)1 << 18;
hipError_t residual_scratch_init();
hipError_t residual_scratch(void **ptr);

// Y (cols x rows, leading dim ldy) = X^T for X rows x cols (leading dim ldx).
hipError_t launch_transpose(const void *X, int64_t ldx, int64_t rows, int64_t cols, void *Y, int64_t ldy,
                            int elem_bytes, hipStream_t stream);

// Split pass + split GEMM for operands in any orientation (planes in ws).
hipError_t launch_split_product(int variant, int nprod, int opa, int opb, int64_t M, int64_t N, int64_t K,
                                const float *A, int64_t lda, const float *B, int64_t ldb, void *C, int64_t ldc,
                                int c_is_f64, void *ws, hipStream_t st);

// One Strassen-Winograd level on the binary64 GEMM (M, N, K even, > 0).
size_t strassen_workspace_bytes(int64_t M, int64_t N, int64_t K);
hipError_t launch_strassen_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
                               int64_t ldb, double *C, int64_t ldc, void *ws, hipStream_t st);

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
    int32_t tiles_m;      // tiles along M
};

// One split job of a grouped launch: the planes of one operand.
struct SplitJob {
    const float *X;
    int64_t ldx, rows, cols;
    uint16_t *planes;
    int64_t pstride;
    int64_t ldp;          // output row length (>= row length; tail zero)
    int64_t tile_begin;
    int32_t tiles_c;
    int32_t nplanes;
    int32_t transpose;
    int32_t pad;
};

// Owner problem and tile coordinates of one tile of a grouped batch (the
// kernels read these, when a launch has the table, instead of searching the
// prefix sums); kind: which variant of a size-class pair computes the tile
// (0 the small one, 1 the large one; 0 in single-variant launches).
struct TileRef {
    int32_t own, tm, tn, kind;
};

// Host tile map of one grouped batch.
struct Layout {
    std::vector<GroupedDesc> descs;
    std::vector<SplitJob> jobs;
    std::vector<int8_t> kinds;   // per descriptor: the pair member it runs on (pair launches)
    int64_t total_tiles = 0;
    int64_t split_tiles = 0;
    size_t ws_bytes = 0;  // split planes of the whole batch
    bool ring_ok = true;  // every problem fits the ring-fused tiles' 31-bit lane offsets
};

int grouped_tile_bm(mm_method method, int variant);
int grouped_tile_bn(mm_method method, int variant);
// Size-class pairs (grouped variant ids MM_PAIR_BASE + p).
struct PairCfg { int small, large, pct; };
int grouped_pair_count(mm_method method);
bool grouped_pair(mm_method method, int variant, PairCfg *out);
// A tile variant of the method or one of its pairs.
bool grouped_variant_valid(mm_method method, int variant);
// Launch order of the problems for a schedule (0: as given; 1, 2: heaviest first).
std::vector<int> schedule_order(const mm_problem *probs, int count, int schedule);
// Descriptors (and, for plane-reading split variants, split jobs with planes
// carved from `ws`; ws may be null while sizing) of the problems in `order`
// tiled by `variant`; empty problems are dropped.
void build_layout(const mm_problem *probs, const std::vector<int> &order, mm_method method, int variant,
                  char *ws, Layout *L);
// Kernel forms of a grouped launch: one workgroup per tile (schedule 3), a
// persistent grid looping over tiles (schedules 0-2), or, for the ring-fused
// split tiles when every problem fits them, the streamed persistent grid
// (schedules 0-2; schedule 2 draws tiles from the work counter).
constexpr int kFormTile = 0, kFormPersistent = 1, kFormStream = 2;
int grouped_form(mm_method method, int variant, int schedule, const Layout &L);
// Tile table of a layout, in tile-id order.
void build_tile_table(const Layout &L, std::vector<TileRef> *out);
// Enqueue [grouped split pass] -> [counter reset] -> grouped GEMM for
// descriptors already in device memory.
// d_tiles: the layout's tile table on the device; required by the streamed
// form, optional for the others (null: they search the prefix sums).
hipError_t grouped_enqueue(mm_method method, int variant, int form, const GroupedDesc *d_descs, int ndesc, int64_t total_tiles,
                           const SplitJob *d_jobs, int njobs, int64_t split_tiles, int *d_counter,
                           const TileRef *d_tiles, hipStream_t st);
// Keep memory freed by hipFreeAsync in the device's default pool.
void retain_default_pool();

// Autotune cache lookup (pure function of key + loaded cache).
int select_variant(mm_method method, int64_t M, int64_t N, int64_t K);
// The variant to run for operands the direct global-to-LDS loads can take
// (direct_ok) or not: a variant whose fallback body spills is swapped.
int variant_for_operands(mm_method method, int variant, bool direct_ok);
// Whether the direct tiles take these operands: element-aligned bases, N at
// least one 16-byte vector, and a tile's rows of A (256) and K step of B (32)
// within 31-bit offsets.
inline bool direct_operands(const void *A, int64_t lda, const void *B, int64_t ldb, int64_t N, int64_t elem) {
    return N >= 16 / elem && (uintptr_t)A % elem == 0 && (uintptr_t)B % elem == 0 &&
           256 * lda * elem < 0x7fffffffLL && 32 * ldb * elem < 0x7fffffffLL;
}
// Variant and schedule of a grouped launch: the cache entry of the batch's
// bucket (method, count, mean M, mean N, mean K) if present, else a size rule.
int select_grouped(const mm_problem *probs, int count, mm_method method, int *schedule);
// The variant of untuned grouped batches (and of the server's small class).
int default_grouped_variant(mm_method method);
void store_grouped(const mm_problem *probs, int count, mm_method method, int variant, int schedule, double ms);

}  // namespace mm
