// Split-precision product of FP32 matrices on the bfloat16 matrix cores.
//
// Split pass: an FP32 value x is written as bfloat16 planes, plane 0 = bf16(x)
// and each further plane = bf16 of what the previous planes leave over; the
// leftover is formed in FP32, where it is exact.  Conversions use the gfx950
// packed convert (round to nearest even).
//
// Split GEMM: C = sum over the method's plane pairs (p, q) of A_p . B_q with
// v_mfma_f32_16x16x32_bf16, two FP32 accumulator sets per output block (the
// leading A_0.B_0 product and the sum of the corrections), recombined per entry
// in binary64.  A planes are M x K row-major; B planes are stored transposed
// (N x K) by the split pass, so both operands are k-contiguous and every MFMA
// fragment is one 16-byte LDS read.
//
// MFMA lane layout (16x16x32 bf16): lane l supplies A[l%16][k-group l/16] and
// B[k-group l/16][l%16], 8 consecutive k each, and receives D[4*(l/16)+v][l%16].
#include "mm_internal.h"

namespace mm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_value(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// ------------------------------------------------------------------ split pass
// Row-major planes: each thread splits 4 consecutive elements of one row.
__global__ void split_rows_kernel(const float *__restrict__ X, int64_t ldx, int64_t rows, int64_t cols, int nplanes,
                                  uint16_t *__restrict__ planes, int64_t plane_stride) {
    const int64_t quads_per_row = (cols + 3) / 4;
    const int64_t total = rows * quads_per_row;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / quads_per_row;
        const int64_t c0 = (t % quads_per_row) * 4;
        const float *src = X + r * ldx + c0;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (c0 + e < cols) ? src[e] : 0.f;
        for (int p = 0; p < nplanes; ++p) {
            uint16_t *dst = planes + p * plane_stride + r * cols + c0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint16_t h = bf16_bits(v[e]);
                if (c0 + e < cols) dst[e] = h;
                v[e] = v[e] - bf16_value(h);
            }
        }
    }
}

// Transposed planes: 64 x 64 tiles through LDS so both the FP32 reads (along
// a row of X) and the bfloat16 writes (along a row of X^T) are coalesced.
__global__ __launch_bounds__(256) void split_transpose_kernel(const float *__restrict__ X, int64_t ldx, int64_t rows,
                                                              int64_t cols, int nplanes, uint16_t *__restrict__ planes,
                                                              int64_t plane_stride) {
    __shared__ float tile[64][65];
    const int64_t tiles_c = (cols + 63) / 64;
    const int64_t r0 = (blockIdx.x / tiles_c) * 64;
    const int64_t c0 = (blockIdx.x % tiles_c) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.f;
    }
    __syncthreads();
    // output element (c, r) of X^T: thread tx walks r
    for (int j = ty; j < 64; j += 4) {
        const int64_t c = c0 + j, r = r0 + tx;
        if (c >= cols || r >= rows) continue;
        float v = tile[tx][j];
        for (int p = 0; p < nplanes; ++p) {
            const uint16_t h = bf16_bits(v);
            planes[p * plane_stride + c * rows + r] = h;
            v = v - bf16_value(h);
        }
    }
}

hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, int nplanes, int transpose,
                        uint16_t *planes, int64_t plane_stride, hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (transpose) {
        const int64_t blocks = ((rows + 63) / 64) * ((cols + 63) / 64);
        if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(split_transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, ldx, rows, cols,
                           nplanes, planes, plane_stride);
    } else {
        int64_t blocks = (rows * ((cols + 3) / 4) + 255) / 256;
        if (blocks > 1 << 20) blocks = 1 << 20;
        hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, ldx, rows, cols,
                           nplanes, planes, plane_stride);
    }
    return hipGetLastError();
}

size_t split_b_offset_bytes(int64_t M, int64_t K, int nprod) {
    const int np = nprod == 3 ? 2 : 3;
    // B planes start 256-byte aligned behind the A planes
    return ((size_t)np * M * K * 2 + 255) & ~(size_t)255;
}

size_t split_workspace_bytes(int64_t M, int64_t N, int64_t K, int nprod) {
    const int np = nprod == 3 ? 2 : 3;
    return split_b_offset_bytes(M, K, nprod) + (size_t)np * N * K * 2;
}

// ------------------------------------------------------------------ split GEMM
// Plane pairs of each method; entry 0 is the leading product.
template <int NPROD> struct SplitTerms;
template <> struct SplitTerms<3> {
    static constexpr int NP = 2;
    static constexpr int n = 3;
    static constexpr int pa[3] = {0, 0, 1};
    static constexpr int pb[3] = {0, 1, 0};
};
template <> struct SplitTerms<6> {
    static constexpr int NP = 3;
    static constexpr int n = 6;
    static constexpr int pa[6] = {0, 0, 1, 0, 1, 2};
    static constexpr int pb[6] = {0, 1, 0, 2, 1, 0};
};

template <int NPROD, int BM_, int BN_, int BK_, int WM_, int WN_>
struct SplitTile {
    using Terms = SplitTerms<NPROD>;
    static constexpr int NP = Terms::NP;
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int NWN = BN / WN;
    static constexpr int NWAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = NWAVES * 64;
    static constexpr int FM = WM / 16, FN = WN / 16;
    static constexpr int KSTEPS = BK / 32;
    static constexpr int LD = BK + 8;                 // bf16 elements per LDS row (16-byte pad)
    static constexpr int A_PLANE = BM * LD, B_PLANE = BN * LD;
    static constexpr int STAGE = NP * (A_PLANE + B_PLANE);
    static constexpr int LDS_ELEMS = 2 * STAGE;
    static constexpr int VROW = BK / 8;               // 16-byte vectors per row
    static constexpr int A_VECS = NP * BM * VROW / NT;
    static constexpr int B_VECS = NP * BN * VROW / NT;
    static_assert(BK % 32 == 0, "BK multiple of 32");
    static_assert((NP * BM * VROW) % NT == 0 && (NP * BN * VROW) % NT == 0, "load split");

    // planes: base of plane 0, plane p at + p*pstride; rows x K k-contiguous.
    static __device__ __forceinline__ void load(u16x8 *regs, int nvec, const uint16_t *__restrict__ planes,
                                                int64_t pstride, int64_t row0, int64_t nrows_total, int64_t K,
                                                int64_t k0, int rows_tile, bool vec_ok) {
        const int tid = threadIdx.x;
        for (int i = 0; i < nvec; ++i) {
            const int v = tid + i * NT;
            const int p = v / (rows_tile * VROW);
            const int rem = v % (rows_tile * VROW);
            const int r = rem / VROW;
            const int c = (rem % VROW) * 8;
            const int64_t gr = row0 + r;
            const uint16_t *src = planes + p * pstride + gr * K + k0 + c;
            if (gr < nrows_total && vec_ok && k0 + c + 8 <= K) {
                regs[i] = *reinterpret_cast<const u16x8 *>(src);
            } else {
                u16x8 t;
#pragma unroll
                for (int e = 0; e < 8; ++e) t[e] = (gr < nrows_total && k0 + c + e < K) ? src[e] : (uint16_t)0;
                regs[i] = t;
            }
        }
    }

    static __device__ __forceinline__ void store(uint16_t *lds, int plane_elems, const u16x8 *regs, int nvec,
                                                 int rows_tile) {
        const int tid = threadIdx.x;
        for (int i = 0; i < nvec; ++i) {
            const int v = tid + i * NT;
            const int p = v / (rows_tile * VROW);
            const int rem = v % (rows_tile * VROW);
            const int r = rem / VROW;
            const int c = (rem % VROW) * 8;
            *reinterpret_cast<u16x8 *>(lds + p * plane_elems + r * LD + c) = regs[i];
        }
    }

    static __device__ __forceinline__ bf16x8 frag(const uint16_t *lds, int row, int kofs) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(lds + row * LD + kofs));
    }

    static __device__ __forceinline__ void compute(const uint16_t *As, const uint16_t *Bs, f32x4 (&lead)[FM][FN],
                                                   f32x4 (&corr)[FM][FN]) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            const int kofs = s * 32 + q * 8;
#pragma unroll
            for (int t = 0; t < Terms::n; ++t) {
                bf16x8 a[FM], b[FN];
#pragma unroll
                for (int fm = 0; fm < FM; ++fm)
                    a[fm] = frag(As + Terms::pa[t] * A_PLANE, wm * WM + fm * 16 + li, kofs);
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    b[fn] = frag(Bs + Terms::pb[t] * B_PLANE, wn * WN + fn * 16 + li, kofs);
#pragma unroll
                for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                    for (int fn = 0; fn < FN; ++fn) {
                        if (t == 0)
                            lead[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], b[fn], lead[fm][fn], 0, 0, 0);
                        else
                            corr[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], b[fn], corr[fm][fn], 0, 0, 0);
                    }
            }
        }
    }

    // Tile (tm, tn) of C from A planes (M x K, stride pa_stride) and transposed
    // B planes (N x K, stride pb_stride).
    static __device__ __forceinline__ void run(const uint16_t *__restrict__ Ap, int64_t pa_stride,
                                               const uint16_t *__restrict__ Bt, int64_t pb_stride, void *C,
                                               int64_t ldc, int c_is_f64, int64_t M, int64_t N, int64_t K, int64_t tm,
                                               int64_t tn, bool vec_ok, uint16_t *smem) {
        const int64_t m0 = tm * BM, n0 = tn * BN;
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        u16x8 ra[A_VECS], rb[B_VECS];
        const int64_t nkt = (K + BK - 1) / BK;
        load(ra, A_VECS, Ap, pa_stride, m0, M, K, 0, BM, vec_ok);
        load(rb, B_VECS, Bt, pb_stride, n0, N, K, 0, BN, vec_ok);
        store(smem, A_PLANE, ra, A_VECS, BM);
        store(smem + NP * A_PLANE, B_PLANE, rb, B_VECS, BN);
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const bool more = kt + 1 < nkt;
            if (more) {
                load(ra, A_VECS, Ap, pa_stride, m0, M, K, (kt + 1) * BK, BM, vec_ok);
                load(rb, B_VECS, Bt, pb_stride, n0, N, K, (kt + 1) * BK, BN, vec_ok);
            }
            const uint16_t *cur = smem + (kt & 1) * STAGE;
            compute(cur, cur + NP * A_PLANE, lead, corr);
            if (more) {
                uint16_t *nxt = smem + ((kt + 1) & 1) * STAGE;
                store(nxt, A_PLANE, ra, A_VECS, BM);
                store(nxt + NP * A_PLANE, B_PLANE, rb, B_VECS, BN);
            }
            __syncthreads();
        }
        // binary64 recombination of the two accumulator sets
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t r = m0 + wm * WM + fm * 16 + q * 4 + v;
                    const int64_t c = n0 + wn * WN + fn * 16 + li;
                    if (r < M && c < N) {
                        const double val = (double)lead[fm][fn][v] + (double)corr[fm][fn][v];
                        if (c_is_f64) ((double *)C)[r * ldc + c] = val;
                        else ((float *)C)[r * ldc + c] = (float)val;
                    }
                }
    }
};

__device__ void tile_order_split(int64_t bid, int64_t tiles_m, int64_t tiles_n, int64_t *tm, int64_t *tn) {
    const int64_t total = tiles_m * tiles_n;
    int64_t b = bid;
    if (total % 8 == 0) b = (bid % 8) * (total / 8) + bid / 8;
    const int group_m = 8;
    const int64_t per_group = (int64_t)group_m * tiles_n;
    const int64_t g = b / per_group;
    const int64_t first_m = g * group_m;
    const int64_t gsize = (tiles_m - first_m) < group_m ? (tiles_m - first_m) : group_m;
    const int64_t in = b % per_group;
    *tm = first_m + in % gsize;
    *tn = in / gsize;
}

template <typename ST>
__global__ __launch_bounds__(ST::NT) void split_gemm_kernel(const uint16_t *__restrict__ Ap, int64_t pa_stride,
                                                            const uint16_t *__restrict__ Bt, int64_t pb_stride,
                                                            void *C, int64_t ldc, int c_is_f64, int64_t M, int64_t N,
                                                            int64_t K, int64_t tiles_m, int64_t tiles_n, int vec_ok) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[ST::LDS_ELEMS];
    int64_t tm, tn;
    tile_order_split(blockIdx.x, tiles_m, tiles_n, &tm, &tn);
    ST::run(Ap, pa_stride, Bt, pb_stride, C, ldc, c_is_f64, M, N, K, tm, tn, vec_ok != 0, smem);
}

template <typename ST>
static hipError_t launch_split_tile(int64_t M, int64_t N, int64_t K, const uint16_t *Ap, const uint16_t *Bt, void *C,
                                    int64_t ldc, int c_is_f64, hipStream_t stream) {
    const int64_t tiles_m = (M + ST::BM - 1) / ST::BM;
    const int64_t tiles_n = (N + ST::BN - 1) / ST::BN;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const int vec_ok = (K % 8 == 0) && ((uintptr_t)Ap % 16 == 0) && ((uintptr_t)Bt % 16 == 0);
    hipLaunchKernelGGL((split_gemm_kernel<ST>), dim3((unsigned)blocks), dim3(ST::NT), 0, stream, Ap, M * K, Bt,
                       N * K, C, ldc, c_is_f64, M, N, K, tiles_m, tiles_n, vec_ok);
    return hipGetLastError();
}

#define MM_SPLIT_VARIANTS(X)        \
    X(0, 128, 128, 32, 64, 64)      \
    X(1, 64, 64, 32, 32, 32)        \
    X(2, 128, 64, 32, 64, 32)

#define MM_S_COUNT(id, bm, bn, bk, wm, wn) +1
#define MM_S_CFG(id, bm, bn, bk, wm, wn) case id: return TileCfg{bm, bn, bk};
int split_variant_count() { return 0 MM_SPLIT_VARIANTS(MM_S_COUNT); }
TileCfg split_variant(int v) {
    switch (v) { MM_SPLIT_VARIANTS(MM_S_CFG) default: return TileCfg{0, 0, 0}; }
}

#define MM_S_LAUNCH(id, bm, bn, bk, wm, wn)                                                                        \
    case id:                                                                                                       \
        return nprod == 3                                                                                          \
                   ? launch_split_tile<SplitTile<3, bm, bn, bk, wm, wn>>(M, N, K, Ap, Bt, C, ldc, c_is_f64, stream) \
                   : launch_split_tile<SplitTile<6, bm, bn, bk, wm, wn>>(M, N, K, Ap, Bt, C, ldc, c_is_f64, stream);

hipError_t launch_gemm_split(int variant, int nprod, int64_t M, int64_t N, int64_t K, const uint16_t *Ap,
                             const uint16_t *Bt, void *C, int64_t ldc, int c_is_f64, hipStream_t stream) {
    switch (variant) {
        MM_SPLIT_VARIANTS(MM_S_LAUNCH)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mm
