// Workgroup tile of the dense product C = A.B on the gfx950 matrix cores, for
// binary64 (v_mfma_f64_16x16x4_f64) and FP32 (v_mfma_f32_16x16x4_f32).
//
// The definition being computed is the row-by-column sum of the paper's
// section III, C[i][j] = sum_k A[i][k] B[k][j], with row-major operands.  The
// paper's own loop nest and its CPU cache-blocking idea are not followed:
// a workgroup owns a BM x BN tile of C, walks K in steps of BK, stages the
// A (BM x BK) and B (BK x BN) slices in LDS through 16-byte coalesced global
// loads (double-buffered, next slice in flight while the current one is
// multiplied), and each 64-lane wave multiplies a WM x WN sub-tile held in
// accumulator registers as (WM/16) x (WN/16) blocks of 16 x 16.
//
// Lane layout of one 16x16x4 MFMA: lane l supplies A[l%16][k(l/16)] and
// B[k(l/16)][l%16]; of the four results it receives, result v is
// D[l/16 + 4v][l%16] for f64 and D[4(l/16) + v][l%16] for f32 (measured on
// gfx950).  Within a BK slice, lane group q = l/16 takes k = q*(BK/4) + s in
// MFMA step s, so each lane reads BK/4 consecutive elements of an A row in one
// LDS access, and 16 lanes read 16 consecutive elements of a B row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    typedef double vec_t __attribute__((ext_vector_type(2)));  // 16 bytes
    static constexpr int VEC = 2;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row (within the 16x16 block) of result v in lane group q
    static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};
template <> struct MfmaOp<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    typedef float vec_t __attribute__((ext_vector_type(4)));   // 16 bytes
    static constexpr int VEC = 4;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};

// Contiguous run of N elements read from LDS as one access where possible.
template <typename T, int N> struct Run { T v[N]; };

template <typename T, int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileGemm {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int NWN = BN / WN;
    static constexpr int NWAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = NWAVES * 64;
    static constexpr int VEC = MfmaOp<T>::VEC;
    static constexpr int FM = WM / 16, FN = WN / 16, KS = BK / 4;
    // Interleave the next slice's LDS stores with this slice's MFMAs
    // (measured: helps the 64-cycle binary64 MFMA, hurts FP32).
    static constexpr bool INTERLEAVE = sizeof(T) == 8;
    // Row padding (elements) keeps the lane groups of an LDS read on distinct
    // banks and every row 16-byte aligned.  A: 16 lanes read 16 rows at one
    // offset, so the row stride is an odd multiple of 16 bytes.  B: the four
    // lane groups read rows KS apart, which must fall 64 bytes (FP32: all 64
    // lanes in one pass) or 128 bytes (binary64: 32 lanes per pass) apart
    // modulo the 256-byte bank row.
    static constexpr int APAD = 16 / sizeof(T);
    static constexpr int BPAD = sizeof(T) == 8 ? 4 : 4;
    static constexpr int AS_LD = BK + APAD;
    static constexpr int BS_LD = BN + BPAD;
    static constexpr int A_STAGE = BM * AS_LD;
    static constexpr int B_STAGE = BK * BS_LD;
    static constexpr int LDS_ELEMS = 2 * (A_STAGE + B_STAGE);
    static constexpr int AV_ROW = BK / VEC;              // 16-byte vectors per A row slice
    static constexpr int BV_ROW = BN / VEC;              // 16-byte vectors per B row slice
    static constexpr int A_VECS = BM * AV_ROW / NT;      // per thread
    static constexpr int B_VECS = BK * BV_ROW / NT;
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "tile shape");
    static_assert(BK % 4 == 0 && BK % VEC == 0, "BK");
    static_assert((BM * AV_ROW) % NT == 0 && (BK * BV_ROW) % NT == 0, "load split");

    typedef typename MfmaOp<T>::acc_t acc_t;
    typedef typename MfmaOp<T>::vec_t vec_t;

    // Global -> registers for the slice starting at k0.  Out-of-range elements
    // (beyond M, N or K) read as zero so ragged edges add nothing.
    static __device__ __forceinline__ void load_a(vec_t (&ra)[A_VECS], const T *__restrict__ A, int64_t lda,
                                                  int rows_left, int64_t K, int64_t k0, bool vec_ok) {
        const int tid = threadIdx.x;
        const bool kfull = vec_ok && (k0 + BK <= K);
#pragma unroll
        for (int i = 0; i < A_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / AV_ROW;
            const int c = (v % AV_ROW) * VEC;
            const T *p = A + (int64_t)r * lda + k0 + c;
            if (r < rows_left && kfull) {
                ra[i] = *reinterpret_cast<const vec_t *>(p);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    ra[i][e] = (r < rows_left && k0 + c + e < K) ? p[e] : T(0);
            }
        }
    }

    static __device__ __forceinline__ void load_b(vec_t (&rb)[B_VECS], const T *__restrict__ B, int64_t ldb,
                                                  int cols_left, int64_t K, int64_t k0, bool vec_ok) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < B_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / BV_ROW;
            const int c = (v % BV_ROW) * VEC;
            const T *p = B + (k0 + r) * ldb + c;
            const bool krow = (k0 + r < K);
            if (krow && vec_ok && c + VEC <= cols_left) {
                rb[i] = *reinterpret_cast<const vec_t *>(p);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    rb[i][e] = (krow && c + e < cols_left) ? p[e] : T(0);
            }
        }
    }

    static __device__ __forceinline__ void store_a(T *As, const vec_t (&ra)[A_VECS]) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < A_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / AV_ROW;
            const int c = (v % AV_ROW) * VEC;
            *reinterpret_cast<vec_t *>(As + r * AS_LD + c) = ra[i];
        }
    }

    static __device__ __forceinline__ void store_b(T *Bs, const vec_t (&rb)[B_VECS]) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < B_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / BV_ROW;
            const int c = (v % BV_ROW) * VEC;
            *reinterpret_cast<vec_t *>(Bs + r * BS_LD + c) = rb[i];
        }
    }

    // K sub-steps [S0, S1) of one BK slice from LDS into the accumulators.
    template <int S0, int S1>
    static __device__ __forceinline__ void compute(const T *As, const T *Bs, acc_t (&acc)[FM][FN]) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
        Run<T, KS> a[FM];
        T b[FN][KS];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
            a[fm] = *reinterpret_cast<const Run<T, KS> *>(As + (wm * WM + fm * 16 + li) * AS_LD + q * KS);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int s = S0; s < S1; ++s)
                b[fn][s] = Bs[(q * KS + s) * BS_LD + wn * WN + fn * 16 + li];
        if (INTERLEAVE) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s = S0; s < S1; ++s)
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    acc[fm][fn] = MfmaOp<T>::mma(a[fm].v[s], b[fn][s], acc[fm][fn]);
        if (INTERLEAVE) __builtin_amdgcn_s_setprio(0);
    }

    // The whole tile (tm, tn): C[tm*BM.., tn*BN..] = A[tm*BM.., :] . B[:, tn*BN..].
    // `smem` holds LDS_ELEMS elements.  vec_ok: leading dimensions and bases
    // allow 16-byte vector access.
    static __device__ __forceinline__ void run(const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                               int64_t ldb, T *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                               int64_t K, int64_t tm, int64_t tn, bool vec_ok, T *smem) {
        const int64_t m0 = tm * BM, n0 = tn * BN;
        const int rows_left = (int)((M - m0) < BM ? (M - m0) : BM);
        const int cols_left = (int)((N - n0) < BN ? (N - n0) : BN);
        const T *Ab = A + m0 * lda;
        const T *Bb = B + n0;

        acc_t acc[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = acc_t{0, 0, 0, 0};

        vec_t ra[A_VECS], rb[B_VECS];
        const int64_t nkt = (K + BK - 1) / BK;
        constexpr int STAGE = A_STAGE + B_STAGE;
        load_a(ra, Ab, lda, rows_left, K, 0, vec_ok);
        load_b(rb, Bb, ldb, cols_left, K, 0, vec_ok);
        store_a(smem, ra);
        store_b(smem + A_STAGE, rb);
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const bool more = kt + 1 < nkt;
            if (more) {
                load_a(ra, Ab, lda, rows_left, K, (kt + 1) * BK, vec_ok);
                load_b(rb, Bb, ldb, cols_left, K, (kt + 1) * BK, vec_ok);
            }
            const T *cur = smem + (kt & 1) * STAGE;
            T *nxt = smem + ((kt + 1) & 1) * STAGE;
            if (INTERLEAVE) {
                // binary64: the next slice is written to the other LDS buffer
                // between the two halves of this slice's MFMAs, so the stores
                // overlap matrix work (the MFMA bursts run at raised priority)
                compute<0, KS / 2>(cur, cur + A_STAGE, acc);
                if (more) {
                    store_a(nxt, ra);
                    store_b(nxt + A_STAGE, rb);
                }
                compute<KS / 2, KS>(cur, cur + A_STAGE, acc);
            } else {
                compute<0, KS>(cur, cur + A_STAGE, acc);
                if (more) {
                    store_a(nxt, ra);
                    store_b(nxt + A_STAGE, rb);
                }
            }
            __syncthreads();
        }

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
                    const int r = wm * WM + fm * 16 + MfmaOp<T>::row(q, v);
                    const int c = wn * WN + fn * 16 + li;
                    if (r < rows_left && c < cols_left) C[(m0 + r) * ldc + n0 + c] = acc[fm][fn][v];
                }
    }
};

// Tile order for a 1-D grid of tiles_m x tiles_n workgroups.  Workgroups are
// handed to the 8 XCDs round-robin, so consecutive ids land on different L2s.
// The id is first regrouped so that each XCD owns a contiguous range, then the
// range is walked in column-major groups of `group_m` tile rows so that the
// workgroups resident on one XCD at a time share A row panels and B column
// panels in that XCD's L2.
__device__ __forceinline__ void tile_order(int64_t bid, int64_t tiles_m, int64_t tiles_n, int group_m,
                                           int64_t *tm, int64_t *tn) {
    const int64_t total = tiles_m * tiles_n;
    int64_t b = bid;
    if (total % 8 == 0) b = (bid % 8) * (total / 8) + bid / 8;
    const int64_t per_group = (int64_t)group_m * tiles_n;
    const int64_t g = b / per_group;
    const int64_t first_m = g * group_m;
    const int64_t gsize = (tiles_m - first_m) < group_m ? (tiles_m - first_m) : group_m;
    const int64_t in = b % per_group;
    *tm = first_m + in % gsize;
    *tn = in / gsize;
}

}  // namespace mm
