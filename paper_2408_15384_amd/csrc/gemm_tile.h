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

#include "gptr.h"

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
    // The same 16 bytes at element alignment: the global loads take any base
    // and leading dimension (the HSA runtime runs the memory system in
    // unaligned mode, and the compiler emits one 16-byte load for it).
    typedef vec_t vec_ua __attribute__((aligned(sizeof(T))));

    // Global -> registers for the slice starting at k0.  Out-of-range elements
    // (beyond M, N or K) read as zero so ragged edges add nothing; a 16-byte
    // chunk wholly in range is one vector load.
    static __device__ __forceinline__ void load_a(vec_t (&ra)[A_VECS], gptr<const T> A, int64_t lda,
                                                  int rows_left, int64_t K, int64_t k0) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < A_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / AV_ROW;
            const int c = (v % AV_ROW) * VEC;
            gptr<const T> p = A + (int64_t)r * lda + k0 + c;
            if (r < rows_left && k0 + c + VEC <= K) {
                ra[i] = *reinterpret_cast<gptr<const vec_ua>>(p);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    ra[i][e] = (r < rows_left && k0 + c + e < K) ? p[e] : T(0);
            }
        }
    }

    static __device__ __forceinline__ void load_b(vec_t (&rb)[B_VECS], gptr<const T> B, int64_t ldb,
                                                  int cols_left, int64_t K, int64_t k0) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < B_VECS; ++i) {
            const int v = tid + i * NT;
            const int r = v / BV_ROW;
            const int c = (v % BV_ROW) * VEC;
            gptr<const T> p = B + (k0 + r) * ldb + c;
            const bool krow = (k0 + r < K);
            if (krow && c + VEC <= cols_left) {
                rb[i] = *reinterpret_cast<gptr<const vec_ua>>(p);
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
    // `smem` holds LDS_ELEMS elements.  vec_ok (whether leading dimensions and
    // bases are 16-byte multiples) is part of the shared tile interface; this
    // body does not need it, since its vector loads are element-aligned.
    static __device__ __forceinline__ void run(const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                               int64_t ldb, T *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                               int64_t K, int64_t tm, int64_t tn, bool vec_ok, T *smem) {
        (void)vec_ok;
        const int64_t m0 = tm * BM, n0 = tn * BN;
        const int rows_left = (int)((M - m0) < BM ? (M - m0) : BM);
        const int cols_left = (int)((N - n0) < BN ? (N - n0) : BN);
        const gptr<const T> Ab = (gptr<const T>)A + m0 * lda;
        const gptr<const T> Bb = (gptr<const T>)B + n0;
        const gptr<T> Cg = (gptr<T>)C;

        acc_t acc[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = acc_t{0, 0, 0, 0};

        vec_t ra[A_VECS], rb[B_VECS];
        const int64_t nkt = (K + BK - 1) / BK;
        constexpr int STAGE = A_STAGE + B_STAGE;
        load_a(ra, Ab, lda, rows_left, K, 0);
        load_b(rb, Bb, ldb, cols_left, K, 0);
        store_a(smem, ra);
        store_b(smem + A_STAGE, rb);
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const bool more = kt + 1 < nkt;
            if (more) {
                load_a(ra, Ab, lda, rows_left, K, (kt + 1) * BK);
                load_b(rb, Bb, ldb, cols_left, K, (kt + 1) * BK);
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
                    if (r < rows_left && c < cols_left) Cg[(m0 + r) * ldc + n0 + c] = acc[fm][fn][v];
                }
    }
};

// Direct-to-LDS form of the tile: buffer_load_dwordx4 ... lds moves 16-byte
// chunks of A and B straight into a ring of STAGES LDS buffers (no staging
// registers, no LDS store instructions), so the loads of K steps kt+1 ..
// kt+STAGES-1 are in flight while step kt is multiplied.  One
// wave-instruction fills 64 consecutive 16-byte LDS slots (lane i -> slot i);
// each lane fetches the chunk that the swizzled layout puts in its slot:
//   A rows (BK elements) : chunk ^ ((row / rows per 256 B) mod chunks per row)
//   B rows (BN elements) : chunk ^ (lane group of the row, shifted so the four
//                          groups of an MFMA read sit in distinct bank ranges)
// which spreads each 16-lane group of an A read and each lane group pair of a
// B read over distinct banks.  The LDS counters still book a share of the
// tile's LDS cycles as conflicts (binary64 256x128: 29% with 8 waves of 64x64,
// 40% with 16 waves of 64x32, 5-5.6 cycles per LDS instruction; the compiler
// merges B reads of columns 32 apart into one ds_read2_b64), but per K step
// the LDS is busy ~900-1,300 cycles against 8,192 MFMA cycles per SIMD, so it
// does not bound the tile.  Rows of A past M and
// column chunks of B past N are clamped in bounds (they only feed entries of
// C that are not stored).  Any K: a last step past K reads through byte
// ranges that end at the operands' last valid elements and clears A's columns
// past K in LDS (clear_a_tail); column chunks of B reaching past N feed only
// entries of C that are not stored.  It takes any leading dimension and
// element-aligned bases (see eligible()); it needs N of at least one vector
// and K slices whose lane offsets fit 31 bits, and other problems run the
// register-staged tile (same tile shape) in the same kernel.
typedef __attribute__((address_space(3))) void mm_lvoid;

template <typename T, int BM_, int BN_, int BK_, int WM_, int WN_, int STAGES_>
struct TileGemmDirect {
    typedef TileGemm<T, BM_, BN_, BK_, WM_, WN_> Fallback;
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, STAGES = STAGES_;
    static constexpr int NWN = BN / WN;
    static constexpr int NWAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = NWAVES * 64;
    static constexpr int VEC = MfmaOp<T>::VEC;
    static constexpr int FM = WM / 16, FN = WN / 16, KS = BK / 4;
    static constexpr int A_CPR = BK * (int)sizeof(T) / 16;    // 16-byte chunks per A row
    static constexpr int B_CPR = BN * (int)sizeof(T) / 16;    // 16-byte chunks per B row
    static constexpr int A_SLOTS = BM * A_CPR, B_SLOTS = BK * B_CPR;
    static constexpr int STAGE_SLOTS = A_SLOTS + B_SLOTS;
    static constexpr int STAGE_ELEMS = STAGE_SLOTS * VEC;
    static constexpr int DIRECT_ELEMS = STAGES * STAGE_ELEMS;
    static constexpr int LDS_ELEMS = DIRECT_ELEMS > Fallback::LDS_ELEMS ? DIRECT_ELEMS : Fallback::LDS_ELEMS;
    static constexpr int LOADS = STAGE_SLOTS / NT;
    static constexpr int A_ROWS_PER_256 = 256 / (A_CPR * 16) > 0 ? 256 / (A_CPR * 16) : 1;
    // bytes between the lane groups of one B read: 32 lanes per pass for
    // binary64 (two groups, 128 B apart), 64 lanes for FP32 (four, 64 B apart)
    static constexpr int B_GROUP_SHIFT = sizeof(T) == 8 ? 8 : 4;   // in chunks
    static constexpr int B_GROUPS = sizeof(T) == 8 ? 2 : 4;
    static_assert(STAGE_SLOTS % NT == 0 && A_SLOTS % 64 == 0, "stage must split into whole wave loads");
    static_assert(A_CPR >= 1 && (A_CPR & (A_CPR - 1)) == 0, "A row chunks");
    static_assert(B_CPR % (B_GROUP_SHIFT * B_GROUPS) == 0 || B_CPR >= B_GROUP_SHIFT * B_GROUPS, "B row chunks");
    static_assert(STAGES >= 2 && STAGES <= 4, "stages");

    typedef typename MfmaOp<T>::acc_t acc_t;

    static __device__ __forceinline__ int swz_a(int row, int c) { return c ^ ((row / A_ROWS_PER_256) & (A_CPR - 1)); }
    static __device__ __forceinline__ int swz_b(int row, int c) {
        return c ^ (((row / KS) & (B_GROUPS - 1)) * B_GROUP_SHIFT);
    }

    // Per-lane byte offset of each ring load within the A (BM x BK) or B
    // (BK x BN) slice of a K step, relative to the slice's first element.
    static __device__ __forceinline__ void sources(int64_t lda, int64_t ldb, int64_t M, int64_t N, int64_t m0,
                                                   int64_t n0, uint32_t (&voff)[LOADS]) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int P = (j * NWAVES + wave) * 64 + lane;
            if (P < A_SLOTS) {
                const int row = P / A_CPR;
                const int c = swz_a(row, P % A_CPR);
                int64_t gr = m0 + row;
                gr = gr < M ? gr : M - 1;
                voff[j] = (uint32_t)(((gr - m0) * lda + c * VEC) * (int64_t)sizeof(T));
            } else {
                const int Q = P - A_SLOTS;
                const int row = Q / B_CPR;
                const int c = swz_b(row, Q % B_CPR);
                int64_t gc = n0 + c * VEC;
                // chunks past N re-read the last chunk holding valid columns
                const int64_t last = (N - 1) / VEC * VEC;
                gc = gc < N ? gc : last;
                voff[j] = (uint32_t)((row * ldb + (gc - n0)) * (int64_t)sizeof(T));
            }
        }
    }

    // The ring loads of one K step as buffer loads into LDS, through one
    // buffer resource per operand based at the slice.  (Buffer rather than
    // global LDS loads: the compiler treats a pending global load into LDS as
    // a flat access and then waits for every outstanding LDS read at each
    // fragment use; with buffer loads its waits stay per sub-step.)
    static __device__ __forceinline__ void issue(const T *A_slice, const T *B_slice, const uint32_t (&voff)[LOADS],
                                                 T *buf, int32_t a_bytes = 0x7fffffff, int32_t b_bytes = 0x7fffffff) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const __amdgpu_buffer_rsrc_t ra = rsrc(A_slice, a_bytes), rb = rsrc(B_slice, b_bytes);
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            // wave-uniform (A_SLOTS % 64 == 0); per load when A fills whole loads
            const bool is_a = A_SLOTS % NT == 0 ? j < A_SLOTS / NT : (j * NWAVES + wave) * 64 < A_SLOTS;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(is_a ? ra : rb, (mm_lvoid *)(buf + (j * NWAVES + wave) * 64 * VEC),
                                                     16, voff[j], 0, 0, 0);
        }
    }

    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const T *base, int32_t bytes = 0x7fffffff) {
        // raw buffer (stride 0), byte range `bytes` (loads past it read zero),
        // gfx9 default format word
        return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, bytes, 0x00020000);
    }

    // The last K step of a K that is not a multiple of BK (`krem` valid
    // entries): the ring loads of that step run with byte ranges ending at the
    // last valid element of each operand, so rows of B past K -- and the
    // chunks of A's last row past K -- read as zero; A's other rows bring the
    // next row's leading elements (or padding) past K, which each lane clears
    // in the LDS slots it filled itself, after its loads have landed and
    // before the barrier that publishes the step.
    static __device__ __forceinline__ void clear_a_tail(T *buf, int krem) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int P = (j * NWAVES + wave) * 64 + lane;
            if (P < A_SLOTS) {
                const int c = swz_a(P / A_CPR, P % A_CPR);
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (c * VEC + e >= krem) buf[P * VEC + e] = T(0);
            }
        }
    }

    // Fragments of one stage, read one MFMA sub-step ahead of the MFMAs that
    // use them.  Sub-step s needs b[.][s] and, at the start of each 16-byte A
    // chunk (s % PER == 0), that chunk of a[.][.]; LDS returns reads in issue
    // order, so the MFMAs of sub-step s wait only for the reads of s, not for
    // those of s + 1 issued before them.  `next` (the ring load of a later
    // stage) is issued after the first reads, off the path to the first MFMA.
    static constexpr int PER = 16 / (int)sizeof(T);
    static constexpr int CH = KS * (int)sizeof(T) / 16 > 0 ? KS * (int)sizeof(T) / 16 : 1;
    static_assert(KS >= PER && CH * PER == KS, "a lane group's K run must be whole 16-byte A chunks");

    static __device__ __forceinline__ void read_sub(const T *As, const T *Bs, int s, int wm, int wn, int li, int q,
                                                    T (&a)[FM][KS], T (&b)[FN][KS]) {
        typedef T v_t __attribute__((ext_vector_type(PER)));
        // B first: the first MFMAs of the sub-step need all of b[.][s] but
        // only the first A chunk
        const int row = q * KS + s;
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int col = wn * WN + fn * 16 + li;
            b[fn][s] = Bs[row * BN + swz_b(row, col / VEC) * VEC + col % VEC];
        }
        if (s % PER == 0) {
            // A: lane group q holds k = q*KS .. q*KS+KS-1 of its row, CH chunks
            const int h = s / PER;
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int arow = wm * WM + fm * 16 + li;
                const v_t v = *reinterpret_cast<const v_t *>(As + arow * BK + swz_a(arow, q * CH + h) * VEC);
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    if (h * PER + e < KS) a[fm][h * PER + e] = v[e];
            }
        }
    }

    template <typename Next>
    static __device__ __forceinline__ void compute(const T *stage, acc_t (&acc)[FM][FN], Next next) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
        const T *As = stage, *Bs = stage + A_SLOTS * VEC;
        T a[FM][KS], b[FN][KS];
        read_sub(As, Bs, 0, wm, wn, li, q, a, b);
        __builtin_amdgcn_sched_barrier(0);
        next();
        // (no raised priority around the MFMAs here: measured 2-5% slower in
        // this body, where the ring needs no LDS stores between the bursts)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS) read_sub(As, Bs, s + 1, wm, wn, li, q, a, b);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = MfmaOp<T>::mma(a[fm][s], b[fn][s], acc[fm][fn]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    template <int N_>
    static __device__ __forceinline__ void wait_vm() {
        __builtin_amdgcn_s_waitcnt((N_ & 15) | (7 << 4) | (15 << 8) | ((N_ >> 4) << 14));
    }

    // Operands the ring takes: N of at least one vector, bases aligned to the
    // element, and a slice's per-lane offsets within the 31-bit buffer range.
    // Leading dimensions need not be multiples of the vector nor bases
    // 16-byte aligned: the direct-to-LDS load fetches its 16 bytes at any
    // element-aligned offset (checked on the GPU with an in-bounds probe at
    // offsets of 0-3 floats), so a row that starts mid-vector is read as
    // chunks that start there; a chunk that runs past the end of a row brings
    // the next row's first elements, which only meet the columns of B past N
    // (never stored) or, past K, the LDS slots the ragged last step clears.
    static __device__ __forceinline__ bool eligible(const T *A, int64_t lda, const T *B, int64_t ldb, int64_t N,
                                                    int64_t K) {
        const int64_t a_span = ((int64_t)(BM - 1) * lda + BK) * (int64_t)sizeof(T);
        const int64_t b_span = ((int64_t)(BK - 1) * ldb + BN) * (int64_t)sizeof(T);
        (void)K;
        return N >= VEC && ((uintptr_t)A % sizeof(T) == 0) && ((uintptr_t)B % sizeof(T) == 0) &&
               a_span < 0x7fffffff && b_span < 0x7fffffff;
    }

    // The K loop over the ring.  RAGGED (K not a multiple of BK, or N not a
    // multiple of the vector): the last step's loads run through byte ranges
    // ending at the operands' last valid elements -- so no load reaches past
    // B's last row, which may end before the vector that holds column N-1
    // does -- and A's columns past K are cleared (clear_a_tail).
    template <bool RAGGED>
    static __device__ __forceinline__ void ring(const T *A_tile, int64_t lda, const T *B_tile, int64_t ldb, int64_t M,
                                                int64_t N, int64_t K, int64_t m0, int64_t n0,
                                                const uint32_t (&voff)[LOADS], acc_t (&acc)[FM][FN], T *smem) {
        const int64_t nkt = (K + BK - 1) / BK;
        const int krem = (int)(K - (nkt - 1) * BK);   // valid entries of the last step, 1..BK
        // byte ranges of the last step, from its slices' bases (every lane
        // offset is below 2^31, so a longer range is capped there)
        auto cap = [](int64_t bytes) { return (int32_t)(bytes < 0x7fffffff ? bytes : 0x7fffffff); };
        const int32_t a_last = RAGGED ? cap(((M - 1 - m0) * lda + krem) * (int64_t)sizeof(T)) : 0x7fffffff;
        const int32_t b_last = RAGGED ? cap(((int64_t)(krem - 1) * ldb + (N - n0)) * (int64_t)sizeof(T)) : 0x7fffffff;
        auto stage = [&](int64_t s_) {
            if (RAGGED && s_ == nkt - 1)
                issue(A_tile + s_ * BK, B_tile + s_ * BK * ldb, voff, smem + (s_ % STAGES) * STAGE_ELEMS, a_last, b_last);
            else
                issue(A_tile + s_ * BK, B_tile + s_ * BK * ldb, voff, smem + (s_ % STAGES) * STAGE_ELEMS);
        };
#pragma unroll
        for (int s = 0; s < STAGES - 1; ++s)
            if (s < nkt) stage(s);
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const int64_t later = (nkt - 1 - kt) < (STAGES - 2) ? (nkt - 1 - kt) : (STAGES - 2);
            if (later >= 2) wait_vm<2 * LOADS>();
            else if (later == 1) wait_vm<LOADS>();
            else wait_vm<0>();
            if (RAGGED && kt == nkt - 1 && krem < BK) clear_a_tail(smem + (kt % STAGES) * STAGE_ELEMS, krem);
            // stage kt is in LDS for every thread, the buffer of step kt-1 is
            // no longer read: a bare barrier (a fenced one would also wait for
            // the later stages' loads)
            __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
            __builtin_amdgcn_s_barrier();
            compute(smem + (kt % STAGES) * STAGE_ELEMS, acc, [&] {
                const int64_t kn = kt + STAGES - 1;
                if (kn < nkt) stage(kn);
            });
        }
    }

    static __device__ __forceinline__ void run(const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                               int64_t ldb, T *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                               int64_t K, int64_t tm, int64_t tn, bool vec_ok, T *smem) {
        if (!eligible(A, lda, B, ldb, N, K)) {
            Fallback::run(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, vec_ok, smem);
            return;
        }
        const int64_t m0 = tm * BM, n0 = tn * BN;
        acc_t acc[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = acc_t{0, 0, 0, 0};
        uint32_t voff[LOADS];
        sources(lda, ldb, M, N, m0, n0, voff);
        // K a multiple of BK: the plain ring; otherwise the ring with a
        // range-limited last step (two loops, so the common one carries none
        // of the last step's bookkeeping: measured 1% on the 8192 product)
        if (K % BK == 0 && N % VEC == 0) ring<false>(A + m0 * lda, lda, B + n0, ldb, M, N, K, m0, n0, voff, acc, smem);
        else ring<true>(A + m0 * lda, lda, B + n0, ldb, M, N, K, m0, n0, voff, acc, smem);
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
                    const int64_t r = m0 + wm * WM + fm * 16 + MfmaOp<T>::row(q, v);
                    const int64_t c = n0 + wn * WN + fn * 16 + li;
                    if (r < M && c < N) ((gptr<T>)C)[r * ldc + c] = acc[fm][fn][v];
                }
        __syncthreads();   // LDS may be refilled by the next tile of a persistent workgroup
    }
};

// Variant selector: S = 0: register-staged tile; S = 10 + b: direct-to-LDS
// ring of b buffers.
template <typename T, int BM, int BN, int BK, int WM, int WN, int S, bool DIRECT = (S >= 10)>
struct TileSel {
    typedef TileGemm<T, BM, BN, BK, WM, WN> type;
};
template <typename T, int BM, int BN, int BK, int WM, int WN, int S>
struct TileSel<T, BM, BN, BK, WM, WN, S, true> {
    typedef TileGemmDirect<T, BM, BN, BK, WM, WN, S - 10> type;
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
