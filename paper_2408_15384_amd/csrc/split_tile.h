// Workgroup tile of the split-precision product on the bfloat16 matrix cores
// (shared by the single-problem and the grouped kernels).
//
// C = sum over the method's plane pairs (p, q) of A_p . B_q with
// v_mfma_f32_16x16x32_bf16, two FP32 accumulator sets per output block (the
// leading A_0.B_0 product and the sum of the corrections), recombined per entry
// in binary64.  A planes are M x K row-major, B planes N x K (transposed), so
// both operands are k-contiguous and each MFMA fragment is one 16-byte LDS read.
//
// MFMA lane layout (16x16x32 bf16, measured on gfx950): lane l supplies
// A[l%16][8*(l/16) .. +7] and B[8*(l/16) .. +7][l%16] and receives
// D[4*(l/16)+v][l%16], v = 0..3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "gptr.h"

namespace mm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// bfloat16 of x, round to nearest even (the gfx950 convert instruction).
__device__ __forceinline__ uint16_t split_bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float split_bf16_value(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// Element-aligned 16-byte FP32 load (the memory system runs in unaligned
// mode, so a vector wholly inside a row needs only element alignment).
typedef float f32x4_ea __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ f32x4 load_f32x4_ea(gptr<const float> p) {
    return *reinterpret_cast<gptr<const f32x4_ea>>(p);
}

// Split v[0..7] into its next bfloat16 plane in place (v keeps the leftover)
// and store the 8 values as one 16-byte store, or element by element where
// the chunk is not 16-byte aligned (vec false) or only n < 8 of it is inside
// the row.
__device__ __forceinline__ void split_store_chunk(float (&v)[8], gptr<uint16_t> dst, int n, bool vec) {
    u16x8 h;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = split_bf16_bits(v[e]);
        v[e] = v[e] - split_bf16_value(h[e]);
    }
    if (vec && n == 8) {
        *reinterpret_cast<gptr<u16x8>>(dst) = h;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (e < n) dst[e] = h[e];
    }
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

template <int NPROD, int BM_, int BN_, int BK_, int WM_, int WN_, int STAGES_ = 1>
struct SplitTile {
    static constexpr bool FUSED = false;
    using Terms = SplitTerms<NPROD>;
    static constexpr int NP = Terms::NP;
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, STAGES = STAGES_;
    static constexpr int NWN = BN / WN;
    static constexpr int NWAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = NWAVES * 64;
    static constexpr int FM = WM / 16, FN = WN / 16;
    static constexpr int KSTEPS = BK / 32;
    // LDS rows hold BK bf16 with no padding; the 16-byte chunks of a row are
    // permuted (chunk ^ swz(row)) so that the 16 lanes of a fragment read (16
    // rows, one chunk) and of a store (whole rows) touch 16 distinct 16-byte
    // bank groups.
    static constexpr int LD = BK;
    static constexpr int A_PLANE = BM * LD, B_PLANE = BN * LD;
    static constexpr int STAGE = NP * (A_PLANE + B_PLANE);
    static constexpr int LDS_ELEMS = 2 * STAGE;
    static constexpr int VROW = BK / 8;               // 16-byte vectors per row
    static constexpr int ROWS_PER_256B = 256 / (VROW * 16) > 0 ? 256 / (VROW * 16) : 1;
    static __device__ __forceinline__ int swz(int row, int chunk) {
        return chunk ^ ((row / ROWS_PER_256B) & (VROW - 1));
    }
    static constexpr int A_VECS = NP * BM * VROW / NT;
    static constexpr int B_VECS = NP * BN * VROW / NT;
    static_assert(BK % 32 == 0, "BK multiple of 32");
    static_assert((NP * BM * VROW) % NT == 0 && (NP * BN * VROW) % NT == 0, "load split");

    // planes: base of plane 0, plane p at + p*pstride; rows x K k-contiguous.
    static __device__ __forceinline__ void load(u16x8 *regs, int nvec, gptr<const uint16_t> planes,
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
            gptr<const uint16_t> src = planes + p * pstride + gr * K + k0 + c;
            if (gr < nrows_total && vec_ok && k0 + c + 8 <= K) {
                regs[i] = *reinterpret_cast<gptr<const u16x8>>(src);
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
            *reinterpret_cast<u16x8 *>(lds + p * plane_elems + r * LD + swz(r, c / 8) * 8) = regs[i];
        }
    }

    static __device__ __forceinline__ bf16x8 frag(const uint16_t *lds, int row, int kofs) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(lds + row * LD + swz(row, kofs / 8) * 8));
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
        const gptr<const uint16_t> Ag = (gptr<const uint16_t>)Ap, Bg = (gptr<const uint16_t>)Bt;
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        if (STAGES == 1) {
            // One register stage: slice kt+1 is loaded while slice kt is multiplied.
            u16x8 ra[A_VECS], rb[B_VECS];
            const int64_t nkt = (K + BK - 1) / BK;
            load(ra, A_VECS, Ag, pa_stride, m0, M, K, 0, BM, vec_ok);
            load(rb, B_VECS, Bg, pb_stride, n0, N, K, 0, BN, vec_ok);
            store(smem, A_PLANE, ra, A_VECS, BM);
            store(smem + NP * A_PLANE, B_PLANE, rb, B_VECS, BN);
            __syncthreads();
            for (int64_t kt = 0; kt < nkt; ++kt) {
                const bool more = kt + 1 < nkt;
                if (more) {
                    load(ra, A_VECS, Ag, pa_stride, m0, M, K, (kt + 1) * BK, BM, vec_ok);
                    load(rb, B_VECS, Bg, pb_stride, n0, N, K, (kt + 1) * BK, BN, vec_ok);
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
        } else {
            // Global loads run two K steps ahead of the MFMAs (two register stages,
            // double-buffered LDS): slice kt+2 is requested while slice kt is
            // multiplied and slice kt+1 waits in registers for its LDS buffer.
            u16x8 ra0[A_VECS], rb0[B_VECS], ra1[A_VECS], rb1[B_VECS];
            const int64_t nkt = (K + BK - 1) / BK;
            load(ra0, A_VECS, Ag, pa_stride, m0, M, K, 0, BM, vec_ok);
            load(rb0, B_VECS, Bg, pb_stride, n0, N, K, 0, BN, vec_ok);
            if (nkt > 1) {
                load(ra1, A_VECS, Ag, pa_stride, m0, M, K, BK, BM, vec_ok);
                load(rb1, B_VECS, Bg, pb_stride, n0, N, K, BK, BN, vec_ok);
            }
            store(smem, A_PLANE, ra0, A_VECS, BM);
            store(smem + NP * A_PLANE, B_PLANE, rb0, B_VECS, BN);
            __syncthreads();
            for (int64_t kt = 0; kt < nkt; kt += 2) {
                // even step kt: register set 1 holds slice kt+1; refill set 0 with kt+2
                if (kt + 2 < nkt) {
                    load(ra0, A_VECS, Ag, pa_stride, m0, M, K, (kt + 2) * BK, BM, vec_ok);
                    load(rb0, B_VECS, Bg, pb_stride, n0, N, K, (kt + 2) * BK, BN, vec_ok);
                }
                compute(smem, smem + NP * A_PLANE, lead, corr);
                if (kt + 1 < nkt) {
                    store(smem + STAGE, A_PLANE, ra1, A_VECS, BM);
                    store(smem + STAGE + NP * A_PLANE, B_PLANE, rb1, B_VECS, BN);
                }
                __syncthreads();
                if (kt + 1 >= nkt) break;
                // odd step kt+1: set 0 holds slice kt+2; refill set 1 with kt+3
                if (kt + 3 < nkt) {
                    load(ra1, A_VECS, Ag, pa_stride, m0, M, K, (kt + 3) * BK, BM, vec_ok);
                    load(rb1, B_VECS, Bg, pb_stride, n0, N, K, (kt + 3) * BK, BN, vec_ok);
                }
                compute(smem + STAGE, smem + STAGE + NP * A_PLANE, lead, corr);
                if (kt + 2 < nkt) {
                    store(smem, A_PLANE, ra0, A_VECS, BM);
                    store(smem + NP * A_PLANE, B_PLANE, rb0, B_VECS, BN);
                }
                __syncthreads();
            }
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
                        if (c_is_f64) ((gptr<double>)(double *)C)[r * ldc + c] = val;
                        else ((gptr<float>)(float *)C)[r * ldc + c] = (float)val;
                    }
                }
    }
};


// ---------------------------------------------------------------------------
// Direct-to-LDS variant: buffer_load_dwordx4 ... lds moves each 16-byte chunk of
// the planes straight into LDS (no staging registers), into a ring of STAGES
// LDS buffers, so the loads of K steps kt+1 .. kt+STAGES-1 are in flight while
// step kt is multiplied.  One wave-instruction fills 64 consecutive 16-byte
// LDS slots (lane i -> slot i); each lane fetches whichever global chunk the
// swizzled layout puts in its slot.  Rows past M (or N) are clamped to the
// last row: they only feed entries of C that are not stored.  K is a
// multiple of 32 (the planes are zero-padded), so no K-tail checks remain.
//
// IL (interleaved planes, 2-plane method only): a row of the planes holds, for
// each 32-element K block, the block of plane 0 and then of plane 1, so one K
// step of a row is one contiguous 128-byte line (one L2 request) instead of
// two 64-byte pieces; an LDS row then holds both planes' 8 chunks.
typedef __attribute__((address_space(3))) void mm_lds_void;

template <int NPROD, int BM_, int BN_, int WM_, int WN_, int STAGES_, bool IL_ = false>
struct SplitTileDirect {
    static constexpr bool FUSED = false;
    static constexpr bool IL = IL_;
    using Terms = SplitTerms<NPROD>;
    static constexpr int NP = Terms::NP;
    static constexpr int BM = BM_, BN = BN_, BK = 32, WM = WM_, WN = WN_;
    // The ring holds STAGES_ buffers when they fit in 152 KiB of LDS (room is
    // left for the grouped kernel's owner table), else as many as fit: a
    // variant asks for a depth, and the 3-plane method may get a shallower one.
    static constexpr int STAGE_BYTES = NP * (BM + BN) * BK * 2;
    static constexpr int LDS_CAP = 152 * 1024;
    static constexpr int STAGES = STAGES_ * STAGE_BYTES <= LDS_CAP ? STAGES_ : LDS_CAP / STAGE_BYTES;
    static constexpr int NWN = BN / WN;
    static constexpr int NWAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = NWAVES * 64;
    static constexpr int FM = WM / 16, FN = WN / 16;
    static constexpr int ROWS = BM + BN;                 // rows of one plane in a stage: A rows, then B rows
    static constexpr int PLANE_CHUNKS = ROWS * 4;        // 4 chunks of 16 bytes per 32-element row
    static constexpr int STAGE_CHUNKS = NP * PLANE_CHUNKS;
    static constexpr int STAGE_ELEMS = STAGE_CHUNKS * 8;
    static constexpr int LDS_ELEMS = STAGES * STAGE_ELEMS;
    static constexpr int LOADS = STAGE_CHUNKS / NT;      // load instructions per thread per stage
    static_assert(STAGE_CHUNKS % NT == 0, "stage must split evenly over the threads");
    static_assert(STAGES >= 2 && STAGES <= 4, "stages");
    // one load instruction (64 slots = 16 rows) never straddles planes or the A/B boundary
    static_assert(BM % 16 == 0 && BN % 16 == 0, "tile sides in whole 16-row groups");
    static_assert(!IL || NP == 2, "interleaved planes are for the 2-plane method");
    // elements of a plane row per K step: one block per plane when interleaved
    static constexpr int KSTEP = IL ? NP * BK : BK;

    // Interleaved LDS rows are 128 bytes (8 chunks), chunk ^ (row/2 mod 8).
    // Separate planes use 64-byte rows placed so that the 16 rows of a
    // fragment read hit the same 16-byte bank groups as that layout: within a
    // 16-row group, 128-byte line l holds rows l and l + 8 (halves), and a
    // row's 4 chunks sit at chunk ^ (row/2 mod 4).  Both read without bank
    // conflicts (the plain 64-byte rows with chunk ^ (row/4 mod 4) took twice
    // the LDS cycles per read).
    static __device__ __forceinline__ int swz8(int row, int chunk) { return chunk ^ ((row >> 1) & 7); }
    static __device__ __forceinline__ int row_elem(int row, int chunk) {
        return (row >> 4) * 512 + (row & 7) * 64 + ((row >> 3) & 1) * 32 + ((chunk ^ ((row >> 1) & 3)) * 8);
    }

    // Source of each load instruction at k = 0 (a K step adds k0): the 64
    // lanes of one instruction fill 16 consecutive rows of one plane (8 rows
    // of the interleaved pair), so the instruction reads through a buffer
    // resource based at the first of those rows (wave-uniform) and each lane
    // adds a 32-bit byte offset below 16 * Kp * 2, which the entry points keep
    // below 2^31 (K < 2^26).

    static __device__ __forceinline__ void sources(const uint16_t *__restrict__ Ap, int64_t pa_stride,
                                                   const uint16_t *__restrict__ Bt, int64_t pb_stride, int64_t Kp,
                                                   int64_t m0, int64_t n0, int64_t M, int64_t N,
                                                   const uint16_t *(&base)[LOADS], uint32_t (&voff)[LOADS]) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if constexpr (IL) {
            // an instruction fills 8 whole LDS rows (both planes); the lane
            // in slot s of row r fetches logical chunk swz8(r, s), which sits
            // at element 8 * chunk of the row's K block
#pragma unroll
            for (int j = 0; j < LOADS; ++j) {
                const int row0 = (j * NWAVES + wave) * 8;   // wave-uniform
                const int row = row0 + (lane >> 3);
                const int c = swz8(row, lane & 7);
                const bool is_a = row0 < BM;
                const int64_t first = is_a ? m0 + row0 : n0 + (row0 - BM);
                const int64_t lim = is_a ? M : N;
                const int64_t g0 = first < lim ? first : lim - 1;
                int64_t gr = first + (lane >> 3);
                gr = gr < lim ? gr : lim - 1;
                base[j] = (is_a ? Ap : Bt) + g0 * (NP * Kp);
                voff[j] = (uint32_t)(((gr - g0) * NP * Kp + c * 8) * 2);
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int P0 = (j * NWAVES + wave) * 64;         // first slot of this instruction (wave-uniform)
            const int plane = P0 / PLANE_CHUNKS;
            const int row0 = (P0 - plane * PLANE_CHUNKS) >> 2;
            // slot i of the 64 (16 rows, all of A or all of B): line i/8 of
            // the 16-row group, half (i/4) % 2, chunk slot i % 4 (row_elem)
            const int row = row0 + (lane >> 3) + ((lane >> 2) & 1) * 8;
            const int c = (lane & 3) ^ ((row >> 1) & 3);     // logical chunk stored in this lane's slot
            const bool is_a = row0 < BM;
            const int64_t first = is_a ? m0 + row0 : n0 + (row0 - BM);
            const int64_t lim = is_a ? M : N;
            const int64_t g0 = first < lim ? first : lim - 1;
            int64_t gr = first + (row - row0);
            gr = gr < lim ? gr : lim - 1;
            base[j] = (is_a ? Ap + plane * pa_stride : Bt + plane * pb_stride) + g0 * Kp;
            voff[j] = (uint32_t)(((gr - g0) * Kp + c * 8) * 2);
        }
    }

    // Issue the loads of the K step at k0 into LDS buffer `buf`: instruction j
    // of wave w fills the 64 slots of block j*NWAVES + w.  (Buffer rather than
    // global LDS loads: the compiler treats a pending global load into LDS as
    // a flat access and then waits for every outstanding LDS read at each
    // fragment use; with buffer loads its waits follow the fragments.)
    static __device__ __forceinline__ void issue(const uint16_t *const (&base)[LOADS], const uint32_t (&voff)[LOADS],
                                                 int64_t k0, uint16_t *buf) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const __amdgpu_buffer_rsrc_t r =
                __builtin_amdgcn_make_buffer_rsrc((void *)(base[j] + k0), (short)0, 0x7fffffff, 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (mm_lds_void *)(buf + (j * NWAVES + wave) * 64 * 8), 16, voff[j],
                                                     0, 0, 0);
        }
    }

    static __device__ __forceinline__ bf16x8 frag(const uint16_t *stage, int plane, int row, int q) {
        if constexpr (IL)
            return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(stage + row * (NP * 32) +
                                                                               swz8(row, plane * 4 + q) * 8));
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(stage + plane * PLANE_CHUNKS * 8 +
                                                                           row_elem(row, q)));
    }

    // Plane whose fragments are read just before the products of term t (one
    // plane ahead of the highest plane term t uses), or -1.
    static constexpr int read_before(int t) {
        int last = 0;   // planes 0..last are read before term t (plane 0 up front)
        for (int u = 0; u < t; ++u) {
            const int want = (Terms::pa[u] > Terms::pb[u] ? Terms::pa[u] : Terms::pb[u]) + 1;
            if (want < NP && want > last) last = want;
        }
        const int want = (Terms::pa[t] > Terms::pb[t] ? Terms::pa[t] : Terms::pb[t]) + 1;
        return want < NP && want > last ? want : -1;
    }

    // The products of one stage.  With 64x64 wave tiles the fragments are
    // read plane by plane, one plane ahead of the products that use them, so
    // a product waits only for its own planes' reads, and `next` (the ring
    // load of a later stage) is issued after the first plane's reads.  Each
    // accumulator takes the terms in their fixed order either way.
    template <typename Next>
    static __device__ __forceinline__ void compute(const uint16_t *stage, f32x4 (&lead)[FM][FN],
                                                   f32x4 (&corr)[FM][FN], Next next) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
        bf16x8 a[NP][FM], b[NP][FN];
        auto read_plane = [&](int p) {
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) b[p][fn] = frag(stage, p, BM + wn * WN + fn * 16 + li, q);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) a[p][fm] = frag(stage, p, wm * WM + fm * 16 + li, q);
        };
        if constexpr (FM * FN < 16) {
            // small wave tiles: few fragments per plane; the compiler's own
            // order measured faster (split3 64x64 at 8192: 5.9 -> 5.5 ms)
            next();
#pragma unroll
            for (int p = 0; p < NP; ++p) read_plane(p);
        } else {
            read_plane(0);
            __builtin_amdgcn_sched_barrier(0);
            next();
        }
#pragma unroll
        for (int t = 0; t < Terms::n; ++t) {
            if constexpr (FM * FN >= 16) {
                if (read_before(t) >= 0) read_plane(read_before(t));
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) {
                    if (t == 0)
                        lead[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][fm], b[0][fn], lead[fm][fn], 0, 0, 0);
                    else
                        corr[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[Terms::pa[t]][fm], b[Terms::pb[t]][fn],
                                                                               corr[fm][fn], 0, 0, 0);
                }
            if constexpr (FM * FN >= 16) __builtin_amdgcn_sched_barrier(0);
        }
    }

    // vmcnt(n) with the other counters left unconstrained (gfx9 encoding).
    template <int N_>
    static __device__ __forceinline__ void wait_vm() {
        __builtin_amdgcn_s_waitcnt((N_ & 15) | (7 << 4) | (15 << 8) | ((N_ >> 4) << 14));
    }

    // Same contract as SplitTile::run; K must be a multiple of 32 and the
    // plane rows K long.  vec_ok is implied by the padded layout.
    static __device__ __forceinline__ void run(const uint16_t *__restrict__ Ap, int64_t pa_stride,
                                               const uint16_t *__restrict__ Bt, int64_t pb_stride, void *C,
                                               int64_t ldc, int c_is_f64, int64_t M, int64_t N, int64_t K, int64_t tm,
                                               int64_t tn, bool, uint16_t *smem) {
        const int64_t m0 = tm * BM, n0 = tn * BN;
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        const int64_t nkt = K / BK;
        const uint16_t *base[LOADS];
        uint32_t voff[LOADS];
        sources(Ap, pa_stride, Bt, pb_stride, K, m0, n0, M, N, base, voff);
#pragma unroll
        for (int s = 0; s < STAGES - 1; ++s)
            if (s < nkt) issue(base, voff, (int64_t)s * KSTEP, smem + s * STAGE_ELEMS);
        for (int64_t kt = 0; kt < nkt; ++kt) {
            // stage kt has landed once at most the later stages' loads are pending
            const int64_t later = (nkt - 1 - kt) < (STAGES - 2) ? (nkt - 1 - kt) : (STAGES - 2);
            if (later >= 2) wait_vm<2 * LOADS>();
            else if (later == 1) wait_vm<LOADS>();
            else wait_vm<0>();
            // Every thread's part of stage kt is in LDS (the wait above) and the
            // buffer of step kt-1 is no longer read.  A bare barrier: a fenced
            // __syncthreads would also wait for the later stages' loads.
            __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));   // lgkmcnt(0) only
            __builtin_amdgcn_s_barrier();
            compute(smem + (kt % STAGES) * STAGE_ELEMS, lead, corr, [&] {
                if (kt + STAGES - 1 < nkt)
                    issue(base, voff, (kt + STAGES - 1) * KSTEP, smem + ((kt + STAGES - 1) % STAGES) * STAGE_ELEMS);
            });
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
                        if (c_is_f64) ((gptr<double>)(double *)C)[r * ldc + c] = val;
                        else ((gptr<float>)(float *)C)[r * ldc + c] = (float)val;
                    }
                }
        __syncthreads();   // LDS may be refilled by the next tile of a persistent workgroup
    }
};

// ---------------------------------------------------------------------------
// Fused form: the tile reads the FP32 operands themselves and splits them on
// the way into LDS, so no plane pass runs before the product and no plane
// workspace exists.  Each K step of 32 is loaded into registers while the
// previous one is multiplied (as SplitTile with one register stage); a
// thread owns units of 8 consecutive k of one row of A or one column of B,
// splits the 8 values into the method's bfloat16 planes exactly as the plane
// pass does (h = bf16(x), x -= h, plane by plane, in FP32) and writes each
// plane's 8 values as one 16-byte chunk of the same swizzled LDS layout.
// The planes, the MFMA sequence and therefore the result are identical to
// SplitTile's on pre-split planes.  A is read along rows (two element-aligned
// 16-byte loads per unit wholly inside K, whatever lda and the base), B down
// its columns with lanes along N, so every load instruction is coalesced.
// Entries past M, N or K read as zero.
template <int NPROD, int BM_, int BN_, int WM_, int WN_>
struct SplitTileFused : SplitTile<NPROD, BM_, BN_, 32, WM_, WN_, 1> {
    static constexpr bool FUSED = true;
    using Base = SplitTile<NPROD, BM_, BN_, 32, WM_, WN_, 1>;
    using Base::BM; using Base::BN; using Base::BK; using Base::WM; using Base::WN;
    using Base::NP; using Base::NWN; using Base::NWAVES; using Base::NT; using Base::FM; using Base::FN;
    using Base::LD; using Base::A_PLANE; using Base::B_PLANE; using Base::STAGE; using Base::LDS_ELEMS;
    static constexpr int CHUNKS = BK / 8;                // 8-element units per row
    static constexpr int A_UNITS = BM * CHUNKS / NT;     // units per thread per K step
    static constexpr int B_UNITS = BN * CHUNKS / NT;
    static_assert((BM * CHUNKS) % NT == 0 && (BN * CHUNKS) % NT == 0, "units must split evenly");

    static __device__ __forceinline__ void load_a(float (&ra)[A_UNITS][8], gptr<const float> A, int64_t lda,
                                                  int64_t m0, int64_t M, int64_t K, int64_t k0) {
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            const int64_t r = m0 + u / CHUNKS;
            const int64_t k = k0 + (u % CHUNKS) * 8;
            gptr<const float> p = A + r * lda + k;
            if (r < M && k + 8 <= K) {
                // element-aligned 16-byte loads: any lda and base (unaligned mode)
                typedef f32x4 f32x4_ua __attribute__((aligned(4)));
                const f32x4 x = *reinterpret_cast<gptr<const f32x4_ua>>(p);
                const f32x4 y = *reinterpret_cast<gptr<const f32x4_ua>>(p + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ra[i][e] = x[e];
                    ra[i][4 + e] = y[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) ra[i][e] = (r < M && k + e < K) ? p[e] : 0.f;
            }
        }
    }

    static __device__ __forceinline__ void load_b(float (&rb)[B_UNITS][8], gptr<const float> B, int64_t ldb,
                                                  int64_t n0, int64_t N, int64_t K, int64_t k0) {
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            const int64_t n = n0 + u % BN;
            const int64_t k = k0 + (u / BN) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[i][e] = (n < N && k + e < K) ? B[(k + e) * ldb + n] : 0.f;
        }
    }

    // Split 8 values into the planes and write them to LDS: plane p of the
    // operand starts at base + p * plane_elems; (row, chunk) is the unit.
    static __device__ __forceinline__ void put(uint16_t *base, int plane_elems, int row, int chunk,
                                               const float (&v)[8]) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = v[e];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            u16x8 h;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                h[e] = split_bf16_bits(x[e]);
                x[e] = x[e] - split_bf16_value(h[e]);
            }
            *reinterpret_cast<u16x8 *>(base + p * plane_elems + row * LD + Base::swz(row, chunk) * 8) = h;
        }
    }

    static __device__ __forceinline__ void put_all(uint16_t *stage, const float (&ra)[A_UNITS][8],
                                                   const float (&rb)[B_UNITS][8]) {
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            put(stage, A_PLANE, u / CHUNKS, u % CHUNKS, ra[i]);
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            put(stage + NP * A_PLANE, B_PLANE, u % BN, u / BN, rb[i]);
        }
    }

    // Tile (tm, tn) of C = A.B for FP32 A (M x K, row-major, lda) and B
    // (K x N, row-major, ldb); any lda, ldb and base alignment.
    static __device__ __forceinline__ void run_fused(const float *A_, int64_t lda, const float *B_, int64_t ldb,
                                                     void *C, int64_t ldc, int c_is_f64, int64_t M, int64_t N,
                                                     int64_t K, int64_t tm, int64_t tn, uint16_t *smem) {
        const int64_t m0 = tm * BM, n0 = tn * BN;
        const gptr<const float> A = (gptr<const float>)A_, B = (gptr<const float>)B_;
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        float ra[A_UNITS][8], rb[B_UNITS][8];
        const int64_t nkt = (K + BK - 1) / BK;
        if (nkt > 0) {
            load_a(ra, A, lda, m0, M, K, 0);
            load_b(rb, B, ldb, n0, N, K, 0);
            put_all(smem, ra, rb);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const bool more = kt + 1 < nkt;
            if (more) {
                load_a(ra, A, lda, m0, M, K, (kt + 1) * BK);
                load_b(rb, B, ldb, n0, N, K, (kt + 1) * BK);
            }
            const uint16_t *cur = smem + (kt & 1) * STAGE;
            Base::compute(cur, cur + NP * A_PLANE, lead, corr);
            if (more) put_all(smem + ((kt + 1) & 1) * STAGE, ra, rb);
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
                    const int64_t r = m0 + wm * WM + fm * 16 + q * 4 + v;
                    const int64_t c = n0 + wn * WN + fn * 16 + li;
                    if (r < M && c < N) {
                        const double val = (double)lead[fm][fn][v] + (double)corr[fm][fn][v];
                        if (c_is_f64) ((gptr<double>)(double *)C)[r * ldc + c] = val;
                        else ((gptr<float>)(float *)C)[r * ldc + c] = (float)val;
                    }
                }
    }
};

// ---------------------------------------------------------------------------
// Fused form with a register ring and buffer loads.  The same planes, LDS
// layout, MFMA sequence and recombination as SplitTileFused (so the same
// bits), with a cheaper and deeper load side:
//  * loads are raw buffer loads through a resource based at the K step's
//    slice (scalar), each lane's byte offsets computed once per tile, so a K
//    step spends no vector instructions on addresses;
//  * entries past the matrix read as zero without vector masking: rows of A
//    past M and columns of B past N get an offset beyond the resource's
//    range (the hardware returns zero for those), as do rows of B past K
//    (they lie beyond the last valid byte); only the A columns past K of
//    the last K step are cleared in registers;
//  * RS K steps are in flight in registers: step kt + RS is requested while
//    step kt is multiplied;
//  * bfloat16 planes are made two values at a time (one packed convert per
//    pair, the pair's leftovers by subtraction).
// Tiles whose per-lane offsets would not fit 31 bits run SplitTileFused.
template <int NPROD, int BM_, int BN_, int WM_, int WN_, int RS_, bool PAIRED_ = false>
struct SplitTileFusedRing : SplitTileFused<NPROD, BM_, BN_, WM_, WN_> {
    using Fused = SplitTileFused<NPROD, BM_, BN_, WM_, WN_>;
    using Base = typename Fused::Base;
    static constexpr bool FUSED = true;
    using Base::BM; using Base::BN; using Base::BK; using Base::WM; using Base::WN;
    using Base::NP; using Base::NWN; using Base::NWAVES; using Base::NT; using Base::FM; using Base::FN;
    using Base::LD; using Base::A_PLANE; using Base::B_PLANE; using Base::STAGE; using Base::LDS_ELEMS;
    static constexpr int RS = RS_;
    // Waves per SIMD the kernels around this tile are compiled for: as many
    // workgroups as the CU's LDS holds (160 KiB, less 64 bytes of kernel
    // state), so the register budget never lowers the occupancy LDS allows.
    static constexpr int WAVES = [] {
        const int wgs = (160 * 1024) / (LDS_ELEMS * 2 + 64);
        const int w = wgs * NWAVES / 4;
        return w < 1 ? 1 : (w > 4 ? 4 : w);
    }();
    // PAIRED: rows r and r + 8 of each 16-row group share one 128-byte LDS
    // line (chunk ^ (row/2 mod 4)), so the 16 rows of a fragment read cover
    // all banks once; otherwise SplitTile's 64-byte rows.
    static constexpr bool PAIRED = PAIRED_;
    static constexpr int CHUNKS = BK / 8;                // 8-element units per 32-wide row

    // Element offset of (row, 16-byte chunk) within a plane.
    static __device__ __forceinline__ int lds_elem(int row, int chunk) {
        if constexpr (PAIRED)
            return (row >> 4) * 512 + (row & 7) * 64 + ((row >> 3) & 1) * 32 + ((chunk ^ ((row >> 1) & 3)) * 8);
        return row * LD + Base::swz(row, chunk) * 8;
    }

    static __device__ __forceinline__ bf16x8 frag(const uint16_t *plane, int row, int chunk) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(plane + lds_elem(row, chunk)));
    }

    // The products of one K step: SplitTile::compute's sequence (terms in
    // order, two accumulator sets) on this tile's LDS layout.
    static __device__ __forceinline__ void compute(const uint16_t *As, const uint16_t *Bs, f32x4 (&lead)[FM][FN],
                                                   f32x4 (&corr)[FM][FN]) {
        using Terms = typename Base::Terms;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / NWN, wn = wave % NWN;
        const int li = lane & 15, q = lane >> 4;
#pragma unroll
        for (int t = 0; t < Terms::n; ++t) {
            bf16x8 a[FM], b[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) a[fm] = frag(As + Terms::pa[t] * A_PLANE, wm * WM + fm * 16 + li, q);
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) b[fn] = frag(Bs + Terms::pb[t] * B_PLANE, wn * WN + fn * 16 + li, q);
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
    static constexpr int A_UNITS = BM * CHUNKS / NT;
    static constexpr int B_UNITS = BN * CHUNKS / NT;
    static_assert(RS >= 1 && RS <= 4, "register stages");
    static_assert((BM * CHUNKS) % NT == 0 && (BN * CHUNKS) % NT == 0, "units must split evenly");
    // byte offset that lies beyond every resource range used here
    static constexpr uint32_t OOB = 0x80000000u;

    struct Regs {
        f32x4 a[A_UNITS][2];
        float b[B_UNITS][8];
    };

    // Per-lane byte offsets of one tile (relative to the K step's slice).
    struct Offs {
        uint32_t a[A_UNITS];
        uint32_t b[B_UNITS][8];
    };

    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float *base, int64_t bytes) {
        const int32_t n = bytes <= 0 ? 0 : (bytes >= 0x7fffffff ? 0x7fffffff : (int32_t)bytes);
        return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, n, 0x00020000);
    }

    // Whether the tile's lane offsets fit (wave-uniform).
    static __device__ __forceinline__ bool ring_ok(int64_t lda, int64_t ldb) {
        return ((int64_t)(BM - 1) * lda + BK) * 4 < 0x7fff0000LL && ((int64_t)(BK - 1) * ldb + BN) * 4 < 0x7fff0000LL;
    }

    static __device__ __forceinline__ void offsets(int64_t lda, int64_t ldb, int rows_left, int cols_left, Offs &o) {
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            const int r = u / CHUNKS, c = u % CHUNKS;
            o.a[i] = r < rows_left ? (uint32_t)(((int64_t)r * lda + c * 8) * 4) : OOB;
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            const int n = u % BN, kc = u / BN;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                o.b[i][e] = n < cols_left ? (uint32_t)(((int64_t)(kc * 8 + e) * ldb + n) * 4) : OOB;
        }
    }

    // Request K step kt of the tile whose A panel starts at Ap (row m0) and B
    // panel at Bp (column n0).
    static __device__ __forceinline__ void load(Regs &R, const Offs &o, const float *Ap, int64_t lda, const float *Bp,
                                                int64_t ldb, int rows_left, int cols_left, int64_t K, int64_t kt) {
        const int64_t k0 = kt * BK;
        const __amdgpu_buffer_rsrc_t ra = rsrc(Ap + k0, ((int64_t)(rows_left - 1) * lda + (K - k0)) * 4);
        const __amdgpu_buffer_rsrc_t rb = rsrc(Bp + k0 * ldb, ((K - 1 - k0) * ldb + cols_left) * 4);
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            R.a[i][0] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, o.a[i], 0, 0));
            R.a[i][1] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, o.a[i] + 16, 0, 0));
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i)
#pragma unroll
            for (int e = 0; e < 8; ++e)
                R.b[i][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, o.b[i][e], 0, 0));
    }

    // bfloat16 planes of 8 values, two at a time: one packed round-to-nearest-
    // even convert per pair, the leftovers formed exactly in FP32.
    static __device__ __forceinline__ void put8(uint16_t *base, int plane_elems, int row, int chunk, float (&x)[8]) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            u32x4 w;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const bf16x2 hb = __builtin_convertvector((f32x2){x[2 * h], x[2 * h + 1]}, bf16x2);
                const uint32_t bits = __builtin_bit_cast(uint32_t, hb);
                w[h] = bits;
                if (p + 1 < NP) {
                    x[2 * h] -= __builtin_bit_cast(float, bits << 16);
                    x[2 * h + 1] -= __builtin_bit_cast(float, bits & 0xffff0000u);
                }
            }
            *reinterpret_cast<u32x4 *>(base + p * plane_elems + lds_elem(row, chunk)) = w;
        }
    }

    // Split one whole K step held in R and write its planes to LDS.
    static __device__ __forceinline__ void put_step(uint16_t *stage, const Regs &R) {
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            float x[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[e] = R.a[i][0][e];
                x[4 + e] = R.a[i][1][e];
            }
            put8(stage, A_PLANE, u / CHUNKS, u % CHUNKS, x);
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = R.b[i][e];
            put8(stage + NP * A_PLANE, B_PLANE, u % BN, u / BN, x);
        }
    }

    // After put_step of a step that ends K: zero, in every plane, the A
    // entries of this thread's units at or past column `kvalid` (B's rows
    // past K already read as zero), and for the zero step of a tile without
    // K (kvalid 0, nothing loaded) its B entries too.  Works on LDS only, so
    // the whole-step path carries no masking and no extra live registers.
    static __device__ __forceinline__ void clear_tail(uint16_t *stage, int kvalid) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            const int u = threadIdx.x + i * NT;
            const int c0 = (u % CHUNKS) * 8;
            if (c0 + 8 <= kvalid) continue;
            const int off = lds_elem(u / CHUNKS, u % CHUNKS);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                u32x4 *w = reinterpret_cast<u32x4 *>(stage + p * A_PLANE + off);
                u32x4 v = {0, 0, 0, 0};
                if (c0 < kvalid) {
                    // the chunk K ends in: keep entries c0 + j, j < kvalid - c0
                    v = *w;
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        v[h] &= (c0 + 2 * h < kvalid ? 0x0000ffffu : 0u) | (c0 + 2 * h + 1 < kvalid ? 0xffff0000u : 0u);
                }
                *w = v;
            }
        }
        if (kvalid <= 0) {
#pragma unroll
            for (int i = 0; i < B_UNITS; ++i) {
                const int u = threadIdx.x + i * NT;
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    *reinterpret_cast<u32x4 *>(stage + NP * A_PLANE + p * B_PLANE + lds_elem(u % BN, u / BN)) =
                        u32x4{0, 0, 0, 0};
            }
        }
    }

    // Split the step held in R (`kvalid` valid K entries, at least BK for a
    // whole step) into LDS.
    static __device__ __forceinline__ void put(uint16_t *stage, const Regs &R, int64_t kvalid) {
        put_step(stage, R);
        if (kvalid < BK) {
            // Keeps this a branch of the last step: clear_tail does nothing
            // when kvalid >= BK, and without the statement the compiler drops
            // the test and runs clear_tail's per-lane tests on every step.
            asm volatile("");
            clear_tail(stage, kvalid > 0 ? (int)kvalid : 0);
        }
    }

    // The products of the K step in `cur`, then the put of the next step
    // (held in Rn, `kn` valid K entries; negative: there is none) into
    // `nxt`.  Products and split stay in sequence: emitting them as one block
    // for the scheduler to interleave measured slower (the longer live ranges
    // cost registers: grouped split6 0.32 -> 0.34 ms, 8192 split6 170 -> 160
    // TFLOP/s), and a wave's matrix and vector instructions do not overlap on
    // a SIMD in any case.
    static __device__ __forceinline__ void step(const uint16_t *cur, uint16_t *nxt, const Regs &Rn, int64_t kn,
                                                f32x4 (&lead)[FM][FN], f32x4 (&corr)[FM][FN]) {
        compute(cur, cur + NP * A_PLANE, lead, corr);
        if (kn >= 0) put(nxt, Rn, kn);
    }

    static __device__ __forceinline__ void epilogue(const f32x4 (&lead)[FM][FN], const f32x4 (&corr)[FM][FN], void *C,
                                                    int64_t ldc, int c_is_f64, int64_t M, int64_t N, int64_t m0,
                                                    int64_t n0) {
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
                        if (c_is_f64) ((gptr<double>)(double *)C)[r * ldc + c] = val;
                        else ((gptr<float>)(float *)C)[r * ldc + c] = (float)val;
                    }
                }
    }

    // Tile (tm, tn) of C = A.B, same contract as SplitTileFused::run_fused.
    static __device__ __forceinline__ void run_fused(const float *A, int64_t lda, const float *B, int64_t ldb,
                                                     void *C, int64_t ldc, int c_is_f64, int64_t M, int64_t N,
                                                     int64_t K, int64_t tm, int64_t tn, uint16_t *smem) {
        if (!ring_ok(lda, ldb)) {
            Fused::run_fused(A, lda, B, ldb, C, ldc, c_is_f64, M, N, K, tm, tn, smem);
            return;
        }
        const int64_t m0 = tm * BM, n0 = tn * BN;
        const int rows_left = (int)((M - m0) < BM ? (M - m0) : BM);
        const int cols_left = (int)((N - n0) < BN ? (N - n0) : BN);
        const float *Ap = A + m0 * lda, *Bp = B + n0;
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        const int64_t nkt = (K + BK - 1) / BK;
        if (nkt > 0) {
            Offs o;
            offsets(lda, ldb, rows_left, cols_left, o);
            Regs R[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r)
                if (r < nkt) load(R[r], o, Ap, lda, Bp, ldb, rows_left, cols_left, K, r);
            put(smem, R[0], K);
            __syncthreads();
            for (int64_t s = 0; s < nkt; s += RS) {
#pragma unroll
                for (int r = 0; r < RS; ++r) {
                    const int64_t kt = s + r;
                    if (kt < nkt) {
                        // slot r held step kt (already in LDS): refill it with kt + RS
                        if (kt + RS < nkt) load(R[r], o, Ap, lda, Bp, ldb, rows_left, cols_left, K, kt + RS);
                        step(smem + (kt & 1) * STAGE, smem + ((kt + 1) & 1) * STAGE, R[(r + 1) % RS],
                             kt + 1 < nkt ? K - (kt + 1) * BK : -1, lead, corr);
                        __syncthreads();
                    }
                }
            }
        }
        epilogue(lead, corr, C, ldc, c_is_f64, M, N, m0, n0);
    }

    // ---------------------------------------------------------------- stream
    // A persistent workgroup's tiles as one stream of K steps: the load side
    // runs one step ahead of the products and crosses into the next tile
    // while the current one is still being multiplied, so a tile's first
    // loads are in flight when its predecessor ends.  Each tile's products,
    // order and recombination are those of run_fused (the same bits).
    // `seq` names the workgroup's i-th tile (seq.tile(i), >= total at the end;
    // seq.draw(i), called at the start of the load side's second-to-last step
    // of the i-th tile, or its only one, lets a dynamic sequence fetch the
    // (i+1)-th).
    // decode(t, g) fills tile t's geometry; every tile must satisfy ring_ok
    // (the caller checks the batch).  A tile without K steps (K == 0) runs one
    // step of zeros.  Per step, in order: [draw], the step's loads, the
    // products of the step before, [opening the next tile: its decode's
    // latency overlaps the loads in flight], the split of the loaded step,
    // [the end of a tile: its epilogue], one barrier.  Each tile is decoded
    // once: the compute side takes the geometry the load side decoded.  The
    // stream keeps one step in flight (RS == 1).

    struct Geo {
        const float *A, *B;
        void *C;
        int64_t lda, ldb, ldc, M, N, K, tm, tn;
    };

    struct LoadCursor {
        const float *Ap, *Bp;
        int64_t lda, ldb, K, nk, k, t;
        int rows_left, cols_left, i;
        Offs o;
    };

    // What the products and the epilogue need of a tile.
    struct ComputeTile {
        void *C;
        int64_t ldc, M, N, m0, n0, nk;
    };

    static __device__ __forceinline__ int64_t steps_of(int64_t K) { return K > 0 ? (K + BK - 1) / BK : 1; }

    // Open sequence position i for loading; its compute geometry goes to `ct`.
    template <typename Seq, typename Decode>
    static __device__ __forceinline__ void open_load(LoadCursor &L, int i, int64_t total, Seq &seq, Decode &decode,
                                                     ComputeTile &ct) {
        L.i = i;
        L.t = seq.tile(i);
        if (L.t >= total) return;
        Geo g;
        decode(L.t, g);
        const int64_t m0 = g.tm * BM, n0 = g.tn * BN;
        L.Ap = g.A + m0 * g.lda;
        L.Bp = g.B + n0;
        L.lda = g.lda;
        L.ldb = g.ldb;
        L.K = g.K;
        L.nk = steps_of(g.K);
        L.k = 0;
        L.rows_left = (int)((g.M - m0) < BM ? (g.M - m0) : BM);
        L.cols_left = (int)((g.N - n0) < BN ? (g.N - n0) : BN);
        offsets(L.lda, L.ldb, L.rows_left, L.cols_left, L.o);
        ct = ComputeTile{g.C, g.ldc, g.M, g.N, m0, n0, L.nk};
    }

    // Request the load cursor's next step into R (kvalid: valid K entries of
    // that step, 0 for the zero step of a K == 0 tile, -1 past the end of the
    // stream) and advance; returns whether that was the tile's last step.
    static __device__ __forceinline__ bool next_load(LoadCursor &L, Regs &R, int64_t &kvalid, int64_t total) {
        if (L.t >= total) {
            kvalid = -1;
            return false;
        }
        if (L.K > 0) {
            load(R, L.o, L.Ap, L.lda, L.Bp, L.ldb, L.rows_left, L.cols_left, L.K, L.k);
            kvalid = L.K - L.k * BK;
        } else {
            kvalid = 0;
        }
        return ++L.k == L.nk;
    }

    template <typename Seq, typename Decode>
    static __device__ __forceinline__ void run_stream(int64_t total, int c_is_f64, Seq seq, Decode decode,
                                                      uint16_t *smem) {
        static_assert(RS == 1, "the stream keeps one step in flight");
        f32x4 lead[FM][FN], corr[FM][FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                lead[fm][fn] = f32x4{0, 0, 0, 0};
                corr[fm][fn] = f32x4{0, 0, 0, 0};
            }
        // compute geometry of opened tiles, by sequence parity: the load side
        // is at most two tiles ahead of the products (one step, and a tile
        // of a single step)
        ComputeTile even, odd;
        LoadCursor L;
        open_load(L, 0, total, seq, decode, even);
        if (L.t >= total) return;
        ComputeTile cur = even;
        int ci = 0;              // sequence position of the tile being multiplied
        int opened = 1;          // positions opened that hold a tile
        int64_t ck = 0;          // its steps done
        // Position L.i + 1 is drawn two steps before the load side needs it,
        // not when L.i opens: claimed early, a workgroup's next tile would
        // wait a whole tile, and the tiles in flight on an XCD would spread
        // over twice the stretch of the tile map (fewer shared panels in L2).
        bool drawn = false;
        Regs R;
        int64_t kv;
        if (L.nk <= 2) {
            seq.draw(0);
            drawn = true;
        }
        if (next_load(L, R, kv, total)) {
            ComputeTile ct;
            open_load(L, 1, total, seq, decode, ct);
            drawn = false;
            if (L.t < total) {
                odd = ct;
                ++opened;
            }
        }
        put(smem, R, kv);
        __syncthreads();
        for (int64_t g = 0;; ++g) {
            // stream step g is in LDS buffer g & 1
            if (!drawn && L.t < total && L.nk - L.k <= 2) {
                seq.draw(L.i);
                drawn = true;
            }
            const bool crossed = next_load(L, R, kv, total);
            const uint16_t *cb = smem + (g & 1) * STAGE;
            compute(cb, cb + NP * A_PLANE, lead, corr);
            if (crossed) {
                ComputeTile ct;
                open_load(L, L.i + 1, total, seq, decode, ct);
                drawn = false;
                if (L.t < total) {
                    if (L.i & 1) odd = ct;
                    else even = ct;
                    ++opened;
                }
            }
            if (kv >= 0) put(smem + ((g + 1) & 1) * STAGE, R, kv);
            if (++ck == cur.nk) {
                epilogue(lead, corr, cur.C, cur.ldc, c_is_f64, cur.M, cur.N, cur.m0, cur.n0);
#pragma unroll
                for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                    for (int fn = 0; fn < FN; ++fn) {
                        lead[fm][fn] = f32x4{0, 0, 0, 0};
                        corr[fm][fn] = f32x4{0, 0, 0, 0};
                    }
                if (++ci >= opened) break;   // the load side found no further tile
                cur = (ci & 1) ? odd : even;
                ck = 0;
            }
            __syncthreads();
        }
    }
};

// Waves per SIMD for a kernel around split tile ST: the ring tiles ask for
// the LDS-limited occupancy, the others for 2 (8-wave tiles) or 1.
template <typename ST, typename = void> struct SplitWaves {
    static constexpr int value = ST::NWAVES >= 8 ? 2 : 1;
};
template <typename ST> struct SplitWaves<ST, std::void_t<decltype(ST::RS)>> {
    static constexpr int value = ST::WAVES;
};

// Variant selector: S = 1, 2 register stages (SplitTile); S = 10 + b: direct
// global-to-LDS ring of b buffers (SplitTileDirect, BK = 32); S = 20: fused
// split (SplitTileFused, BK = 32, FP32 operands, no plane pass); S = 20 + r
// (r = 1..4): the fused split with buffer loads and r K steps in flight in
// registers (SplitTileFusedRing); S = 30 + r: the same with paired 128-byte
// LDS lines.
// IL asks the direct tile of the 2-plane method for interleaved planes.
template <int NPROD, int BM, int BN, int BK, int WM, int WN, int S, bool IL = false,
          int KIND = (S > 30 ? 4 : S > 20 ? 3 : S == 20 ? 2 : S >= 10 ? 1 : 0)>
struct SplitTileSel {
    typedef SplitTile<NPROD, BM, BN, BK, WM, WN, S> type;
};
template <int NPROD, int BM, int BN, int BK, int WM, int WN, int S, bool IL>
struct SplitTileSel<NPROD, BM, BN, BK, WM, WN, S, IL, 1> {
    typedef SplitTileDirect<NPROD, BM, BN, WM, WN, S - 10, IL && NPROD == 3> type;
};
template <int NPROD, int BM, int BN, int BK, int WM, int WN, int S, bool IL>
struct SplitTileSel<NPROD, BM, BN, BK, WM, WN, S, IL, 2> {
    static_assert(BK == 32, "the fused tile steps K by 32");
    typedef SplitTileFused<NPROD, BM, BN, WM, WN> type;
};
template <int NPROD, int BM, int BN, int BK, int WM, int WN, int S, bool IL>
struct SplitTileSel<NPROD, BM, BN, BK, WM, WN, S, IL, 3> {
    static_assert(BK == 32, "the fused tile steps K by 32");
    typedef SplitTileFusedRing<NPROD, BM, BN, WM, WN, S - 20> type;
};
template <int NPROD, int BM, int BN, int BK, int WM, int WN, int S, bool IL>
struct SplitTileSel<NPROD, BM, BN, BK, WM, WN, S, IL, 4> {
    static_assert(BK == 32, "the fused tile steps K by 32");
    typedef SplitTileFusedRing<NPROD, BM, BN, WM, WN, S - 30, true> type;
};

}  // namespace mm
