// Grouped products: many independent C_i = A_i.B_i of different shapes in one
// persistent launch.
//
// Size-class pairs run each problem on the smaller or the larger of two tile
// variants of one workgroup size (chosen on the host from the padded work of
// each); the tile table carries each tile's kind.
//
// Tile map: problem i contributes ceil(M_i/BM) * ceil(N_i/BN) tiles; the host
// stores the exclusive prefix sum of these counts in each descriptor.  A
// persistent grid (the number of workgroups the chip holds at once) walks the
// global tile ids -- by a fixed stride, or from an atomic work counter -- and
// finds the owning problem by binary search over the prefix sums.  Each tile is
// computed by the same tile body as the single-problem kernels, so a problem's
// result is bit-identical to the single-problem result with the same variant.
//
// The split methods first run one grouped split pass over every operand of
// every problem (64 x 64 tiles, A planes row-major, B planes transposed) into a
// workspace, then the grouped split GEMM.  A plan captures this sequence once
// into a HIP graph and replays it; descriptors live at fixed device addresses
// and are refreshed (stream-ordered) before each replay.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "mm_internal.h"
#include "gemm_tile.h"
#include "split_tile.h"
#include "variants.h"

namespace mm {

// ------------------------------------------------------------------ device side

// The owner search reads the prefix sums from LDS when they fit (CAP entries,
// tile ids below 2^31): one pass of global loads per workgroup instead of a
// chain of dependent global loads per tile.
template <int CAP, typename D>
__device__ __forceinline__ bool stage_begins(const D *__restrict__ descs, int count, int64_t total_tiles,
                                             int32_t *s_begin) {
    const bool cached = count <= CAP && total_tiles <= (int64_t)0x7fffffff;
    if (cached) {
        for (int i = threadIdx.x; i < count; i += blockDim.x) s_begin[i] = (int32_t)descs[i].tile_begin;
        __syncthreads();
    }
    return cached;
}

template <typename D>
__device__ __forceinline__ int find_owner(const D *__restrict__ descs, const int32_t *s_begin, bool cached, int count,
                                          int64_t t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = cached ? (int64_t)s_begin[mid] : descs[mid].tile_begin;
        if (b <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Tile ids and owner indices are the same in every lane; reading them from
// the first lane makes that visible to the compiler, so the descriptor is
// fetched with scalar loads into scalar registers rather than occupying
// vector registers next to the accumulators.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One workgroup per tile: workgroups are dispatched to the 8 XCDs round-
// robin.  Chunks of kChunk consecutive tiles (mostly of one problem, sharing
// its A row panel) go to one XCD, whose L2 then serves the shared panels;
// chunk c goes to XCD c % 8, so every XCD still takes heavy and light work in
// the order of the tile map.  A bijection on [0, round_up(tiles, 8 kChunk)).
constexpr int kChunk = 8;
constexpr int kCounters = 8;   // work counters of schedule 2 (the streamed form uses one per XCD)
__device__ __forceinline__ int64_t chunked_tile(int64_t bid) {
    const int64_t xcd = bid % 8, local = bid / 8;
    return ((local / kChunk) * 8 + xcd) * kChunk + local % kChunk;
}
inline int64_t chunked_grid(int64_t tiles) { return (tiles + 8 * kChunk - 1) / (8 * kChunk) * (8 * kChunk); }

constexpr int kOwnerCap = 1024;     // problems whose prefix sums are staged in LDS
constexpr int kJobCap = 2048;       // split jobs likewise

// Work counter: thread 0 draws the ticket of the workgroup's next tile when a
// tile starts (its latency hides behind the tile's loads); after the tile the
// ticket is broadcast through LDS.  Ticket j names tile gridDim.x + j, since
// the first gridDim.x tiles are taken by blockIdx.
__device__ __forceinline__ int draw_ticket(int *counter) {
    return (counter && threadIdx.x == 0) ? atomicAdd(counter, 1) : 0;
}

__device__ __forceinline__ int64_t next_tile(int64_t cur, const int *counter, int ticket, int64_t *slot) {
    if (!counter) return cur + gridDim.x;
    if (threadIdx.x == 0) *slot = (int64_t)ticket + gridDim.x;
    __syncthreads();
    return uniform(*slot);
}

// Tile coordinates of a problem's local tile index: column-major within
// groups of two tile rows, so that runs of consecutive tiles (which the
// one-workgroup-per-tile form keeps on one XCD) share A and B panels.
__device__ __forceinline__ void local_tile(int64_t local, int64_t tiles_m, int64_t tiles_n, int64_t *tm, int64_t *tn) {
    const int64_t per_group = 2 * tiles_n;
    const int64_t first_m = (local / per_group) * 2;
    const int64_t gsize = tiles_m - first_m < 2 ? tiles_m - first_m : 2;
    const int64_t in = local % per_group;
    *tm = uniform(first_m + in % gsize);
    *tn = uniform(in / gsize);
}

// Owner problem and coordinates of tile t: one load from the launch's tile
// table when it has one, else a binary search over the descriptors' prefix
// sums (staged in LDS when `cached`) and the in-problem order of local_tile.
__device__ __forceinline__ void locate(const GroupedDesc *__restrict__ descs, const int32_t *s_begin, bool cached,
                                       int count, const TileRef *__restrict__ tiles, int64_t t, int *own, int64_t *tm,
                                       int64_t *tn) {
    if (tiles) {
        const TileRef r = tiles[t];
        *own = uniform(r.own);
        *tm = uniform(r.tm);
        *tn = uniform(r.tn);
        return;
    }
    *own = uniform(find_owner(descs, s_begin, cached, count, t));
    const GroupedDesc &d = descs[*own];
    local_tile(t - d.tile_begin, d.tiles_m, d.tiles_n, tm, tn);
}

// One tile of a grouped launch: run the single-problem tile body on tile
// (tm, tn) of problem d.
template <typename TG, typename T>
__device__ __forceinline__ void grouped_dense_tile(const GroupedDesc &d, int64_t tm, int64_t tn, T *smem) {
    const bool vec_ok = (d.lda % TG::VEC == 0) && (d.ldb % TG::VEC == 0) && ((uintptr_t)d.A % 16 == 0) &&
                        ((uintptr_t)d.B % 16 == 0);
    TG::run((const T *)d.A, d.lda, (const T *)d.B, d.ldb, (T *)d.C, d.ldc, d.M, d.N, d.K, tm, tn, vec_ok, smem);
}

template <typename ST>
__device__ __forceinline__ void grouped_split_tile(const GroupedDesc &d, int64_t tm, int64_t tn, uint16_t *smem) {
    if constexpr (ST::FUSED) {
        // descriptors hold the FP32 operands themselves
        ST::run_fused((const float *)d.A, d.lda, (const float *)d.B, d.ldb, d.C, d.ldc, 0, d.M, d.N, d.K, tm, tn, smem);
    } else {
        const bool vec_ok = (d.K % 8 == 0) && ((uintptr_t)d.A % 16 == 0) && ((uintptr_t)d.B % 16 == 0);
        ST::run((const uint16_t *)d.A, d.M * d.K, (const uint16_t *)d.B, d.N * d.K, d.C, d.ldc, 0, d.M, d.N, d.K, tm,
                tn, vec_ok, smem);
    }
}

// Two forms of each grouped kernel.  PERSISTENT: a grid the chip holds at
// once loops over the tiles (fixed stride, or tickets from the work counter).
// Otherwise one workgroup per tile, in tile order, dispatched by the
// hardware: no loop, so the tile body keeps the registers of the single-problem
// kernel (the loop over tiles costs registers: the compiler hoists the per-
// thread index arithmetic of the tile body out of it).
// Two waves per SIMD are asked of 4-wave tiles whose LDS lets two workgroups
// share a CU; otherwise one.
template <typename TG, typename T, bool PERSISTENT>
__global__ __launch_bounds__(TG::NT, (TG::NWAVES <= 4 && TG::LDS_ELEMS * sizeof(T) <= 76 * 1024 ? 2 : 1)) void grouped_gemm_kernel(
    const GroupedDesc *__restrict__ descs, int count, int64_t total_tiles, int *counter,
    const TileRef *__restrict__ tiles) {
    __shared__ __attribute__((aligned(16))) T smem[TG::LDS_ELEMS];
    int own;
    int64_t tm, tn;
    if constexpr (PERSISTENT) {
        __shared__ int32_t s_begin[kOwnerCap];
        __shared__ int64_t slot;
        const bool cached = !tiles && stage_begins<kOwnerCap>(descs, count, total_tiles, s_begin);
        for (int64_t t = blockIdx.x; t < total_tiles;) {
            const int ticket = draw_ticket(counter);
            locate(descs, s_begin, cached, count, tiles, t, &own, &tm, &tn);
            grouped_dense_tile<TG, T>(descs[own], tm, tn, smem);
            __syncthreads();
            t = next_tile(t, counter, ticket, &slot);
        }
    } else {
        const int64_t t = chunked_tile(blockIdx.x);
        if (t < total_tiles) {
            locate(descs, nullptr, false, count, tiles, t, &own, &tm, &tn);
            grouped_dense_tile<TG, T>(descs[own], tm, tn, smem);
        }
    }
}

template <typename ST, bool PERSISTENT>
__global__ __launch_bounds__(ST::NT, PERSISTENT ? (ST::NWAVES >= 8 ? 2 : 1) : SplitWaves<ST>::value) void grouped_split_gemm_kernel(
    const GroupedDesc *__restrict__ descs, int count, int64_t total_tiles, int *counter,
    const TileRef *__restrict__ tiles) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[ST::LDS_ELEMS];
    int own;
    int64_t tm, tn;
    if constexpr (PERSISTENT) {
        __shared__ int32_t s_begin[kOwnerCap];
        __shared__ int64_t slot;
        const bool cached = !tiles && stage_begins<kOwnerCap>(descs, count, total_tiles, s_begin);
        for (int64_t t = blockIdx.x; t < total_tiles;) {
            const int ticket = draw_ticket(counter);
            locate(descs, s_begin, cached, count, tiles, t, &own, &tm, &tn);
            grouped_split_tile<ST>(descs[own], tm, tn, smem);
            __syncthreads();
            t = next_tile(t, counter, ticket, &slot);
        }
    } else {
        const int64_t t = chunked_tile(blockIdx.x);
        if (t < total_tiles) {
            locate(descs, nullptr, false, count, tiles, t, &own, &tm, &tn);
            grouped_split_tile<ST>(descs[own], tm, tn, smem);
        }
    }
}

// Size-class pair kernels.  Each tile's kind, read from the tile table (which
// these launches always have), picks the small or the large variant's tile
// body; the two share the workgroup size and one LDS array (the larger of
// their two).  Same two forms as above.
template <typename TS, typename TL> struct PairLds {
    static constexpr int value = TS::LDS_ELEMS > TL::LDS_ELEMS ? TS::LDS_ELEMS : TL::LDS_ELEMS;
};

template <typename TS, typename TL, typename E, bool SPLIT>
__device__ __forceinline__ void grouped_pair_tile(const GroupedDesc *__restrict__ descs,
                                                  const TileRef *__restrict__ tiles, int64_t t, E *smem) {
    const TileRef r = tiles[t];
    const GroupedDesc &d = descs[uniform(r.own)];
    const int64_t tm = uniform(r.tm), tn = uniform(r.tn);
    if constexpr (SPLIT) {
        static_assert(TS::FUSED && TL::FUSED, "split pairs read the FP32 operands (no plane pass)");
        if (uniform(r.kind)) grouped_split_tile<TL>(d, tm, tn, smem);
        else grouped_split_tile<TS>(d, tm, tn, smem);
    } else {
        if (uniform(r.kind)) grouped_dense_tile<TL, E>(d, tm, tn, smem);
        else grouped_dense_tile<TS, E>(d, tm, tn, smem);
    }
}

// Waves per SIMD the pair kernels are compiled for: what the dense and split
// kernels above ask of their tile, for the pair's larger LDS array.
template <typename TS, typename TL, typename E, bool SPLIT, bool PERSISTENT> struct PairWaves {
    static constexpr int dense = TS::NWAVES <= 4 && PairLds<TS, TL>::value * sizeof(E) <= 76 * 1024 ? 2 : 1;
    static constexpr int split_tile = SplitWaves<TS>::value < SplitWaves<TL>::value ? SplitWaves<TS>::value
                                                                                    : SplitWaves<TL>::value;
    static constexpr int value = !SPLIT ? dense : PERSISTENT ? (TS::NWAVES >= 8 ? 2 : 1) : split_tile;
};

template <typename TS, typename TL, typename E, bool SPLIT, bool PERSISTENT>
__global__ __launch_bounds__(TS::NT, (PairWaves<TS, TL, E, SPLIT, PERSISTENT>::value)) void grouped_pair_kernel(
    const GroupedDesc *__restrict__ descs, int count, int64_t total_tiles, int *counter,
    const TileRef *__restrict__ tiles) {
    static_assert(TS::NT == TL::NT, "the two variants of a pair share one workgroup size");
    __shared__ __attribute__((aligned(16))) E smem[PairLds<TS, TL>::value];
    (void)count;
    if constexpr (PERSISTENT) {
        __shared__ int64_t slot;
        for (int64_t t = blockIdx.x; t < total_tiles;) {
            const int ticket = draw_ticket(counter);
            grouped_pair_tile<TS, TL, E, SPLIT>(descs, tiles, t, smem);
            __syncthreads();
            t = next_tile(t, counter, ticket, &slot);
        }
    } else {
        const int64_t t = chunked_tile(blockIdx.x);
        if (t < total_tiles) grouped_pair_tile<TS, TL, E, SPLIT>(descs, tiles, t, smem);
    }
}

// Streamed persistent form of the fused ring tiles: each workgroup runs its
// sequence of tiles as one stream of K steps, loading the next tile's first
// steps while the current tile is multiplied (SplitTileFusedRing::run_stream).
// Without a counter a workgroup takes tiles blockIdx.x + i * gridDim.x;
// with one (schedule 2) its first tile is blockIdx.x and each
// further tile is gridDim.x + a ticket of the work counter, drawn by thread 0
// as soon as the previous tile is opened for loading and passed to the other
// waves through a small LDS ring (a barrier precedes each read).  Every
// problem of the batch satisfies the tile's offset limits (checked on the
// host).
struct StaticSeq {
    int64_t first, stride;
    __device__ __forceinline__ int64_t tile(int i) const { return first + (int64_t)i * stride; }
    __device__ __forceinline__ void draw(int) {}
};

// Tickets per XCD: the workgroups of XCD x (blockIdx.x % 8, since workgroups
// are dispatched to the XCDs round-robin) walk that XCD's share of the tile
// map -- chunks of kChunk consecutive tiles, chunk c on XCD c % 8, as the
// one-workgroup-per-tile form places them -- drawing positions from the XCD's
// own counter, so tiles that share a problem's panels share an L2.  The grid
// is a multiple of 8.
// Thread 0 draws position i + 1's ticket in draw(i) but writes it to LDS only
// when tile(i + 1) is asked for, so the atomic's latency passes while the
// workgroup multiplies instead of holding up the next barrier.
struct TicketSeq {
    int *counter;       // 8 counters, one per XCD
    int64_t *ring;      // LDS, 8 entries: tile of sequence position i at i % 8
    int pending = -1;   // thread 0: the position whose ticket is in flight
    int ticket = 0;     // thread 0: that ticket
    __device__ __forceinline__ static int64_t chunked(int64_t xcd, int64_t local) {
        return ((local / kChunk) * 8 + xcd) * kChunk + local % kChunk;
    }
    __device__ __forceinline__ int64_t tile(int i) const {
        if (i == 0) return chunked(blockIdx.x % 8, blockIdx.x / 8);
        if (threadIdx.x == 0 && pending == i)
            ring[i & 7] = chunked(blockIdx.x % 8, (int64_t)(gridDim.x / 8) + ticket);
        __syncthreads();   // thread 0's write of position i is visible
        return uniform(ring[i & 7]);
    }
    __device__ __forceinline__ void draw(int i) {
        if (threadIdx.x == 0) {
            ticket = atomicAdd(counter + blockIdx.x % 8, 1);
            pending = i + 1;
        }
    }
};

template <typename ST>
__global__ __launch_bounds__(ST::NT, ST::WAVES) void grouped_split_stream_kernel(const GroupedDesc *__restrict__ descs,
                                                                          int count, int64_t total_tiles,
                                                                          int *counter,
                                                                          const TileRef *__restrict__ tiles) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[ST::LDS_ELEMS];
    __shared__ int64_t s_ring[8];
    (void)count;
    auto decode = [&](int64_t t, typename ST::Geo &g) {
        const TileRef ref = tiles[t];
        const GroupedDesc &d = descs[uniform(ref.own)];
        const int64_t tm = uniform(ref.tm), tn = uniform(ref.tn);
        g.A = (const float *)d.A;
        g.B = (const float *)d.B;
        g.C = d.C;
        g.lda = d.lda;
        g.ldb = d.ldb;
        g.ldc = d.ldc;
        g.M = d.M;
        g.N = d.N;
        g.K = d.K;
        g.tm = tm;
        g.tn = tn;
    };
    if (counter) ST::run_stream(total_tiles, 0, TicketSeq{counter, s_ring}, decode, smem);
    else ST::run_stream(total_tiles, 0, StaticSeq{blockIdx.x, gridDim.x}, decode, smem);
}

__global__ __launch_bounds__(256) void grouped_split_kernel(const SplitJob *__restrict__ jobs, int njobs,
                                                            int64_t total_tiles) {
    __shared__ float tile[64][65];
    __shared__ int32_t s_begin[kJobCap];
    const int cq = (threadIdx.x & 15) * 4, rq = threadIdx.x >> 4;
    const bool cached = stage_begins<kJobCap>(jobs, njobs, total_tiles, s_begin);
    for (int64_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        const SplitJob &j = jobs[uniform(find_owner(jobs, s_begin, cached, njobs, t))];
        const gptr<const float> X = (gptr<const float>)j.X;
        const gptr<uint16_t> planes = (gptr<uint16_t>)j.planes;
        const int64_t local = t - j.tile_begin;
        const int64_t r0 = (local / j.tiles_c) * 64, c0 = (local % j.tiles_c) * 64;
        // 16 threads read one 64-float row segment as 16-byte loads
        for (int i = rq; i < 64; i += 16) {
            const int64_t r = r0 + i, c = c0 + cq;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (r < j.rows) {
                const gptr<const float> src = X + r * j.ldx + c;
                if (c + 4 <= j.cols) {
                    const f32x4 q = load_f32x4_ea(src);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = q[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (c + e < j.cols) v[e] = src[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) tile[i][cq + e] = v[e];
        }
        __syncthreads();
        // 8 consecutive outputs per thread and plane, one 16-byte store when
        // aligned.  Transposed: output row c0+a walks r from r0+b; plain:
        // output row r0+a walks c from c0+b.  Output rows hold j.ldp elements;
        // the tail past the data is zero.
        const bool vec = j.ldp % 8 == 0 && j.pstride % 8 == 0 && (uintptr_t)j.planes % 16 == 0;
        for (int k = threadIdx.x; k < 64 * 8; k += 256) {
            const int a = k >> 3, b = (k & 7) * 8;
            const int64_t row = j.transpose ? c0 + a : r0 + a;            // output row
            const int64_t col = j.transpose ? r0 + b : c0 + b;            // first output column
            if (row >= (j.transpose ? j.cols : j.rows) || col >= j.ldp) continue;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = j.transpose ? tile[b + e][a] : tile[a][b + e];
            const int n = j.ldp - col < 8 ? (int)(j.ldp - col) : 8;
            for (int p = 0; p < j.nplanes; ++p) split_store_chunk(v, planes + p * j.pstride + row * j.ldp + col, n, vec);
        }
        __syncthreads();
    }
}

// Clears the work counters (one per XCD) with a kernel, not a memset node.
__global__ void reset_counter_kernel(int *counter) {
    if (threadIdx.x < kCounters) counter[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ variants

typedef const void *KernelPtr;

struct KernelInfo {
    KernelPtr fn = nullptr;
    int nt = 0, bm = 0, bn = 0;
    bool stream = false;   // a streamed persistent form exists (ring-fused split tiles)
    bool table = false;    // the kernel reads the tile table (size-class pairs)
};

// Ring-fused split tiles with one K step in flight (the only ones with a
// streamed persistent form).
template <typename T, typename = void> struct has_ring : std::false_type {};
template <typename T> struct has_ring<T, std::void_t<decltype(T::RS)>> : std::bool_constant<T::RS == 1> {};

template <typename TG, typename T>
static KernelPtr dense_kernel(int form) {
    return form == kFormTile ? (KernelPtr)&grouped_gemm_kernel<TG, T, false>
                             : (KernelPtr)&grouped_gemm_kernel<TG, T, true>;
}

template <typename ST>
static KernelPtr split_kernel(int form) {
    if (form == kFormStream) {
        if constexpr (has_ring<ST>::value) return (KernelPtr)&grouped_split_stream_kernel<ST>;
        return nullptr;
    }
    return form == kFormTile ? (KernelPtr)&grouped_split_gemm_kernel<ST, false>
                             : (KernelPtr)&grouped_split_gemm_kernel<ST, true>;
}

template <typename ST>
static constexpr bool split_has_stream() { return has_ring<ST>::value; }

// Tile type of each variant id, for the pair kernels.
template <int V> struct F64Var;
template <int V> struct F32Var;
template <int V> struct S3Var;
template <int V> struct S6Var;
#define MM_TV_F64(id, bm_, bn_, bk, wm, wn, st) \
    template <> struct F64Var<id> { typedef TileSel<double, bm_, bn_, bk, wm, wn, st>::type type; };
#define MM_TV_F32(id, bm_, bn_, bk, wm, wn, st) \
    template <> struct F32Var<id> { typedef TileSel<float, bm_, bn_, bk, wm, wn, st>::type type; };
#define MM_TV_S(id, bm_, bn_, bk, wm, wn, st)                                                          \
    template <> struct S3Var<id> { typedef SplitTileSel<3, bm_, bn_, bk, wm, wn, st>::type type; }; \
    template <> struct S6Var<id> { typedef SplitTileSel<6, bm_, bn_, bk, wm, wn, st>::type type; };
MM_F64_VARIANTS(MM_TV_F64)
MM_F32_VARIANTS(MM_TV_F32)
MM_SPLIT_VARIANTS(MM_TV_S)

template <typename TS, typename TL, typename E, bool SPLIT>
static KernelInfo pair_kernel(int form) {
    KernelInfo k;
    k.fn = form == kFormStream ? nullptr
           : form == kFormTile ? (KernelPtr)&grouped_pair_kernel<TS, TL, E, SPLIT, false>
                               : (KernelPtr)&grouped_pair_kernel<TS, TL, E, SPLIT, true>;
    k.nt = TS::NT;
    k.table = true;
    return k;
}

static KernelInfo pair_kernel_for(mm_method method, int pair, int form) {
#define MM_GP_F64(p, s_, l_, pct) case p: return pair_kernel<F64Var<s_>::type, F64Var<l_>::type, double, false>(form);
#define MM_GP_F32(p, s_, l_, pct) case p: return pair_kernel<F32Var<s_>::type, F32Var<l_>::type, float, false>(form);
#define MM_GP_S3(p, s_, l_, pct) case p: return pair_kernel<S3Var<s_>::type, S3Var<l_>::type, uint16_t, true>(form);
#define MM_GP_S6(p, s_, l_, pct) case p: return pair_kernel<S6Var<s_>::type, S6Var<l_>::type, uint16_t, true>(form);
    switch (method) {
        case MM_F64: switch (pair) { MM_F64_PAIRS(MM_GP_F64) default: break; } break;
        case MM_F32: switch (pair) { MM_F32_PAIRS(MM_GP_F32) default: break; } break;
        case MM_SPLIT_BF16_3: switch (pair) { MM_SPLIT_PAIRS(MM_GP_S3) default: break; } break;
        case MM_SPLIT_BF16_6: switch (pair) { MM_SPLIT_PAIRS(MM_GP_S6) default: break; } break;
    }
    return KernelInfo();
}

int grouped_pair_count(mm_method method) {
#define MM_PAIR_ONE(p, s_, l_, pct) +1
    switch (method) {
        case MM_F64: return 0 MM_F64_PAIRS(MM_PAIR_ONE);
        case MM_F32: return 0 MM_F32_PAIRS(MM_PAIR_ONE);
        case MM_SPLIT_BF16_3:
        case MM_SPLIT_BF16_6: return 0 MM_SPLIT_PAIRS(MM_PAIR_ONE);
    }
    return 0;
}

bool grouped_pair(mm_method method, int variant, PairCfg *out) {
    const int p = variant - MM_PAIR_BASE;
#define MM_PAIR_CFG(p_, s_, l_, pct) case p_: *out = PairCfg{s_, l_, pct}; return true;
    switch (method) {
        case MM_F64: switch (p) { MM_F64_PAIRS(MM_PAIR_CFG) default: return false; }
        case MM_F32: switch (p) { MM_F32_PAIRS(MM_PAIR_CFG) default: return false; }
        case MM_SPLIT_BF16_3:
        case MM_SPLIT_BF16_6: switch (p) { MM_SPLIT_PAIRS(MM_PAIR_CFG) default: return false; }
    }
    return false;
}

bool grouped_variant_valid(mm_method method, int variant) {
    PairCfg pc;
    return (variant >= 0 && variant < mm_variant_count(method)) || grouped_pair(method, variant, &pc);
}

static KernelInfo kernel_for(mm_method method, int variant, int form = kFormPersistent) {
    if (variant >= MM_PAIR_BASE) return pair_kernel_for(method, variant - MM_PAIR_BASE, form);
    KernelInfo k;
#define MM_GK_F64(id, bm_, bn_, bk, wm, wn, st) \
    case id: { typedef TileSel<double, bm_, bn_, bk, wm, wn, st>::type TG; k.fn = form == kFormStream ? nullptr : dense_kernel<TG, double>(form); k.nt = TG::NT; k.bm = bm_; k.bn = bn_; break; }
#define MM_GK_F32(id, bm_, bn_, bk, wm, wn, st) \
    case id: { typedef TileSel<float, bm_, bn_, bk, wm, wn, st>::type TG; k.fn = form == kFormStream ? nullptr : dense_kernel<TG, float>(form); k.nt = TG::NT; k.bm = bm_; k.bn = bn_; break; }
#define MM_GK_S3(id, bm_, bn_, bk, wm, wn, st) \
    case id: { typedef SplitTileSel<3, bm_, bn_, bk, wm, wn, st>::type ST; k.fn = split_kernel<ST>(form); k.nt = ST::NT; k.bm = bm_; k.bn = bn_; k.stream = split_has_stream<ST>(); break; }
#define MM_GK_S6(id, bm_, bn_, bk, wm, wn, st) \
    case id: { typedef SplitTileSel<6, bm_, bn_, bk, wm, wn, st>::type ST; k.fn = split_kernel<ST>(form); k.nt = ST::NT; k.bm = bm_; k.bn = bn_; k.stream = split_has_stream<ST>(); break; }
    switch (method) {
        case MM_F64: switch (variant) { MM_F64_VARIANTS(MM_GK_F64) default: break; } break;
        case MM_F32: switch (variant) { MM_F32_VARIANTS(MM_GK_F32) default: break; } break;
        case MM_SPLIT_BF16_3: switch (variant) { MM_SPLIT_VARIANTS(MM_GK_S3) default: break; } break;
        case MM_SPLIT_BF16_6: switch (variant) { MM_SPLIT_VARIANTS(MM_GK_S6) default: break; } break;
    }
    return k;
}

int grouped_form(mm_method method, int variant, int schedule, const Layout &L) {
    if (schedule == 3) return kFormTile;
    if (L.ring_ok && kernel_for(method, variant, kFormTile).stream) return kFormStream;
    return kFormPersistent;
}

int grouped_tile_bm(mm_method method, int variant) { return kernel_for(method, variant).bm; }
int grouped_tile_bn(mm_method method, int variant) { return kernel_for(method, variant).bn; }

// Workgroups of `fn` resident on the whole chip at once.
static int persistent_grid(KernelPtr fn, int nt) {
    static std::mutex mu;
    static std::map<std::pair<int, KernelPtr>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, fn);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    DeviceInfo d;
    int cus = device_info(&d) == MM_OK ? d.cus : 256;
    const int g = per_cu * cus;
    cache[key] = g;
    return g;
}

// Workgroups of a grouped launch: one per tile (rounded up so that runs of
// kChunk tiles go to one XCD), or the persistent grid capped by the tile count
// (the streamed form keeps it a multiple of 8: its tickets are per XCD).
static int64_t launch_grid(int form, const KernelInfo &k, int64_t total_tiles) {
    if (form == kFormTile) return chunked_grid(total_tiles);
    int64_t g = persistent_grid(k.fn, k.nt);
    if (form == kFormStream) {
        const int64_t cap = (total_tiles + 7) / 8 * 8;
        return g < cap ? g : cap;
    }
    return g < total_tiles ? g : total_tiles;
}

// ------------------------------------------------------------------ host layout

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static TileCfg tile_cfg(mm_method method, int variant) {
    return method == MM_F64 ? f64_variant(variant) : method == MM_F32 ? f32_variant(variant) : split_variant(variant);
}

// The member of a size-class pair that computes an M x N x K problem: the
// small variant when its tiles execute at most pct % of the large one's
// padded work (rows, columns and K rounded up to the tile), else the large.
static int pair_kind(mm_method method, const PairCfg &pc, int64_t M, int64_t N, int64_t K) {
    auto work = [&](int v) {
        const TileCfg c = tile_cfg(method, v);
        const int64_t k = K > 0 ? K : 1;
        return (double)(cdiv(M, c.bm) * c.bm) * (double)(cdiv(N, c.bn) * c.bn) * (double)(cdiv(k, c.bk) * c.bk);
    };
    return work(pc.small) * 100.0 <= pc.pct * work(pc.large) ? 0 : 1;
}

// order: problem indices in launch order (schedule already applied).
void build_layout(const mm_problem *probs, const std::vector<int> &order, mm_method method, int variant,
                         char *ws, Layout *L) {
    PairCfg pc{};
    const bool pair = grouped_pair(method, variant, &pc);
    const bool split_method = method == MM_SPLIT_BF16_3 || method == MM_SPLIT_BF16_6;
    // fused split tiles read the FP32 operands themselves: no planes, no jobs
    // (the members of split pairs are all fused)
    const bool split = split_method && !pair && !split_variant_fused(variant);
    const int np = method == MM_SPLIT_BF16_3 ? 2 : 3;
    L->descs.clear();
    L->jobs.clear();
    L->kinds.clear();
    L->total_tiles = 0;
    L->split_tiles = 0;
    L->ring_ok = true;
    size_t off = 0;
    for (int idx : order) {
        const mm_problem &p = probs[idx];
        if (p.M == 0 || p.N == 0) continue;
        const int kind = pair ? pair_kind(method, pc, p.M, p.N, p.K) : 0;
        const int v = pair ? (kind ? pc.large : pc.small) : variant;
        const int bm = grouped_tile_bm(method, v), bn = grouped_tile_bn(method, v);
        GroupedDesc d;
        std::memset(&d, 0, sizeof d);
        d.M = p.M;
        d.N = p.N;
        d.K = p.K;
        d.A = p.A;
        d.lda = p.lda;
        d.B = p.B;
        d.ldb = p.ldb;
        d.C = p.C;
        d.ldc = p.ldc;
        d.tiles_n = (int32_t)cdiv(p.N, bn);
        d.tiles_m = (int32_t)cdiv(p.M, bm);
        d.tile_begin = L->total_tiles;
        L->total_tiles += cdiv(p.M, bm) * d.tiles_n;
        // per-lane byte offsets of the ring-fused tiles (BK = 32) fit 31 bits
        if (((int64_t)(bm - 1) * p.lda + 32) * 4 >= 0x7fff0000LL || ((int64_t)31 * p.ldb + bn) * 4 >= 0x7fff0000LL)
            L->ring_ok = false;
        if (split) {
            const int64_t Kp = split_padded_k(p.K);
            const size_t abytes = align256((size_t)np * p.M * Kp * 2);
            const size_t bbytes = align256((size_t)np * p.N * Kp * 2);
            uint16_t *ap = ws ? (uint16_t *)(ws + off) : nullptr;
            uint16_t *bp = ws ? (uint16_t *)(ws + off + abytes) : nullptr;
            off += abytes + bbytes;
            d.A = ap;
            d.B = bp;
            d.K = Kp;     // the planes carry K rounded up to 32, zero-filled
            d.lda = Kp;
            d.ldb = Kp;
            if (p.K > 0) {
                SplitJob ja{(const float *)p.A, p.lda, p.M, p.K, ap, p.M * Kp, Kp, L->split_tiles,
                            (int32_t)cdiv(p.K, 64), np, 0, 0};
                L->split_tiles += cdiv(p.M, 64) * ja.tiles_c;
                L->jobs.push_back(ja);
                SplitJob jb{(const float *)p.B, p.ldb, p.K, p.N, bp, p.N * Kp, Kp, L->split_tiles,
                            (int32_t)cdiv(p.N, 64), np, 1, 0};
                L->split_tiles += cdiv(p.K, 64) * jb.tiles_c;
                L->jobs.push_back(jb);
            }
        }
        L->descs.push_back(d);
        L->kinds.push_back((int8_t)kind);
    }
    L->ws_bytes = off;
}

// Tile coordinates in the order the device's local_tile gives them:
// column-major within groups of two tile rows.
void build_tile_table(const Layout &L, std::vector<TileRef> *out) {
    out->resize((size_t)L.total_tiles);
    for (size_t i = 0; i < L.descs.size(); ++i) {
        const GroupedDesc &d = L.descs[i];
        const int64_t n = (int64_t)d.tiles_m * d.tiles_n;
        for (int64_t local = 0; local < n; ++local) {
            const int64_t per_group = 2 * (int64_t)d.tiles_n;
            const int64_t first_m = (local / per_group) * 2;
            const int64_t gsize = d.tiles_m - first_m < 2 ? d.tiles_m - first_m : 2;
            const int64_t in = local % per_group;
            TileRef &r = (*out)[(size_t)(d.tile_begin + local)];
            r.own = (int32_t)i;
            r.tm = (int32_t)(first_m + in % gsize);
            r.tn = (int32_t)(in / gsize);
            r.kind = L.kinds.empty() ? 0 : L.kinds[i];
        }
    }
}

// Launch order of the problems.  0: as given; 1, 2 and 3: largest K*M*N first
// (heaviest tiles start first).  How tiles reach workgroups: 0 and 1 a
// persistent grid by fixed stride, 2 a persistent grid pulling from a work
// counter, 3 one workgroup per tile dispatched in tile order by the hardware.
std::vector<int> schedule_order(const mm_problem *probs, int count, int schedule) {
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    if (schedule >= 1) {
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const double wa = (double)probs[a].K * probs[a].M * probs[a].N;
            const double wb = (double)probs[b].K * probs[b].M * probs[b].N;
            return wa > wb;
        });
    }
    return order;
}

// Enqueue the whole grouped sequence for descriptors already on the device.
// d_counter (schedule 2 only) is the work counter; persistent == false runs
// one workgroup per tile (schedule 3).
hipError_t grouped_enqueue(mm_method method, int variant, int form, const GroupedDesc *d_descs, int ndesc,
                          int64_t total_tiles, const SplitJob *d_jobs, int njobs, int64_t split_tiles, int *d_counter,
                          const TileRef *d_tiles, hipStream_t st) {
    if (ndesc == 0) return hipSuccess;
    const bool persistent = form != kFormTile;
    const KernelInfo k = kernel_for(method, variant, form);
    if (!k.fn) return hipErrorInvalidValue;
    if ((form == kFormStream || k.table) && !d_tiles) return hipErrorInvalidValue;
    if (!persistent && chunked_grid(total_tiles) > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if (njobs > 0 && split_tiles > 0) {
        int64_t g = split_tiles < 4096 ? split_tiles : 4096;
        hipLaunchKernelGGL(grouped_split_kernel, dim3((unsigned)g), dim3(256), 0, st, d_jobs, njobs, split_tiles);
    }
    if (!persistent) d_counter = nullptr;
    if (d_counter) hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, d_counter);
    const int64_t grid = launch_grid(form, k, total_tiles);
    void *args[] = {(void *)&d_descs, (void *)&ndesc, (void *)&total_tiles, (void *)&d_counter, (void *)&d_tiles};
    return hipLaunchKernel(k.fn, dim3((unsigned)grid), dim3(k.nt), args, 0, st);
}

static mm_status validate(const mm_problem *probs, int32_t count, mm_method method) {
    if (count < 0) return fail(MM_E_INVAL, "count < 0");
    if (count > 0 && !probs) return fail(MM_E_INVAL, "probs is NULL");
    if (method < MM_F64 || method > MM_SPLIT_BF16_6) return fail(MM_E_INVAL, "unknown method");
    const size_t e = method == MM_F64 ? 8 : 4;
    for (int i = 0; i < count; ++i) {
        const mm_problem &p = probs[i];
        mm_status s = check_gemm_args(p.M, p.N, p.K, p.A, p.lda, p.B, p.ldb, p.C, p.ldc, e, e);
        if (s == MM_OK && method >= MM_SPLIT_BF16_3) s = check_split_k(p.K);
        if (s != MM_OK) return fail(s, "problem " + std::to_string(i) + ": " + mm_last_error());
    }
    return MM_OK;
}

}  // namespace mm

// ------------------------------------------------------------------ plans

struct mm_grouped_plan {
    mm_method method;
    int variant = 0;
    int schedule = 0;
    int device = 0;
    std::vector<int64_t> shapes;          // M, N, K per problem as given
    std::vector<int> order;
    mm::Layout layout;
    mm::GroupedDesc *d_descs = nullptr;
    mm::SplitJob *d_jobs = nullptr;
    int *d_counter = nullptr;
    mm::TileRef *d_tiles = nullptr;   // tile table (owner and coordinates of every tile)
    void *ws = nullptr;
    // pinned staging ring for descriptor refreshes: each slot holds the
    // descriptors, then (at a 256-byte boundary) the split jobs
    static constexpr int RING = 4;
    char *h_ring = nullptr;
    size_t ring_stride = 0;
    hipEvent_t ring_ev[RING] = {};
    int ring_pos = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace mm {

// Releases everything a plan owns.  Best effort: a failing release (after a
// device error) must not stop the others, so return codes are not acted on.
static void destroy_plan(mm_grouped_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    for (auto &e : p->ring_ev)
        if (e) {
            (void)hipEventSynchronize(e);   // the pinned ring may still feed a copy
            (void)hipEventDestroy(e);
        }
    if (p->h_ring) (void)hipHostFree(p->h_ring);
    if (p->d_descs) (void)hipFree(p->d_descs);
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}

static mm_status create_plan(const mm_problem *probs, int32_t count, mm_method method, int variant, int schedule,
                             mm_grouped_plan **out) {
    mm_grouped_plan *p = new mm_grouped_plan();
    p->method = method;
    p->variant = variant;
    p->schedule = schedule;
    hipError_t e = hipGetDevice(&p->device);
    for (int i = 0; i < count; ++i) {
        p->shapes.push_back(probs[i].M);
        p->shapes.push_back(probs[i].N);
        p->shapes.push_back(probs[i].K);
    }
    p->order = schedule_order(probs, count, schedule);
    build_layout(probs, p->order, method, variant, nullptr, &p->layout);  // sizing
    if (e == hipSuccess && p->layout.ws_bytes) e = hipMalloc(&p->ws, p->layout.ws_bytes);
    if (e == hipSuccess) build_layout(probs, p->order, method, variant, (char *)p->ws, &p->layout);
    const size_t nd = p->layout.descs.size(), nj = p->layout.jobs.size();
    if (e == hipSuccess && nd) e = hipMalloc(&p->d_descs, nd * sizeof(GroupedDesc));
    if (e == hipSuccess && nj) e = hipMalloc(&p->d_jobs, nj * sizeof(SplitJob));
    if (e == hipSuccess && schedule == 2) e = hipMalloc(&p->d_counter, kCounters * sizeof(int));
    const int form = grouped_form(method, variant, schedule, p->layout);
    if (e == hipSuccess && p->layout.total_tiles > 0) {
        // the tile table depends on the shapes only: uploaded once (the
        // kernels then read each tile's owner and coordinates with one load)
        std::vector<TileRef> table;
        build_tile_table(p->layout, &table);
        e = hipMalloc(&p->d_tiles, table.size() * sizeof(TileRef));
        if (e == hipSuccess)
            e = hipMemcpy(p->d_tiles, table.data(), table.size() * sizeof(TileRef), hipMemcpyHostToDevice);
    }
    p->ring_stride = align256(nd * sizeof(GroupedDesc)) + align256(nj * sizeof(SplitJob));
    if (e == hipSuccess && nd) e = hipHostMalloc((void **)&p->h_ring, mm_grouped_plan::RING * p->ring_stride, 0);
    for (int i = 0; e == hipSuccess && i < mm_grouped_plan::RING; ++i) e = hipEventCreateWithFlags(&p->ring_ev[i], hipEventDisableTiming);
    if (e == hipSuccess && nd) e = hipMemcpy(p->d_descs, p->layout.descs.data(), nd * sizeof(GroupedDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess && nj) e = hipMemcpy(p->d_jobs, p->layout.jobs.data(), nj * sizeof(SplitJob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess && nd) {
        e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = grouped_enqueue(method, variant, form, p->d_descs, (int)nd, p->layout.total_tiles, p->d_jobs, (int)nj,
                                    p->layout.split_tiles, p->d_counter, p->d_tiles, p->capture_stream);
            hipError_t ce = hipStreamEndCapture(p->capture_stream, &p->graph);
            e = le != hipSuccess ? le : ce;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "grouped plan creation");
    }
    *out = p;
    return MM_OK;
}

static bool same_shapes(const mm_grouped_plan *p, const mm_problem *probs, int32_t count) {
    if ((int64_t)p->shapes.size() != 3 * (int64_t)count) return false;
    for (int i = 0; i < count; ++i)
        if (p->shapes[3 * i] != probs[i].M || p->shapes[3 * i + 1] != probs[i].N || p->shapes[3 * i + 2] != probs[i].K)
            return false;
    return true;
}

static mm_status run_plan(mm_grouped_plan *p, const mm_problem *probs, hipStream_t st, bool refresh) {
    const size_t nd = p->layout.descs.size();
    if (nd == 0) return MM_OK;
    if (refresh) {
        // Operand pointers may have changed: rebuild descriptors (the workspace
        // and tile map are unchanged) and refresh them in stream order.
        build_layout(probs, p->order, p->method, p->variant, (char *)p->ws, &p->layout);
        // The ring slot is reused only once the copies that last read it have
        // finished (its event), so the call does not wait for the stream.
        const size_t nj = p->layout.jobs.size();
        const int slot = p->ring_pos;
        p->ring_pos = (p->ring_pos + 1) % mm_grouped_plan::RING;
        MM_HIP(hipEventSynchronize(p->ring_ev[slot]));
        char *h = p->h_ring + slot * p->ring_stride;
        std::memcpy(h, p->layout.descs.data(), nd * sizeof(GroupedDesc));
        MM_HIP(hipMemcpyAsync(p->d_descs, h, nd * sizeof(GroupedDesc), hipMemcpyHostToDevice, st));
        if (nj) {
            // split jobs point at the caller's FP32 operands
            char *hj = h + align256(nd * sizeof(GroupedDesc));
            std::memcpy(hj, p->layout.jobs.data(), nj * sizeof(SplitJob));
            MM_HIP(hipMemcpyAsync(p->d_jobs, hj, nj * sizeof(SplitJob), hipMemcpyHostToDevice, st));
        }
        MM_HIP(hipEventRecord(p->ring_ev[slot], st));
    }
    MM_HIP(hipGraphLaunch(p->exec, st));
    return MM_OK;
}

// Host -> device upload of a one-shot launch's descriptors and split jobs.
// The bytes are packed into one of a few pinned buffers per device and copied
// in stream order; an event recorded after the copy guards the buffer, which is
// reused only once that copy has finished.  The call therefore never waits for
// the stream's earlier work -- at most for the copy of the call kRing uploads
// back.  Buffers grow (to the next power of two, 64 KiB at least) and are kept
// for the life of the process.
namespace {
constexpr int kRing = 8;
struct PinnedSlot {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
};
struct PinnedRing {
    std::mutex mu;
    PinnedSlot slot[kRing];
    int pos = 0;
};
PinnedRing &pinned_ring(int dev) {
    static std::mutex mu;
    static std::map<int, PinnedRing *> rings;   // one per device, never freed
    std::lock_guard<std::mutex> lock(mu);
    PinnedRing *&r = rings[dev];
    if (!r) r = new PinnedRing();
    return *r;
}
}  // namespace

// One piece of an upload: `bytes` from host `src` to byte `offset` of the
// destination.
struct Piece {
    size_t offset;
    const void *src;
    size_t bytes;
};

static mm_status upload_staged(char *dst, const Piece *pieces, int npieces, hipStream_t st) {
    int dev = 0;
    MM_HIP(hipGetDevice(&dev));
    size_t total = 0;
    for (int i = 0; i < npieces; ++i)
        if (pieces[i].bytes) total = std::max(total, pieces[i].offset + pieces[i].bytes);
    if (total == 0) return MM_OK;
    PinnedRing &r = pinned_ring(dev);
    std::lock_guard<std::mutex> lock(r.mu);
    PinnedSlot &s = r.slot[r.pos];
    r.pos = (r.pos + 1) % kRing;
    if (s.ev) MM_HIP(hipEventSynchronize(s.ev));   // the copy that last read this buffer is done
    else MM_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    if (s.cap < total) {
        size_t want = (size_t)64 << 10;
        while (want < total) want *= 2;
        if (s.host) MM_HIP(hipHostFree(s.host));
        s.host = nullptr;
        s.cap = 0;
        MM_HIP(hipHostMalloc((void **)&s.host, want, 0));
        s.cap = want;
    }
    for (int i = 0; i < npieces; ++i)
        if (pieces[i].bytes) std::memcpy(s.host + pieces[i].offset, pieces[i].src, pieces[i].bytes);
    MM_HIP(hipMemcpyAsync(dst, s.host, total, hipMemcpyHostToDevice, st));
    MM_HIP(hipEventRecord(s.ev, st));
    return MM_OK;
}

// One-shot launch without a plan: workspace and descriptors stream-ordered;
// the call only enqueues work.
static mm_status run_once(const mm_problem *probs, int32_t count, mm_method method, int variant, int schedule,
                          hipStream_t st) {
    std::vector<int> order = schedule_order(probs, count, schedule);
    Layout L;
    build_layout(probs, order, method, variant, nullptr, &L);
    const size_t nd = L.descs.size();
    if (nd == 0) return MM_OK;
    const int form = grouped_form(method, variant, schedule, L);
    std::vector<TileRef> table;
    if (form == kFormStream || kernel_for(method, variant, form).table) build_tile_table(L, &table);
    // device buffer: descriptors | split jobs | work counters | tile table | split workspace
    const size_t desc_bytes = align256(nd * sizeof(GroupedDesc));
    const size_t job_bytes = align256(L.jobs.size() * sizeof(SplitJob) + 1);
    const size_t counter_bytes = 256;
    const size_t table_bytes = align256(table.size() * sizeof(TileRef));
    const size_t ws_offset = desc_bytes + job_bytes + counter_bytes + table_bytes;
    char *buf = nullptr;
    MM_HIP(hipMallocAsync((void **)&buf, ws_offset + L.ws_bytes, st));
    build_layout(probs, order, method, variant, buf + ws_offset, &L);
    GroupedDesc *d_descs = (GroupedDesc *)buf;
    SplitJob *d_jobs = (SplitJob *)(buf + desc_bytes);
    int *d_counter = schedule == 2 ? (int *)(buf + desc_bytes + job_bytes) : nullptr;
    const size_t table_offset = desc_bytes + job_bytes + counter_bytes;
    TileRef *d_tiles = table.empty() ? nullptr : (TileRef *)(buf + table_offset);
    const Piece pieces[] = {{0, L.descs.data(), nd * sizeof(GroupedDesc)},
                            {desc_bytes, L.jobs.data(), L.jobs.size() * sizeof(SplitJob)},
                            {table_offset, table.data(), table.size() * sizeof(TileRef)}};
    mm_status s = upload_staged(buf, pieces, 3, st);
    hipError_t e = hipSuccess;
    if (s == MM_OK)
        e = grouped_enqueue(method, variant, form, d_descs, (int)nd, L.total_tiles, d_jobs, (int)L.jobs.size(),
                            L.split_tiles, d_counter, d_tiles, st);
    hipError_t e2 = hipFreeAsync(buf, st);
    if (s != MM_OK) return s;
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "grouped launch");
    return MM_OK;
}

}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_gemm_grouped(const mm_problem *probs, int32_t count, mm_method method, mm_grouped_plan **plan_inout,
                          void *stream) {
    try {
        mm_status s = validate(probs, count, method);
        if (s != MM_OK) return s;
        hipStream_t st = (hipStream_t)stream;
        if (plan_inout && *plan_inout) {
            mm_grouped_plan *p = *plan_inout;
            if (p->method != method || !same_shapes(p, probs, count))
                return fail(MM_E_INVAL, "plan was built for other shapes or another method");
            return run_plan(p, probs, st, true);
        }
        if (count == 0) return MM_OK;
        if ((s = check_arch()) != MM_OK) return s;
        int schedule = 0;
        const int variant = select_grouped(probs, count, method, &schedule);
        if (!plan_inout) return run_once(probs, count, method, variant, schedule, st);
        mm_grouped_plan *p = nullptr;
        s = create_plan(probs, count, method, variant, schedule, &p);
        if (s != MM_OK) return s;
        *plan_inout = p;
        return run_plan(p, probs, st, false);
    } catch (const std::bad_alloc &) {
        return fail(MM_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(MM_E_DEVICE, "internal error");
    }
}

mm_status mm_grouped_plan_launch(mm_grouped_plan *plan, void *stream) {
    try {
        if (!plan) return fail(MM_E_INVAL, "plan is NULL");
        return run_plan(plan, nullptr, (hipStream_t)stream, false);
    } catch (...) {
        return fail(MM_E_DEVICE, "internal error");
    }
}

mm_status mm_grouped_plan_destroy(mm_grouped_plan *plan) {
    try {
        destroy_plan(plan);
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "internal error");
    }
}

mm_status mm_grouped_plan_info(const mm_grouped_plan *plan, int32_t *variant_out, int32_t *schedule_out,
                               int64_t *tiles_out, int32_t *grid_out, int32_t *uses_graph_out) {
    if (!plan) return fail(MM_E_INVAL, "plan is NULL");
    if (variant_out) *variant_out = plan->variant;
    if (schedule_out) *schedule_out = plan->schedule;
    if (tiles_out) *tiles_out = plan->layout.total_tiles;
    if (grid_out) {
        const int form = grouped_form(plan->method, plan->variant, plan->schedule, plan->layout);
        const int64_t g = launch_grid(form, kernel_for(plan->method, plan->variant, form), plan->layout.total_tiles);
        *grid_out = (int32_t)(g < 0x7fffffffLL ? g : 0x7fffffffLL);
    }
    if (uses_graph_out) *uses_graph_out = plan->exec != nullptr;
    return MM_OK;
}

// Internal (also exported for tuning): explicit variant and schedule.
mm_status mm_gemm_grouped_config(const mm_problem *probs, int32_t count, mm_method method, int32_t variant,
                                 int32_t schedule, mm_grouped_plan **plan_inout, void *stream) {
    try {
        mm_status s = validate(probs, count, method);
        if (s != MM_OK) return s;
        if (!grouped_variant_valid(method, variant)) return fail(MM_E_INVAL, "no such variant or pair");
        if (schedule < 0 || schedule > 3) return fail(MM_E_INVAL, "schedule must be 0, 1, 2 or 3");
        hipStream_t st = (hipStream_t)stream;
        if (plan_inout && *plan_inout) {
            mm_grouped_plan *p = *plan_inout;
            if (p->method != method || !same_shapes(p, probs, count) || p->variant != variant || p->schedule != schedule)
                return fail(MM_E_INVAL, "plan was built for another configuration");
            return run_plan(p, probs, st, true);
        }
        if (count == 0) return MM_OK;
        if ((s = check_arch()) != MM_OK) return s;
        if (!plan_inout) return run_once(probs, count, method, variant, schedule, st);
        mm_grouped_plan *p = nullptr;
        s = create_plan(probs, count, method, variant, schedule, &p);
        if (s != MM_OK) return s;
        *plan_inout = p;
        return run_plan(p, probs, st, false);
    } catch (...) {
        return fail(MM_E_DEVICE, "internal error");
    }
}

int32_t mm_grouped_pair_count(mm_method method) { return grouped_pair_count(method); }

mm_status mm_grouped_pair_info(mm_method method, int32_t pair, int32_t *small_out, int32_t *large_out,
                               int32_t *pct_out) {
    PairCfg pc;
    if (pair < 0 || !grouped_pair(method, MM_PAIR_BASE + pair, &pc)) return fail(MM_E_INVAL, "no such pair");
    if (small_out) *small_out = pc.small;
    if (large_out) *large_out = pc.large;
    if (pct_out) *pct_out = pc.pct;
    return MM_OK;
}

}  // extern "C"
