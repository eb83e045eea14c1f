// Tile-variant selection and the autotuner.
//
// The variant used for a product is a pure function of (method, M, N, K) and
// the loaded cache: a cache entry written by mm_autotune for the shape's
// bucket (method, ceil(log2 M), ceil(log2 N), ceil(log2 K)) wins, otherwise a
// fixed cost model over the exact shape applies.  Selection never depends on load or timing at call time,
// so the same shape always runs the same kernel (results are reproducible
// bit for bit, alone or inside a batch).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "mm_internal.h"

namespace mm {

namespace {

typedef std::tuple<int, int, int, int> Key;

struct Entry {
    int variant;
    double ms;
    int schedule;   // grouped entries only
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;

int clog2(int64_t x) {
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

Key key_of(mm_method m, int64_t M, int64_t N, int64_t K) {
    return Key((int)m, clog2(M), clog2(N), clog2(K));
}

// Default rule: a cost model over a few candidate tiles per method.  Tiles
// are dealt round-robin over the 256 compute units, so the busiest unit
// computes ceil(tiles / 256) of them, each at 1/256 of the rate the variant
// sustains on a large product (measured on MI355X, in TFLOP/s of 2MNK).  The
// model picks the candidate whose busiest unit finishes first; it charges
// the padding of ragged edge tiles and the idle units of a small grid, which
// is what decides between tile sizes.  Split variants that read planes are
// also charged their plane pass: the FP32 operands read once and the planes
// written once at 5.5 TB/s, plus 6 us for its two launches; fused split
// variants have no pass.
struct Candidate {
    int variant;
    int bm, bn;
    double rate;
    bool plane_pass;
};

// The large binary64 tile is the 16-wave 256x128 ring (64x32 wave tiles, four
// waves per SIMD): equal to the 8-wave one at 8192, 2-8% faster at 3072-6144.
// FP32 adds the 16-wave 256x256 ring (64x64 wave tiles: half the fragment
// reads and barriers per product of the 256x128 one; 146.5 against 142.6
// TFLOP/s at 8192, +2.7% at 4096 and 16384).
// The 16-wave 128x128 binary64 ring (32x32 wave tiles, K step 32) is the
// large candidate: 15.32 against 15.44 ms for the 256x128 ring at 8192, 6.49
// against 7.25-7.30 at 6144, equal at 4096, and the best at 1792-2048.
// The binary64 32x32 candidate is the 2-buffer ring with a K step of 32 (half
// the barriers of the 16-step rings): 640: 16.4 against 20.6 us for the
// 4-buffer 16-step ring, 768: 24.6 against 31.3, 1280: 86 against 92 (64x64),
// 1536: 126 against 129 (64x32); 2-4% behind the 64x64 and 64x32 rings at
// 2304-2560, which its rate leaves to them from 2560.
// The binary64 64x64 candidate is the 16-wave ring (16x16 wave tiles, K step
// 32): four waves per SIMD where one 64x64 tile per CU leaves the 4-wave ring
// one (1024: 43-46 against 47-48 us; 6144: 6.99 against 7.27 ms; equal at
// 3072 and 5120).
// The 64x32 ring runs at 0.87x the 64x64 ring's rate on a full grid (2048:
// 293 against 255 us) but splits the work finer, so it wins where the 64x64
// grid leaves its last round of CUs mostly empty (1536: 131 against 147 us,
// 1792: 209 against 221); the 32x32 ring with a K step of 32 has since taken
// those sizes, and the rate here (58) leaves it the near-ties only.  The FP32
// 32x64 ring does the same for the FP32
// 64x64 one: even on a grid of equal rounds (2048: 149 against 141 us) it is
// within 6%, and it wins where it leaves fewer rounds (1536: +14%, 1792: +5%,
// 2560: +2%).
const Candidate kF64Cand[] = {{18, 128, 128, 71.6, false}, {15, 256, 128, 71.0, false}, {3, 128, 64, 56.5, false},
                              {17, 64, 64, 67.5, false}, {19, 32, 32, 59.5, false}, {16, 64, 32, 58.0, false}};
const Candidate kF32Cand[] = {{14, 256, 256, 146.5, false}, {13, 256, 128, 142.6, false}, {3, 128, 128, 126.5, false},
                              {8, 64, 64, 141.0, false}, {10, 32, 32, 95.0, false}, {15, 32, 64, 134.0, false}};
const Candidate kSplit3Unfused[] = {{14, 256, 128, 438.0, true}, {6, 128, 128, 364.0, true}, {8, 64, 64, 319.0, true}};
const Candidate kSplit6Unfused[] = {{9, 256, 128, 214.0, true}, {6, 128, 128, 190.0, true}, {8, 64, 64, 100.4, true}};
// Fused candidates are the ring forms with one K step in flight and paired
// LDS lines (64x64 and 128x64; rates at 8192 on MI355X), which replaced the
// register-staged fused tiles at every size measured (512 ... 8192).
const Candidate kSplit3Cand[] = {{14, 256, 128, 438.0, true}, {6, 128, 128, 364.0, true}, {8, 64, 64, 319.0, true},
                                 {15, 64, 64, 236.0, false},  {16, 128, 64, 265.0, false}};
const Candidate kSplit6Cand[] = {{9, 256, 128, 214.0, true}, {6, 128, 128, 190.0, true}, {8, 64, 64, 100.4, true},
                                 {15, 64, 64, 154.6, false}, {16, 128, 64, 166.7, false}};

constexpr double kCUs = 256.0;

template <size_t NC>
int pick(const Candidate (&c)[NC], int64_t M, int64_t N, int64_t K, int planes) {
    int best = c[0].variant;
    double best_t = 0;
    bool have = false;
    const double k = (double)std::max<int64_t>(K, 1);
    for (size_t i = 0; i < NC; ++i) {
        const double tiles = (double)((M + c[i].bm - 1) / c[i].bm) * (double)((N + c[i].bn - 1) / c[i].bn);
        double t = std::ceil(tiles / kCUs) * 2.0 * c[i].bm * c[i].bn * k * kCUs / (c[i].rate * 1e12);
        if (c[i].plane_pass) t += ((double)M * k + k * (double)N) * (4.0 + 2.0 * planes) / 5.5e12 + 6e-6;
        if (!have || t < best_t) {
            best = c[i].variant;
            best_t = t;
            have = true;
        }
    }
    return best;
}

}  // namespace

int default_unfused_split_variant(mm_method method, int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0) return 1;
    return method == MM_SPLIT_BF16_3 ? pick(kSplit3Unfused, M, N, K, 2) : pick(kSplit6Unfused, M, N, K, 3);
}

namespace {

int default_variant(mm_method method, int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0) return 1;
    switch (method) {
        case MM_F64: return pick(kF64Cand, M, N, K, 0);
        case MM_F32: return pick(kF32Cand, M, N, K, 0);
        case MM_SPLIT_BF16_3: return pick(kSplit3Cand, M, N, K, 2);
        case MM_SPLIT_BF16_6: return pick(kSplit6Cand, M, N, K, 3);
    }
    return 0;
}

// Grouped batches are keyed by (100 + method, ceil(log2 count),
// ceil(log2 mean(M*N)), ceil(log2 mean K)).
Key grouped_key(const mm_problem *probs, int count, mm_method method) {
    double mn = 0, k = 0;
    for (int i = 0; i < count; ++i) {
        mn += (double)probs[i].M * probs[i].N;
        k += (double)probs[i].K;
    }
    const int64_t c = count > 0 ? count : 1;
    return Key(100 + (int)method, clog2(c), clog2((int64_t)(mn / c + 0.5)), clog2((int64_t)(k / c + 0.5)));
}

}  // namespace

// Tile variant of untuned grouped batches: 64x64 tiles (the 2-buffer direct
// ring for binary64 and FP32, the ring-fused split for the split methods) --
// among the autotuner's best on the 512-problem batch of dimensions 32..1024
// (binary64: 0.584 ms against 0.607-0.653 for the 3-buffer ring).
int default_grouped_variant(mm_method method) {
    switch (method) {
        case MM_F64: return 7;
        case MM_F32: return 8;
        default: return 15;
    }
}

// Default for grouped batches: 64x64 tiles (many small problems are dominated
// by tile quantisation and balance), heaviest problems first, one workgroup
// per tile.
int select_grouped(const mm_problem *probs, int count, mm_method method, int *schedule) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_cache.find(grouped_key(probs, count, method));
        if (it != g_cache.end()) {
            *schedule = it->second.schedule;
            return it->second.variant;
        }
    }
    *schedule = 3;
    return default_grouped_variant(method);
}

void store_grouped(const mm_problem *probs, int count, mm_method method, int variant, int schedule, double ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[grouped_key(probs, count, method)] = Entry{variant, ms, schedule};
}

// The FP32 256x256 ring's register-staged body (which runs operands the
// direct loads cannot take) holds more than the 128 registers its occupancy
// allows and spills: 101 against 131 TFLOP/s for the 256x128 variant's at
// 8192.  Such operands run the 256x128 variant instead.
int variant_for_operands(mm_method method, int variant, bool direct_ok) {
    if (!direct_ok && method == MM_F32 && variant == 14) return 13;
    return variant;
}

int select_variant(mm_method method, int64_t M, int64_t N, int64_t K) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_cache.find(key_of(method, M, N, K));
        if (it != g_cache.end()) return it->second.variant;
    }
    return default_variant(method, M, N, K);
}

}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_autotune(mm_method method, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
                      int64_t ldb, void *C, int64_t ldc, int32_t warmup, int32_t reps, int32_t *variant_out,
                      double *ms_out, void *stream) {
    try {
        if (warmup < 0 || reps < 1) return fail(MM_E_INVAL, "warmup >= 0 and reps >= 1 required");
        if (M <= 0 || N <= 0 || K <= 0) return fail(MM_E_INVAL, "autotune needs a non-empty product");
        const int nv = mm_variant_count(method);
        if (nv <= 0) return fail(MM_E_INVAL, "unknown method");
        hipStream_t st = (hipStream_t)stream;
        void *ws = nullptr;
        size_t ws_bytes = 0;
        if (method == MM_SPLIT_BF16_3 || method == MM_SPLIT_BF16_6) {
            ws_bytes = mm_split_workspace_bytes(M, N, K, method == MM_SPLIT_BF16_3 ? 3 : 6);
            MM_HIP(hipMalloc(&ws, ws_bytes));
        }
        hipEvent_t e0, e1;
        MM_HIP(hipEventCreate(&e0));
        MM_HIP(hipEventCreate(&e1));
        int best = -1;
        double best_ms = 0;
        mm_status status = MM_OK;
        for (int v = 0; v < nv && status == MM_OK; ++v) {
            std::vector<float> times;
            for (int r = 0; r < warmup + reps && status == MM_OK; ++r) {
                if (hipEventRecord(e0, st) != hipSuccess) { status = MM_E_DEVICE; break; }
                status = mm_gemm_variant(method, v, M, N, K, A, lda, B, ldb, C, ldc, ws, ws_bytes, stream);
                if (status != MM_OK) break;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    status = MM_E_DEVICE;
                    break;
                }
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    status = MM_E_DEVICE;
                    break;
                }
                if (r >= warmup) times.push_back(ms);
            }
            if (status != MM_OK) break;
            std::sort(times.begin(), times.end());
            const double med = times[times.size() / 2];
            if (best < 0 || med < best_ms) {
                best = v;
                best_ms = med;
            }
        }
        // best-effort cleanup: a failure here cannot change the measurement
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ws) (void)hipFree(ws);
        if (status != MM_OK) return status;
        {
            std::lock_guard<std::mutex> lock(g_mu);
            g_cache[key_of(method, M, N, K)] = Entry{best, best_ms, 0};
        }
        if (variant_out) *variant_out = best;
        if (ms_out) *ms_out = best_ms;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "autotune failed");
    }
}

mm_status mm_gemm_grouped_config(const mm_problem *probs, int32_t count, mm_method method, int32_t variant,
                                 int32_t schedule, mm_grouped_plan **plan_inout, void *stream);

mm_status mm_grouped_autotune(const mm_problem *probs, int32_t count, mm_method method, int32_t warmup, int32_t reps,
                              int32_t *variant_out, int32_t *schedule_out, double *ms_out, void *stream) {
    try {
        if (warmup < 0 || reps < 1) return fail(MM_E_INVAL, "warmup >= 0 and reps >= 1 required");
        if (count <= 0 || !probs) return fail(MM_E_INVAL, "autotune needs a non-empty batch");
        const int nv = mm_variant_count(method);
        if (nv <= 0) return fail(MM_E_INVAL, "unknown method");
        // every tile variant, then every size-class pair
        std::vector<int> ids;
        for (int v = 0; v < nv; ++v) ids.push_back(v);
        for (int p = 0; p < grouped_pair_count(method); ++p) ids.push_back(MM_PAIR_BASE + p);
        hipStream_t st = (hipStream_t)stream;
        hipEvent_t e0, e1;
        MM_HIP(hipEventCreate(&e0));
        MM_HIP(hipEventCreate(&e1));
        int best_v = -1, best_s = 0;
        double best_ms = 0;
        mm_status status = MM_OK;
        for (size_t vi = 0; vi < ids.size() && status == MM_OK; ++vi) {
            const int v = ids[vi];
            for (int sch = 0; sch <= 3 && status == MM_OK; ++sch) {
                mm_grouped_plan *plan = nullptr;
                std::vector<float> times;
                for (int r = 0; r < warmup + reps; ++r) {
                    if (hipEventRecord(e0, st) != hipSuccess) { status = MM_E_DEVICE; break; }
                    status = mm_gemm_grouped_config(probs, count, method, v, sch, &plan, stream);
                    if (status != MM_OK) break;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        status = MM_E_DEVICE;
                        break;
                    }
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        status = MM_E_DEVICE;
                        break;
                    }
                    if (r >= warmup) times.push_back(ms);
                }
                if (plan) {
                    if (hipStreamSynchronize(st) != hipSuccess) status = MM_E_DEVICE;
                    (void)mm_grouped_plan_destroy(plan);
                }
                if (status != MM_OK) break;
                std::sort(times.begin(), times.end());
                const double med = times[times.size() / 2];
                if (best_v < 0 || med < best_ms) {
                    best_v = v;
                    best_s = sch;
                    best_ms = med;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (status != MM_OK) return status;
        store_grouped(probs, count, method, best_v, best_s, best_ms);
        if (variant_out) *variant_out = best_v;
        if (schedule_out) *schedule_out = best_s;
        if (ms_out) *ms_out = best_ms;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "grouped autotune failed");
    }
}

mm_status mm_autotune_clear(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
    return MM_OK;
}

// File format (one JSON object):
// {"arch": "gfx950", "version": "...", "entries": [[k0, k1, k2, k3, variant, ms, schedule], ...]}
mm_status mm_autotune_save(const char *path) {
    try {
        if (!path) return fail(MM_E_INVAL, "path is NULL");
        std::ostringstream os;
        os << "{\"arch\": \"gfx950\", \"version\": \"" << mm_version() << "\", \"entries\": [";
        {
            std::lock_guard<std::mutex> lock(g_mu);
            bool first = true;
            for (auto &kv : g_cache) {
                if (!first) os << ", ";
                first = false;
                os << "[" << std::get<0>(kv.first) << ", " << std::get<1>(kv.first) << ", " << std::get<2>(kv.first)
                   << ", " << std::get<3>(kv.first) << ", " << kv.second.variant << ", " << kv.second.ms << ", "
                   << kv.second.schedule << "]";
            }
        }
        os << "]}\n";
        std::string tmp = std::string(path) + ".tmp";
        {
            std::ofstream f(tmp);
            if (!f) return fail(MM_E_INVAL, std::string("cannot write ") + tmp);
            f << os.str();
            if (!f) return fail(MM_E_INVAL, std::string("write failed: ") + tmp);
        }
        if (std::rename(tmp.c_str(), path) != 0) return fail(MM_E_INVAL, std::string("cannot rename to ") + path);
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "autotune save failed");
    }
}

static bool find_string_field(const std::string &s, const char *name, std::string *out) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t p = s.find(pat);
    if (p == std::string::npos) return false;
    p = s.find('"', s.find(':', p + pat.size()));
    if (p == std::string::npos) return false;
    size_t e = s.find('"', p + 1);
    if (e == std::string::npos) return false;
    *out = s.substr(p + 1, e - p - 1);
    return true;
}

mm_status mm_autotune_load(const char *path) {
    try {
        if (!path) return fail(MM_E_INVAL, "path is NULL");
        std::ifstream f(path);
        if (!f) return fail(MM_E_INVAL, std::string("cannot read ") + path);
        std::stringstream ss;
        ss << f.rdbuf();
        const std::string s = ss.str();
        std::string arch, version;
        if (!find_string_field(s, "arch", &arch) || arch != "gfx950")
            return fail(MM_E_INVAL, "autotune cache is for another architecture");
        if (!find_string_field(s, "version", &version) || version != mm_version())
            return fail(MM_E_INVAL, "autotune cache is for another library version");
        size_t p = s.find("\"entries\"");
        if (p == std::string::npos) return fail(MM_E_INVAL, "no entries");
        p = s.find('[', p);
        if (p == std::string::npos) return fail(MM_E_INVAL, "malformed entries");
        std::map<Key, Entry> fresh;
        ++p;
        while (true) {
            size_t open = s.find('[', p);
            size_t close_all = s.find(']', p);
            if (open == std::string::npos || (close_all != std::string::npos && close_all < open)) break;
            size_t close = s.find(']', open);
            if (close == std::string::npos) return fail(MM_E_INVAL, "malformed entry");
            double v[7];
            if (std::sscanf(s.c_str() + open + 1, "%lf , %lf , %lf , %lf , %lf , %lf , %lf", &v[0], &v[1], &v[2],
                            &v[3], &v[4], &v[5], &v[6]) != 7)
                return fail(MM_E_INVAL, "malformed entry");
            const int k0 = (int)v[0], variant = (int)v[4], schedule = (int)v[6];
            const int method = k0 >= 100 ? k0 - 100 : k0;
            // grouped entries (key 100 + method) may name a size-class pair
            const bool known = method >= 0 && method <= 3 &&
                               (k0 >= 100 ? grouped_variant_valid((mm_method)method, variant)
                                          : variant >= 0 && variant < mm_variant_count((mm_method)method));
            if (!known || schedule < 0 || schedule > 3)
                return fail(MM_E_INVAL, "entry names an unknown method, variant or schedule");
            fresh[Key(k0, (int)v[1], (int)v[2], (int)v[3])] = Entry{variant, v[5], schedule};
            p = close + 1;
        }
        std::lock_guard<std::mutex> lock(g_mu);
        g_cache = fresh;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "autotune load failed");
    }
}

}  // extern "C"
