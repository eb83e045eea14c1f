// Serving: a continuous-batching request loop for products of many sizes.
//
// Clients submit requests (device operands, a method and an arrival time) from
// any thread.  One scheduler thread per server:
//   * retires launches whose completion event has fired: every request in them
//     is finished, its latency (completion - arrival) recorded and its bytes
//     released;
//   * admits queued requests strictly in arrival order while the bytes in
//     flight plus the request's bytes (A, B, C and split workspace) fit in the
//     budget; the head never gets overtaken, so no request starves;
//   * packs the admitted requests into the next free slot -- one HIP stream --
//     as one grouped launch per (method, size class) present, one workgroup
//     per tile, heaviest problems first, so requests that arrive while others
//     run start as soon as a slot and budget free up and their work overlaps
//     with the launches in flight.
// Every request of a (method, size class) runs with one fixed tile variant, so
// a request's result is bit-identical alone and in any mix.
//
// Dry-run mode (dry_run_tflops > 0) replaces the device by a timing model:
// each launch completes sum(2MNK)/rate seconds after it starts; nothing is
// written.  It exists to test admission, ordering, batching and statistics on
// hosts without a GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mm_internal.h"

namespace mm {

namespace {

typedef std::chrono::steady_clock Clock;

struct Request {
    uint64_t id;
    mm_problem p;
    mm_method method;
    double arrival;
    uint64_t bytes;
    bool done = false;
    mm_status status = MM_OK;
    double latency_ms = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> ids;
    uint64_t bytes = 0;
    double flop = 0;
    double dry_done_at = 0;
    // per (method, class) group: device descriptors / split jobs and pinned
    // staging
    char *ws = nullptr;       // split workspace, grown when a batch needs more
    size_t ws_cap = 0;
    std::vector<char *> ws_retired;   // outgrown workspaces, freed with the server
    GroupedDesc *d_descs = nullptr;
    SplitJob *d_jobs = nullptr;
    GroupedDesc *h_descs = nullptr;
    SplitJob *h_jobs = nullptr;
};

constexpr int kGroups = 8;  // one grouped launch per (method, size class)

uint64_t elem_bytes(mm_method m) { return m == MM_F64 ? 8 : 4; }

// Bytes a request holds while in flight: its operands and result, plus its
// bfloat16 planes when its variant reads planes (fused split variants make
// none).
uint64_t request_bytes(const mm_problem &p, mm_method m, bool planes) {
    const uint64_t e = elem_bytes(m);
    uint64_t b = e * ((uint64_t)p.M * p.K + (uint64_t)p.K * p.N + (uint64_t)p.M * p.N);
    if (planes && (m == MM_SPLIT_BF16_3 || m == MM_SPLIT_BF16_6) && p.M > 0 && p.N > 0 && p.K > 0)
        b += 2 * 256 + split_workspace_bytes(p.M, p.N, p.K, m == MM_SPLIT_BF16_3 ? 3 : 6);
    return b;
}

// Default variant per method and size class: the single-product rule for a
// 2048^3 product (large), the untuned grouped batch's tile (small: a batch of
// small requests is one grouped launch of many small problems).
int default_serve_variant(mm_method m, bool large) {
    return large ? select_variant(m, 2048, 2048, 2048) : default_grouped_variant(m);
}

}  // namespace
}  // namespace mm

struct mm_server {
    mm_serve_config cfg;
    double dry_tflops = 0;
    uint64_t dry_fail_id = 0;
    mm::Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, mm::Request> reqs;
    uint64_t next_id = 1;
    uint64_t in_flight_bytes = 0;
    uint64_t peak_bytes = 0;
    std::vector<mm::Slot> slots;
    int variant[8];  // index: method + 4 * large
    int64_t large_mn = 0;
    std::thread thread;
    bool stopping = false;
    // statistics
    std::vector<double> latencies;
    uint64_t completed = 0, failed = 0, launches = 0, launched_requests = 0;
    double useful_flop = 0;
    double first_arrival = -1, last_done = 0;

    double now() const { return std::chrono::duration<double>(mm::Clock::now() - t0).count(); }
};

namespace mm {

static void finish(mm_server *s, Slot &slot, mm_status st) {
    const double t = s->now();
    for (uint64_t id : slot.ids) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) continue;
        Request &r = it->second;
        r.done = true;
        r.status = (s->dry_tflops > 0 && s->dry_fail_id && id == s->dry_fail_id) ? MM_E_DEVICE : st;
        r.latency_ms = (t - r.arrival) * 1e3;
        s->latencies.push_back(r.latency_ms);
        ++s->completed;
        if (r.status != MM_OK) ++s->failed;
        else s->useful_flop += 2.0 * (double)r.p.M * (double)r.p.N * (double)r.p.K;
        if (t > s->last_done) s->last_done = t;
    }
    s->in_flight_bytes -= slot.bytes;
    slot.ids.clear();
    slot.bytes = 0;
    slot.busy = false;
    s->cv_done.notify_all();
}

// Enqueue one batch on a slot.  Called with the lock held.
static mm_status launch(mm_server *s, Slot &slot, const std::vector<uint64_t> &ids) {
    slot.ids = ids;
    slot.busy = true;
    slot.bytes = 0;
    slot.flop = 0;
    for (uint64_t id : ids) {
        slot.bytes += s->reqs[id].bytes;
        slot.flop += 2.0 * (double)s->reqs[id].p.M * s->reqs[id].p.N * s->reqs[id].p.K;
    }
    ++s->launches;
    s->launched_requests += ids.size();
    if (s->dry_tflops > 0) {
        slot.dry_done_at = s->now() + slot.flop / (s->dry_tflops * 1e12);
        return MM_OK;
    }
    const int cap = s->cfg.max_batch;
    // group the batch by (method, size class) and size the split workspace
    std::vector<mm_problem> probs[kGroups];
    std::vector<int> order[kGroups];
    Layout L[kGroups];
    size_t ws_need = 0;
    for (int g = 0; g < kGroups; ++g) {
        const mm_method m = (mm_method)(g % 4);
        const bool large = g >= 4;
        for (uint64_t id : ids) {
            const Request &r = s->reqs[id];
            if (r.method == m && ((r.p.M * r.p.N >= s->large_mn) == large)) probs[g].push_back(r.p);
        }
        if (probs[g].empty()) continue;
        const int variant = s->variant[g];
        order[g] = schedule_order(probs[g].data(), (int)probs[g].size(), 3);
        build_layout(probs[g].data(), order[g], m, variant, nullptr,
                     &L[g]);
        ws_need += (L[g].ws_bytes + 255) & ~(size_t)255;
    }
    if (ws_need > slot.ws_cap) {
        // Growth doubles, and the outgrown buffer is kept until the server is
        // destroyed: hipFree waits for the whole device, which stalled every
        // other slot's launches (served p99 4.1-7.2 ms against 2.7-3.5 ms
        // with tiles that need no workspace).  Kept buffers total less than
        // the largest one.
        char *fresh = nullptr;
        const size_t want = std::max(ws_need, 2 * slot.ws_cap);
        MM_HIP(hipMalloc((void **)&fresh, want));
        if (slot.ws) slot.ws_retired.push_back(slot.ws);
        slot.ws = fresh;
        slot.ws_cap = want;
    }
    size_t ws_off = 0;
    for (int g = 0; g < kGroups; ++g) {
        if (probs[g].empty()) continue;
        const mm_method m = (mm_method)(g % 4);
        const int variant = s->variant[g];
        if (L[g].descs.empty()) continue;
        if (L[g].ws_bytes) {
            build_layout(probs[g].data(), order[g], m, variant,
                         slot.ws + ws_off, &L[g]);
            ws_off += (L[g].ws_bytes + 255) & ~(size_t)255;
        }
        GroupedDesc *hd = slot.h_descs + (size_t)g * cap;
        SplitJob *hj = slot.h_jobs + (size_t)g * 2 * cap;
        std::memcpy(hd, L[g].descs.data(), L[g].descs.size() * sizeof(GroupedDesc));
        GroupedDesc *dd = slot.d_descs + (size_t)g * cap;
        SplitJob *dj = slot.d_jobs + (size_t)g * 2 * cap;
        MM_HIP(hipMemcpyAsync(dd, hd, L[g].descs.size() * sizeof(GroupedDesc), hipMemcpyHostToDevice, slot.stream));
        if (!L[g].jobs.empty()) {
            std::memcpy(hj, L[g].jobs.data(), L[g].jobs.size() * sizeof(SplitJob));
            MM_HIP(hipMemcpyAsync(dj, hj, L[g].jobs.size() * sizeof(SplitJob), hipMemcpyHostToDevice, slot.stream));
        }
        // one workgroup per tile in tile order (grouped schedule 3): launches
        // of other slots interleave with it workgroup by workgroup (measured
        // p50/p99 0.40/3.1-3.4 ms against 0.45/3.4-3.9 ms for a persistent
        // grid pulling from a work counter, at 20k requests/s)
        MM_HIP(grouped_enqueue(m, variant, kFormTile, dd, (int)L[g].descs.size(), L[g].total_tiles, dj, (int)L[g].jobs.size(),
                               L[g].split_tiles, nullptr, nullptr, slot.stream));
    }
    MM_HIP(hipEventRecord(slot.done, slot.stream));
    return MM_OK;
}

// A launch that failed part-way may have left copies and kernels on the slot's
// stream that still read its pinned staging and the requests' operands: drain
// the stream before the slot and the requests are released.
static void finish_failed(mm_server *s, Slot &slot, mm_status st) {
    if (s->dry_tflops <= 0 && slot.stream) (void)hipStreamSynchronize(slot.stream);
    finish(s, slot, st);
}

static void scheduler_main(mm_server *s) {
    if (s->dry_tflops <= 0) (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        // 1. retire finished launches
        for (Slot &slot : s->slots) {
            if (!slot.busy) continue;
            if (s->dry_tflops > 0) {
                if (s->now() >= slot.dry_done_at) finish(s, slot, MM_OK);
                continue;
            }
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipSuccess) finish(s, slot, MM_OK);
            else if (q != hipErrorNotReady) finish(s, slot, MM_E_DEVICE);
        }
        // 2. admit in arrival order into free slots
        for (Slot &slot : s->slots) {
            if (slot.busy || s->queue.empty()) continue;
            std::vector<uint64_t> batch;
            uint64_t bytes = s->in_flight_bytes;
            while (!s->queue.empty() && (int)batch.size() < s->cfg.max_batch) {
                const Request &r = s->reqs[s->queue.front()];
                if (bytes + r.bytes > s->cfg.budget_bytes) break;  // head waits; nobody overtakes it
                bytes += r.bytes;
                batch.push_back(s->queue.front());
                s->queue.pop_front();
            }
            if (batch.empty()) break;
            s->in_flight_bytes = bytes;
            if (bytes > s->peak_bytes) s->peak_bytes = bytes;
            mm_status st;
            try {
                st = launch(s, slot, batch);
            } catch (...) {  // host allocation failure while packing the batch
                st = MM_E_NOMEM;
            }
            if (st != MM_OK) finish_failed(s, slot, st);
        }
        bool any_busy = false;
        for (Slot &slot : s->slots) any_busy = any_busy || slot.busy;
        if (s->stopping && s->queue.empty() && !any_busy) break;
        // 3. wait for work: poll completions while launches are in flight
        if (any_busy) {
            lock.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            lock.lock();
        } else {
            s->cv_work.wait(lock, [s] { return s->stopping || !s->queue.empty(); });
        }
    }
}

static void release(mm_server *s) {
    for (Slot &slot : s->slots) {
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
        if (slot.ws) (void)hipFree(slot.ws);
        for (char *w : slot.ws_retired) (void)hipFree(w);
        if (slot.d_descs) (void)hipFree(slot.d_descs);
        if (slot.d_jobs) (void)hipFree(slot.d_jobs);
        if (slot.h_descs) (void)hipHostFree(slot.h_descs);
        if (slot.h_jobs) (void)hipHostFree(slot.h_jobs);
    }
    delete s;
}

}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_serve_create(const mm_serve_config *cfg, mm_server **out) {
    try {
        if (!cfg || !out) return fail(MM_E_INVAL, "NULL argument");
        if (cfg->slots < 1 || cfg->slots > 16) return fail(MM_E_INVAL, "slots must be 1..16");
        if (cfg->max_batch < 1 || cfg->max_batch > 4096) return fail(MM_E_INVAL, "max_batch must be 1..4096");
        if (cfg->queue_capacity < 1) return fail(MM_E_INVAL, "queue_capacity must be positive");
        if (cfg->budget_bytes == 0) return fail(MM_E_INVAL, "budget_bytes must be positive");
        for (int m = 0; m < 4; ++m)
            if (cfg->variants[m] < -1 || cfg->variants[m] >= mm_variant_count((mm_method)m) ||
                cfg->variants_large[m] < -1 || cfg->variants_large[m] >= mm_variant_count((mm_method)m))
                return fail(MM_E_INVAL, "no such variant for method " + std::to_string(m));
        if (cfg->large_mn < 0) return fail(MM_E_INVAL, "large_mn must be >= 0");
        mm_server *s = new mm_server();
        s->cfg = *cfg;
        s->large_mn = cfg->large_mn > 0 ? cfg->large_mn : (int64_t)1024 * 1024;
        for (int m = 0; m < 4; ++m) {
            s->variant[m] = cfg->variants[m] >= 0 ? cfg->variants[m] : default_serve_variant((mm_method)m, false);
            s->variant[m + 4] =
                cfg->variants_large[m] >= 0 ? cfg->variants_large[m] : default_serve_variant((mm_method)m, true);
        }
        s->dry_tflops = cfg->dry_run_tflops;
        s->dry_fail_id = cfg->dry_run_fail_id;
        s->t0 = Clock::now();
        s->slots.resize(cfg->slots);
        if (s->dry_tflops <= 0) {
            hipError_t e = hipSetDevice(cfg->device);
            if (e == hipSuccess) {
                const mm_status as = check_arch();
                if (as != MM_OK) {
                    release(s);
                    return as;
                }
            }
            const size_t cap = cfg->max_batch;
            for (Slot &slot : s->slots) {
                if (e == hipSuccess) e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
                if (e == hipSuccess) e = hipMalloc(&slot.d_descs, kGroups * cap * sizeof(GroupedDesc));
                if (e == hipSuccess) e = hipMalloc(&slot.d_jobs, kGroups * 2 * cap * sizeof(SplitJob));
                if (e == hipSuccess) e = hipHostMalloc((void **)&slot.h_descs, kGroups * cap * sizeof(GroupedDesc), 0);
                if (e == hipSuccess) e = hipHostMalloc((void **)&slot.h_jobs, kGroups * 2 * cap * sizeof(SplitJob), 0);
            }
            if (e != hipSuccess) {
                release(s);
                return hip_fail(e, "server setup");
            }
        }
        s->thread = std::thread(scheduler_main, s);
        *out = s;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "server setup failed");
    }
}

mm_status mm_serve_submit(mm_server *s, const mm_problem *req, mm_method method, double arrival_s, uint64_t *id_out) {
    try {
        if (!s || !req || !id_out) return fail(MM_E_INVAL, "NULL argument");
        if (method < MM_F64 || method > MM_SPLIT_BF16_6) return fail(MM_E_INVAL, "unknown method");
        const uint64_t e = elem_bytes(method);
        mm_status st = check_gemm_args(req->M, req->N, req->K, req->A, req->lda, req->B, req->ldb, req->C, req->ldc, e, e);
        if (st == MM_OK && method >= MM_SPLIT_BF16_3) st = check_split_k(req->K);
        if (st != MM_OK) return st;
        // the size class decides the variant, and the variant whether planes exist
        const int group = (int)method + (req->M * req->N >= s->large_mn ? 4 : 0);
        const uint64_t bytes = request_bytes(*req, method, !split_variant_fused(s->variant[group]));
        if (bytes > s->cfg.budget_bytes) return fail(MM_E_NOMEM, "request larger than the server budget");
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stopping) return fail(MM_E_INVAL, "server is stopping");
        if ((int64_t)s->queue.size() >= s->cfg.queue_capacity) return fail(MM_E_BUSY, "queue full");
        Request r;
        r.id = s->next_id++;
        r.p = *req;
        r.method = method;
        r.arrival = arrival_s >= 0 ? arrival_s : s->now();
        r.bytes = bytes;
        if (s->first_arrival < 0 || r.arrival < s->first_arrival) s->first_arrival = r.arrival;
        s->reqs.emplace(r.id, r);
        s->queue.push_back(r.id);
        *id_out = r.id;
        s->cv_work.notify_one();
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "submit failed");
    }
}

mm_status mm_serve_wait(mm_server *s, uint64_t id, int64_t timeout_us, mm_status *req_status, double *latency_ms) {
    try {
        if (!s) return fail(MM_E_INVAL, "NULL server");
        std::unique_lock<std::mutex> lock(s->mu);
        if (s->reqs.find(id) == s->reqs.end()) return fail(MM_E_INVAL, "unknown request id (or already waited for)");
        // A request leaves the table when its first waiter collects it; another
        // thread waiting on the same id then wakes and reports it as unknown.
        auto ready = [&] {
            auto it = s->reqs.find(id);
            return it == s->reqs.end() || it->second.done;
        };
        if (timeout_us < 0) s->cv_done.wait(lock, ready);
        else if (!s->cv_done.wait_for(lock, std::chrono::microseconds(timeout_us), ready))
            return fail(MM_E_TIMEOUT, "request still pending");
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return fail(MM_E_INVAL, "request already collected by another waiter");
        const Request r = it->second;
        s->reqs.erase(it);
        s->cv_done.notify_all();
        if (req_status) *req_status = r.status;
        if (latency_ms) *latency_ms = r.latency_ms;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "wait failed");
    }
}

double mm_serve_clock(const mm_server *s) { return s ? s->now() : 0.0; }

mm_status mm_serve_stats(mm_server *s, mm_serve_stats_t *out) {
    try {
        if (!s || !out) return fail(MM_E_INVAL, "NULL argument");
        std::lock_guard<std::mutex> lock(s->mu);
        std::memset(out, 0, sizeof *out);
        out->completed = s->completed;
        out->failed = s->failed;
        std::vector<double> lat = s->latencies;
        std::sort(lat.begin(), lat.end());
        if (!lat.empty()) {
            // nearest rank: the ceil(q*n)-th smallest
            auto rank = [&](double q) { return lat[std::max<size_t>(1, (size_t)std::ceil(q * lat.size())) - 1]; };
            out->p50_ms = rank(0.50);
            out->p99_ms = rank(0.99);
            double sum = 0;
            for (double v : lat) sum += v;
            out->mean_ms = sum / lat.size();
            out->max_ms = lat.back();
        }
        out->useful_flop = s->useful_flop;
        out->first_arrival_s = s->first_arrival < 0 ? 0 : s->first_arrival;
        out->last_done_s = s->last_done;
        const double span = s->last_done - out->first_arrival_s;
        out->tflops = span > 0 ? s->useful_flop / span / 1e12 : 0;
        out->peak_bytes = s->peak_bytes;
        out->launches = s->launches;
        out->mean_batch = s->launches ? (double)s->launched_requests / s->launches : 0;
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "stats failed");
    }
}

mm_status mm_serve_destroy(mm_server *s) {
    try {
        if (!s) return MM_OK;
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->stopping = true;
            s->cv_work.notify_all();
        }
        if (s->thread.joinable()) s->thread.join();
        release(s);
        return MM_OK;
    } catch (...) {
        return fail(MM_E_DEVICE, "destroy failed");
    }
}

}  // extern "C"
