// Autotuner: picks the pre-placement depth and the persistent launch shape
// (workgroup size, waves per CU, steps between scheduler visits, entries per
// work-head claim) for a board size by timing full counts on the device; for
// the boards whose count runs in chunks (N = 21..23), the depth, timed on one
// chunk.
//
// The paper tunes the pre-placed rows and the block/stack configuration by
// hand (Section 4.1, Table 3; Section 4.2, Table 4); here the same choices are
// measured.  The search is coordinate-wise: depth first (with the default
// launch shape), then the workgroup size, waves per CU, the visit interval and
// the size of the per-wave claimed blocks (the persistent scheduler's
// counterpart of a queue depth), each trial a complete persistent count over
// the resident frontier, stopping early when the time budget is spent.  Every
// trial is recorded for the caller.  Results are kept per (device, n) for the
// process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "nq_internal.h"

namespace nqi {

namespace {

struct TuneKey {
    int device;
    uint32_t n;
    bool operator<(const TuneKey& o) const {
        return device != o.device ? device < o.device : n < o.n;
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, nq_tuned> g_tune_cache;

// The frontier of one trial depth, resident on the device for the tuning,
// with the trial's 8-byte total.
struct TrialFrontier {
    DeviceFrontier fr;
    unsigned long long* total = nullptr;
    ~TrialFrontier() {
        if (total) (void)hipFree(total);
    }
    int load(uint32_t n, uint32_t depth, hipStream_t s) {
        int rc = build_device_frontier(n, depth, s, &fr);
        if (rc != NQ_OK) return rc;
        hipError_t e = hipMalloc((void**)&total, 16);
        if (e != hipSuccess) {
            set_hip_error(e);
            total = nullptr;
            return e == hipErrorOutOfMemory ? NQ_ENOMEM : NQ_EDEVICE;
        }
        return NQ_OK;
    }
};

// One timed persistent count; *ms is the device time of zero + DFS.
int trial(uint32_t n, uint32_t depth, const TrialFrontier& tf, uint32_t wg_size,
          uint32_t waves_per_cu, uint32_t refill, uint32_t claim, hipStream_t s, double* ms,
          uint64_t* total_out) {
    const DeviceFrontier& fr = tf.fr;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    const uint32_t frames = std::max<uint32_t>(1, frames_needed(n, depth));
    LaunchCfg cfg;
    rc = plan_launch(dev, NQ_MODE_PERSISTENT, wg_size, waves_per_cu, frames, fr.len, false,
                     leafctr_ok(n, depth), &cfg, false, false, n);
    if (rc != NQ_OK) return rc;
    DfsParams P{};
    P.cols = fr.cols; P.ld = fr.ld; P.rd = fr.rd; P.weight = fr.w;
    P.totals = tf.total; P.head = tf.total + 1;
    P.len = fr.len; P.n = n; P.frames = frames; P.refill_every = refill; P.reverse = 1;
    P.idle_min = default_idle_min();
    P.claim = claim ? claim : default_claim(fr.len, cfg);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        set_hip_error(e);
        if (a) (void)hipEventDestroy(a);
        return NQ_EDEVICE;
    }
    rc = NQ_OK;
    e = hipEventRecord(a, s);
    if (e == hipSuccess) {
        rc = launch_zero_u64(tf.total, 1, s);
        if (rc == NQ_OK) rc = launch_dfs(cfg, P, s);
        e = hipEventRecord(b, s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    unsigned long long t = 0;
    if (e == hipSuccess) e = hipMemcpy(&t, tf.total, 8, hipMemcpyDeviceToHost);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    if (rc != NQ_OK) return rc;
    *ms = f;
    *total_out = t;
    return NQ_OK;
}

// Boards whose count runs in chunks: the depth is measured on one chunk (the
// middle one of the plan's chunk count), which every depth counts the same
// way, in wall-clock time, since a deeper chunk also spends more time in its
// device expansion.  The first depth is timed twice (the first run also loads
// the code objects).
int autotune_chunked(uint32_t n, const ChunkPlan& plan, uint32_t lo, uint32_t hi,
                     double budget_ms, nq_tuned* out, nq_tune_trial* table, uint32_t capacity,
                     uint32_t* out_count) {
    if (lo == 0) lo = std::max(kChunkHostDepth, plan.depth - 1);
    if (hi == 0) hi = std::min(n - 2, plan.depth + 1);
    if (lo < kChunkHostDepth || lo > hi || hi > n) return NQ_EINVAL;
    if (budget_ms <= 0) budget_ms = 60000.0;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{s};
    nq_opts o{};
    o.mode = NQ_MODE_PERSISTENT;
    o.stream = s;
    const uint32_t index = plan.chunks / 2;
    nq_tuned best{};
    best.ms = 1e300;
    double spent = 0.0;
    unsigned __int128 expect = 0;
    bool have_expect = false;
    uint32_t trials = 0;
    for (uint32_t d = lo; d <= hi && spent < budget_ms; ++d) {
        for (int rep = 0; rep < (d == lo ? 2 : 1) && spent < budget_ms; ++rep) {
            double ms = 0.0;
            unsigned __int128 total = 0;
            const int rc = time_chunk(n, d, plan.chunks, index, o, &ms, &total);
            if (rc != NQ_OK) return rc;
            if (table && trials < capacity)
                table[trials] = nq_tune_trial{d, 0u, 0u, 0u, 0u, plan.chunks, ms, 0u};
            ++trials;
            spent += ms;
            if (have_expect && total != expect) return NQ_EDEVICE;   // counts must agree
            expect = total;
            have_expect = true;
            if (ms < best.ms) {
                best.depth = d;
                best.ms = ms;
            }
        }
    }
    best.chunks = plan.chunks;
    best.trials = trials;
    best.count = (uint64_t)expect;          // a chunk of n <= 23: below 2^64
    if (out_count) *out_count = std::min(trials, table ? capacity : 0u);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{dev, n}] = best;
    }
    *out = best;
    return NQ_OK;
}

}  // namespace

int tune_lookup(uint32_t n, nq_tuned* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NQ_ENOENT;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find({dev, n});
    if (it == g_tune_cache.end()) return NQ_ENOENT;
    *out = it->second;
    return NQ_OK;
}

int autotune(uint32_t n, uint32_t depth_lo, uint32_t depth_hi, double budget_ms, nq_tuned* out,
             nq_tune_trial* table, uint32_t capacity, uint32_t* out_count) {
    if (n < 4 || n > NQ_MAX_N || !out || (table && !capacity)) return NQ_EINVAL;
    if (const ChunkPlan* plan = chunk_plan(n))
        return autotune_chunked(n, *plan, depth_lo, depth_hi, budget_ms, out, table, capacity,
                                out_count);
    if (depth_lo == 0) depth_lo = std::max<uint32_t>(1, std::min<uint32_t>(n - 2, n > 12 ? n - 14 : 1));
    if (depth_hi == 0) depth_hi = std::min<uint32_t>(n - 2, depth_lo + 4);
    if (depth_lo > depth_hi || depth_hi > n) return NQ_EINVAL;
    if (budget_ms <= 0) budget_ms = 60000.0;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{s};

    nq_tuned best{};
    best.ms = 1e300;
    double spent = 0.0;
    uint64_t expect = 0;
    bool have_expect = false;
    uint32_t trials = 0;
    auto consider = [&](uint32_t depth, const TrialFrontier& fr, uint32_t wg, uint32_t wpc,
                        uint32_t rf, uint32_t claim) -> int {
        double ms = 0;
        uint64_t total = 0;
        int rc = trial(n, depth, fr, wg, wpc, rf, claim, s, &ms, &total);
        if (rc == NQ_EINVAL && wg != 0) return NQ_OK;   // this workgroup size does not fit
        if (rc != NQ_OK) return rc;
        if (table && trials < capacity)
            table[trials] = nq_tune_trial{depth, wg, wpc, rf, claim, 0u, ms, fr.fr.len};
        ++trials;
        spent += ms;
        if (have_expect && total != expect) return NQ_EDEVICE;   // counts must agree
        expect = total;
        have_expect = true;
        if (ms < best.ms) {
            best.depth = depth; best.wg_size = wg; best.waves_per_cu = wpc;
            best.refill_every = rf; best.claim = claim; best.ms = ms;
        }
        return NQ_OK;
    };

    try {
        // 1. depth, default launch shape.  Each depth is timed twice, the first
        //    run also warming the code object.
        for (uint32_t d = depth_lo; d <= depth_hi && spent < budget_ms; ++d) {
            TrialFrontier fr;
            int rc = fr.load(n, d, s);
            if (rc != NQ_OK) return rc;
            for (int rep = 0; rep < 2 && spent < budget_ms; ++rep)
                if ((rc = consider(d, fr, 0, 0, 512, 0)) != NQ_OK) return rc;
        }
        // 2. workgroup size, waves per CU, the visit interval and the claim
        //    block at the best depth (0 = the default of each).
        TrialFrontier fr;
        int rc = fr.load(n, best.depth, s);
        if (rc != NQ_OK) return rc;
        const uint32_t d = best.depth;
        for (uint32_t wg : {64u, 128u, 256u}) {
            if (spent >= budget_ms) break;
            if ((rc = consider(d, fr, wg, 0, best.refill_every, best.claim)) != NQ_OK) return rc;
        }
        for (uint32_t wpc : {8u, 16u, 24u}) {
            if (spent >= budget_ms) break;
            if ((rc = consider(d, fr, best.wg_size, wpc, best.refill_every, best.claim)) != NQ_OK)
                return rc;
        }
        for (uint32_t rf : {128u, 2048u}) {
            if (spent >= budget_ms) break;
            if ((rc = consider(d, fr, best.wg_size, best.waves_per_cu, rf, best.claim)) != NQ_OK)
                return rc;
        }
        for (uint32_t cl : {32u, 1024u}) {
            if (spent >= budget_ms) break;
            if ((rc = consider(d, fr, best.wg_size, best.waves_per_cu, best.refill_every, cl)) !=
                NQ_OK)
                return rc;
        }
    } catch (const std::bad_alloc&) {
        return NQ_ENOMEM;
    }
    best.trials = trials;
    best.count = expect;
    if (out_count) *out_count = std::min(trials, table ? capacity : 0u);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{dev, n}] = best;
    }
    *out = best;
    return NQ_OK;
}

}  // namespace nqi

extern "C" int nq_autotune(uint32_t n, uint32_t depth_lo, uint32_t depth_hi, double budget_ms,
                           nq_tuned* out) {
    try {
        return nqi::autotune(n, depth_lo, depth_hi, budget_ms, out, nullptr, 0, nullptr);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_autotune_trials(uint32_t n, uint32_t depth_lo, uint32_t depth_hi,
                                  double budget_ms, nq_tuned* out, nq_tune_trial* trials,
                                  uint32_t capacity, uint32_t* out_count) {
    if (!trials || !out_count) return NQ_EINVAL;
    try {
        return nqi::autotune(n, depth_lo, depth_hi, budget_ms, out, trials, capacity, out_count);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_tuned_lookup(uint32_t n, nq_tuned* out) {
    if (n < 1 || n > NQ_MAX_N || !out) return NQ_EINVAL;
    try {
        return nqi::tune_lookup(n, out);
    } catch (...) {
        return NQ_ENOMEM;
    }
}
