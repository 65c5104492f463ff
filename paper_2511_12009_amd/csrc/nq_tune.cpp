// Autotuner: picks the pre-placement depth and the persistent launch shape
// (waves per CU, steps between scheduler visits) for a board size by timing
// full counts on the device.
//
// The paper tunes the pre-placed rows and the block/stack configuration by
// hand (Section 4.1, Table 3; Section 4.2, Table 4); here the same choices are
// measured.  The search is coordinate-wise: depth first (with the default
// launch shape), then waves per CU, the visit interval and the size of the
// per-wave claimed blocks, each trial a
// complete persistent count over the resident frontier, stopping early when the
// time budget is spent.  Results are kept per (device, n) for the process.
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
int trial(uint32_t n, uint32_t depth, const TrialFrontier& tf, uint32_t waves_per_cu,
          uint32_t refill, uint32_t claim, hipStream_t s, double* ms, uint64_t* total_out) {
    const DeviceFrontier& fr = tf.fr;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    const uint32_t frames = std::max<uint32_t>(1, frames_needed(n, depth));
    LaunchCfg cfg;
    rc = plan_launch(dev, NQ_MODE_PERSISTENT, 0, waves_per_cu, frames, fr.len, false,
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

int autotune(uint32_t n, uint32_t depth_lo, uint32_t depth_hi, double budget_ms, nq_tuned* out) {
    if (n < 4 || n > NQ_MAX_N || !out) return NQ_EINVAL;
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
    int trials = 0;
    auto consider = [&](uint32_t depth, const TrialFrontier& fr, uint32_t wpc, uint32_t rf,
                        uint32_t claim, bool* better) -> int {
        double ms = 0;
        uint64_t total = 0;
        int rc = trial(n, depth, fr, wpc, rf, claim, s, &ms, &total);
        if (rc != NQ_OK) return rc;
        ++trials;
        spent += ms;
        if (have_expect && total != expect) return NQ_EDEVICE;   // counts must agree
        expect = total;
        have_expect = true;
        *better = ms < best.ms;
        if (*better) {
            best.depth = depth; best.waves_per_cu = wpc; best.refill_every = rf;
            best.claim = claim; best.ms = ms;
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
            bool b = false;
            for (int rep = 0; rep < 2 && spent < budget_ms; ++rep)
                if ((rc = consider(d, fr, 0, 512, 0, &b)) != NQ_OK) return rc;
        }
        // 2. waves per CU, the visit interval and the claim block at the best
        //    depth (claim 0 = the size-derived default).
        TrialFrontier fr;
        int rc = fr.load(n, best.depth, s);
        if (rc != NQ_OK) return rc;
        const uint32_t d = best.depth;
        for (uint32_t wpc : {8u, 16u, 24u}) {
            if (spent >= budget_ms) break;
            bool b = false;
            if ((rc = consider(d, fr, wpc, best.refill_every, best.claim, &b)) != NQ_OK) return rc;
        }
        for (uint32_t rf : {128u, 2048u}) {
            if (spent >= budget_ms) break;
            bool b = false;
            if ((rc = consider(d, fr, best.waves_per_cu, rf, best.claim, &b)) != NQ_OK) return rc;
        }
        for (uint32_t cl : {32u, 1024u}) {
            if (spent >= budget_ms) break;
            bool b = false;
            if ((rc = consider(d, fr, best.waves_per_cu, best.refill_every, cl, &b)) != NQ_OK)
                return rc;
        }
    } catch (const std::bad_alloc&) {
        return NQ_ENOMEM;
    }
    best.trials = (uint32_t)trials;
    best.count = expect;
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
        return nqi::autotune(n, depth_lo, depth_hi, budget_ms, out);
    } catch (...) {
        return NQ_ENOMEM;
    }
}
