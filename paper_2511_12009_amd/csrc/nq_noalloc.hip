// nq_count_subproblems_noalloc: the subproblem count for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid allocation).  The only scratch the DFS kernels need
// beyond the caller's buffers is the persistent scheduler's 64-bit work head;
// here it lives in a file-scope device array instead of a per-call
// allocation.  Every call on one device shares that device's array, so calls
// that overlap on one device race on the head.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "nq_internal.h"

namespace nqi {

namespace {

// Bytes of the static scratch: the work head in its first 8 bytes, the rest
// unused.
constexpr size_t kScratchBytes = 256;

static __device__ __align__(256) unsigned long long scratch[kScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_on_current_device(unsigned long long** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    if (dev < 0 || dev >= kMaxDevices) return NQ_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) { set_hip_error(e); return NQ_EDEVICE; }
        g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[dev];
    return NQ_OK;
}

}  // namespace

}  // namespace nqi

using namespace nqi;

extern "C" int nq_count_subproblems_noalloc(uint32_t n, const uint32_t* d_cols,
                                            const uint32_t* d_ld, const uint32_t* d_rd,
                                            const uint8_t* d_weight, uint64_t len,
                                            uint64_t* d_counts, uint64_t* d_total,
                                            const nq_opts* opts) {
    if (n < 1 || n > NQ_MAX_N_WIDE) return NQ_EINVAL;
    if (opts && (opts->flags & ~NQ_FLAGS_COUNT) != 0) return NQ_EINVAL;
    // timing would create events; the caller times the stream itself
    if (opts && opts->kernel_ms_out) return NQ_EINVAL;
    const uint32_t min_placed = opts ? std::min(opts->depth, n) : 0u;
    const bool wide = opts && (opts->flags & NQ_FLAG_WIDE_TOTAL);
    if (n > NQ_MAX_N && ((d_total && !wide) || min_placed + 20u < n)) return NQ_EINVAL;
    if (len == 0) return NQ_OK;
    if (!d_cols || !d_ld || !d_rd) return NQ_EINVAL;
    try {
        unsigned long long* head = nullptr;
        int rc = scratch_on_current_device(&head);
        if (rc != NQ_OK) return rc;
        DeviceInfo dev;
        if ((rc = device_info(&dev)) != NQ_OK) return rc;
        const uint32_t mode =
            (opts && opts->mode != NQ_MODE_AUTO) ? opts->mode : (uint32_t)NQ_MODE_PERSISTENT;
        const uint32_t frames = std::max<uint32_t>(1, frames_needed(n, min_placed));
        const bool kings = opts && (opts->flags & NQ_FLAG_KINGS);
        uint64_t* d_nodes = opts ? opts->d_nodes : nullptr;
        LaunchCfg cfg;
        rc = plan_launch(dev, mode, opts ? opts->wg_size : 0, opts ? opts->waves_per_cu : 0,
                         frames, len, d_nodes != nullptr, leafctr_ok(n, min_placed), &cfg, false,
                         kings, n);
        if (rc != NQ_OK) return rc;
        DfsParams P{};
        P.cols = d_cols; P.ld = d_ld; P.rd = d_rd; P.weight = d_weight;
        P.counts = d_counts;
        P.totals = reinterpret_cast<unsigned long long*>(d_total);
        P.nodes = d_nodes;
        P.head = head;                       // zeroed by a kernel in launch_dfs
        P.len = len; P.n = n; P.frames = frames;
        P.refill_every = (opts && opts->refill_every) ? opts->refill_every : 512u;
        P.idle_min = default_idle_min();
        P.claim = (opts && opts->claim) ? opts->claim : default_claim(len, cfg);
        P.reverse = (opts && (opts->flags & NQ_FLAG_FORWARD_ORDER)) ? 0u : 1u;
        P.wide = wide ? 1u : 0u;
        return launch_dfs(cfg, P, opts ? opts->stream : nullptr);
    } catch (...) {
        return NQ_EINVAL;
    }
}
