// Ragged batches: many independent counts in one persistent DFS launch,
// captured once as a HIP graph and replayed.
//
// The frontiers of all instances (Section 1 pre-placement, each at its own
// depth) are concatenated; every entry carries its instance id, and the kernel
// reads the board size of that instance, so lanes of one wave may work on
// different boards.  The graph holds: zero the per-instance totals, zero the
// work head, the persistent DFS kernel, and the copy of the totals into pinned
// host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "nq_internal.h"
#include "nq_trace.h"

struct nq_batch {
    uint32_t ninst = 0;
    uint64_t entries = 0;
    void* dev = nullptr;                 // one device allocation for every array
    unsigned long long* d_totals = nullptr;
    unsigned long long* h_totals = nullptr;   // pinned
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    nqi::LaunchCfg cfg{};
    nqi::DfsParams P{};
};

namespace nqi {

namespace {

void release(nq_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->dev) (void)hipFree(b->dev);
    if (b->h_totals) (void)hipHostFree(b->h_totals);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Default depth of one instance: 5, or n - 11 for large boards, so that no
// instance needs more than 9 stack frames (10 KB of LDS per wave: 16 resident
// waves per CU) and the largest instances are cut into tens of millions of
// subtrees (their frontiers are built by device expansion).
uint32_t batch_default_depth(uint32_t n, uint32_t requested) {
    uint32_t k = requested ? requested : std::max<uint32_t>(5u, n > 11 ? n - 11 : 0u);
    const uint32_t cap = n > 2 ? n - 2 : 1u;
    return std::max<uint32_t>(1u, std::min(k, cap));
}

int batch_create(uint32_t ninst, const uint32_t* ns, const uint32_t* depths, const nq_opts* opts,
                 nq_batch** out) {
    if (!out || ninst == 0 || !ns) return NQ_EINVAL;
    if (opts && (opts->flags & ~NQ_FLAGS_COUNT) != 0) return NQ_EINVAL;
    // queens only; per-instance totals are 64-bit (every board <= 28)
    if (opts && (opts->flags & (NQ_FLAG_KINGS | NQ_FLAG_WIDE_TOTAL))) return NQ_EINVAL;
    for (uint32_t i = 0; i < ninst; ++i) {
        if (ns[i] < 1 || ns[i] > NQ_MAX_N) return NQ_EINVAL;
        if (depths && (depths[i] < 1 || depths[i] > ns[i])) return NQ_EINVAL;
    }
    nq_batch* b = new (std::nothrow) nq_batch();
    if (!b) return NQ_ENOMEM;
    b->ninst = ninst;
    int rc = NQ_OK;
    hipError_t e;
    auto fail = [&](int code) {
        release(b);
        return code;
    };
    TraceRange trace("batch_create");
    try {
        if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
            set_hip_error(e);
            return fail(NQ_EDEVICE);
        }
        // Every instance's frontier on the device (deep ones by device
        // expansion), then one concatenated copy with instance ids.
        std::vector<uint32_t> k(ninst);
        std::vector<uint64_t> off(ninst + 1, 0);
        std::vector<DeviceFrontier> fr(ninst);
        uint32_t frames = 1, max_n = 1;
        bool leafctr = true;
        for (uint32_t i = 0; i < ninst; ++i) {
            k[i] = depths ? depths[i] : batch_default_depth(ns[i], opts ? opts->depth : 0);
            if ((rc = build_device_frontier(ns[i], k[i], b->stream, &fr[i])) != NQ_OK)
                return fail(rc);
            off[i + 1] = off[i] + fr[i].len;
            frames = std::max(frames, frames_needed(ns[i], k[i]));
            leafctr = leafctr && leafctr_ok(ns[i], k[i]);
            max_n = std::max(max_n, ns[i]);
        }
        const uint64_t total = off[ninst];
        b->entries = total;
        // Device layout: cols | ld | rd | inst | weight | inst_n | totals | head.
        const size_t o_ld = total * 4, o_rd = 2 * total * 4, o_inst = 3 * total * 4;
        const size_t o_w = 4 * total * 4, o_n = align_up(o_w + total, 16);
        const size_t o_tot = align_up(o_n + ninst * 4ull, 16), o_head = o_tot + ninst * 8ull;
        const size_t bytes = o_head + 64;
        if ((e = hipMalloc(&b->dev, bytes)) != hipSuccess) {
            set_hip_error(e);
            return fail(e == hipErrorOutOfMemory ? NQ_ENOMEM : NQ_EDEVICE);
        }
        if ((e = hipHostMalloc((void**)&b->h_totals, std::max<size_t>(8, ninst * 8ull))) !=
            hipSuccess) {
            set_hip_error(e);
            return fail(NQ_ENOMEM);
        }
        std::memset(b->h_totals, 0, std::max<size_t>(8, ninst * 8ull));
        char* d = static_cast<char*>(b->dev);
        const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
        for (uint32_t i = 0; i < ninst; ++i) {
            const uint64_t o = off[i], m = fr[i].len;
            if (m == 0) continue;
            if ((e = hipMemcpyAsync(d + o * 4, fr[i].cols, m * 4, d2d, b->stream)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(d + o_ld + o * 4, fr[i].ld, m * 4, d2d, b->stream)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(d + o_rd + o * 4, fr[i].rd, m * 4, d2d, b->stream)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(d + o_w + o, fr[i].w, m, d2d, b->stream)) != hipSuccess) {
                set_hip_error(e);
                return fail(NQ_EDEVICE);
            }
            rc = launch_fill_u32(reinterpret_cast<uint32_t*>(d + o_inst) + o, i, m, b->stream);
            if (rc != NQ_OK) return fail(rc);
        }
        {
            std::vector<uint32_t> hn(ns, ns + ninst);
            if ((e = hipMemcpyAsync(d + o_n, hn.data(), ninst * 4ull, hipMemcpyHostToDevice,
                                    b->stream)) != hipSuccess ||
                (e = hipStreamSynchronize(b->stream)) != hipSuccess) {
                set_hip_error(e);
                return fail(NQ_EDEVICE);
            }
        }
        fr.clear();                                   // per-instance copies no longer needed
        b->d_totals = reinterpret_cast<unsigned long long*>(d + o_tot);
        DfsParams& P = b->P;
        P.cols = reinterpret_cast<uint32_t*>(d);
        P.ld = reinterpret_cast<uint32_t*>(d + o_ld);
        P.rd = reinterpret_cast<uint32_t*>(d + o_rd);
        P.inst = reinterpret_cast<uint32_t*>(d + o_inst);
        P.weight = reinterpret_cast<uint8_t*>(d + o_w);
        P.inst_n = reinterpret_cast<uint32_t*>(d + o_n);
        P.ninst = ninst;
        P.totals = b->d_totals;
        P.head = reinterpret_cast<unsigned long long*>(d + o_head);
        P.counts = nullptr;
        P.nodes = nullptr;
        P.len = total;
        P.n = 0;
        P.frames = frames;
        P.refill_every = (opts && opts->refill_every) ? opts->refill_every : 512u;
        P.idle_min = default_idle_min();
        P.reverse = (opts && (opts->flags & NQ_FLAG_FORWARD_ORDER)) ? 0u : 1u;
        DeviceInfo dev;
        if ((rc = device_info(&dev)) != NQ_OK) return fail(rc);
        if ((rc = plan_launch(dev, NQ_MODE_PERSISTENT, opts ? opts->wg_size : 0,
                              opts ? opts->waves_per_cu : 0, frames, total, false, leafctr,
                              &b->cfg, false, false, max_n)) != NQ_OK)
            return fail(rc);
        P.claim = (opts && opts->claim) ? opts->claim : default_claim(total, b->cfg);
        // Capture: zero totals, zero head + DFS, totals to pinned host memory.
        if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) !=
            hipSuccess) {
            set_hip_error(e);
            return fail(NQ_EDEVICE);
        }
        rc = launch_zero_u64(b->d_totals, ninst, b->stream);
        if (rc == NQ_OK) rc = launch_dfs(b->cfg, P, b->stream);
        if (rc == NQ_OK && ninst) {
            e = hipMemcpyAsync(b->h_totals, b->d_totals, ninst * 8ull, hipMemcpyDeviceToHost,
                               b->stream);
            if (e != hipSuccess) { set_hip_error(e); rc = NQ_EDEVICE; }
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->stream, &g);
        b->graph = g;
        if (rc != NQ_OK) return fail(rc);
        if (e != hipSuccess) { set_hip_error(e); return fail(NQ_EDEVICE); }
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
            set_hip_error(e);
            return fail(NQ_EDEVICE);
        }
    } catch (const std::bad_alloc&) {
        return fail(NQ_ENOMEM);
    }
    *out = b;
    return NQ_OK;
}

int batch_run(nq_batch* b, uint64_t* out_totals, double* ms) {
    TraceRange t("batch_run");
    if (!b || (b->ninst && !out_totals)) return NQ_EINVAL;
    hipError_t e;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (ms) {
        if ((e = hipEventCreate(&ea)) != hipSuccess || (e = hipEventCreate(&eb)) != hipSuccess ||
            (e = hipEventRecord(ea, b->stream)) != hipSuccess) {
            set_hip_error(e);
            if (ea) (void)hipEventDestroy(ea);
            if (eb) (void)hipEventDestroy(eb);
            return NQ_EDEVICE;
        }
    }
    e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess && ms) e = hipEventRecord(eb, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && ms) {
        float f = 0.f;
        e = hipEventElapsedTime(&f, ea, eb);
        *ms = f;
    }
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    for (uint32_t i = 0; i < b->ninst; ++i) out_totals[i] = b->h_totals[i];
    return NQ_OK;
}

}  // namespace nqi

extern "C" int nq_batch_create(uint32_t ninst, const uint32_t* ns, const uint32_t* depths,
                               const nq_opts* opts, nq_batch** out) {
    try {
        return nqi::batch_create(ninst, ns, depths, opts, out);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_batch_run(nq_batch* b, uint64_t* out_totals, double* kernel_ms) {
    try {
        return nqi::batch_run(b, out_totals, kernel_ms);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" uint64_t nq_batch_entries(const nq_batch* b) { return b ? b->entries : 0; }

extern "C" int nq_batch_destroy(nq_batch* b) {
    if (!b) return NQ_EINVAL;
    nqi::release(b);
    return NQ_OK;
}

extern "C" int nq_count_batch(uint32_t ninst, const uint32_t* ns, const uint32_t* depths,
                              const nq_opts* opts, uint64_t* out_totals) {
    if (ninst == 0) return NQ_OK;
    if (!ns || !out_totals) return NQ_EINVAL;
    nq_batch* b = nullptr;
    int rc = NQ_OK;
    try {
        rc = nqi::batch_create(ninst, ns, depths, opts, &b);
        if (rc != NQ_OK) return rc;
        double ms = 0.0;
        rc = nqi::batch_run(b, out_totals, opts && opts->kernel_ms_out ? &ms : nullptr);
        if (rc == NQ_OK && opts && opts->kernel_ms_out) *opts->kernel_ms_out = ms;
    } catch (...) {
        rc = NQ_ENOMEM;
    }
    if (b) nqi::release(b);
    return rc;
}
