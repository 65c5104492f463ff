// C-ABI entry points: status text, nq_count, nq_count_subproblems, nq_count_batch,
// nq_count_resumable.
#include <hip/hip_runtime.h>
#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nq_internal.h"
#include "nq_trace.h"

namespace nqi {

static thread_local int g_last_hip_error = 0;

// Boards beyond 28 (128-bit totals): at most this many rows below a prefix,
// so that a per-subproblem count (at most 20! < 2^62 placements) and its
// weighted value stay within 64 bits.
constexpr uint32_t kMaxRowsBelowWide = 20;

// Largest kings board whose total fits in 64 bits.
constexpr uint32_t kMaxKingsN = 21;

void set_hip_error(int err) { g_last_hip_error = err; }

// Boards whose automatic count runs in chunks, with the depth and chunk count
// measured best (nq_autotune re-measures the depth for the device at hand):
// N = 21 at depth 10 in 16 chunks (8.86 s against 9.0 s for the whole depth-9
// frontier), N = 22 at depth 11 in 64 chunks (79.9 s against 86.4 s), N = 23
// at depth 11 in 64 chunks (753 s; depth 11 beat 9 and 10 on the same chunk).
namespace {
constexpr ChunkPlan kChunkPlans[] = {{21, 10, 16}, {22, 11, 64}, {23, 11, 64}};
}  // namespace

const ChunkPlan* chunk_plan(uint32_t n) {
    for (const ChunkPlan& p : kChunkPlans)
        if (p.n == n) return &p;
    return nullptr;
}

namespace {

#define NQ_HIP(call)                                       \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) {                            \
            set_hip_error((int)e_);                        \
            return NQ_EDEVICE;                             \
        }                                                  \
    } while (0)

// Device buffer released on scope exit.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes) {
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            set_hip_error((int)e);
            p = nullptr;
            cap = 0;
            return e == hipErrorOutOfMemory ? NQ_ENOMEM : NQ_EDEVICE;
        }
        cap = bytes;
        return NQ_OK;
    }
    // Keeps the buffer when it holds `bytes`, else replaces it (contents lost).
    int ensure(size_t bytes) {
        if (p && cap >= bytes) return NQ_OK;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            cap = 0;
            if (e != hipSuccess) { set_hip_error((int)e); return NQ_EDEVICE; }
        }
        return alloc(bytes);
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Event pair timing the DFS launch on a stream.
struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    int start(hipStream_t s) {
        NQ_HIP(hipEventCreate(&a));
        NQ_HIP(hipEventCreate(&b));
        NQ_HIP(hipEventRecord(a, s));
        return NQ_OK;
    }
    int stop(hipStream_t s, double* ms) {
        NQ_HIP(hipEventRecord(b, s));
        NQ_HIP(hipEventSynchronize(b));
        float f = 0.f;
        NQ_HIP(hipEventElapsedTime(&f, a, b));
        *ms = (double)f;
        return NQ_OK;
    }
};

uint32_t opt_mode(const nq_opts* o) {
    uint32_t m = o ? o->mode : 0u;
    return m == NQ_MODE_AUTO ? (uint32_t)NQ_MODE_PERSISTENT : m;
}

// Default pre-placement depth: the shallowest depth whose frontier has at least
// 2^29 entries (a few thousand DFS nodes per entry at N = 20, small enough for
// the persistent scheduler to balance), capped so that every subtree keeps
// two rows of search and the frontier stays under 2^32 entries.  Sizes are
// exact up to depth 8 (host enumeration) and extrapolated by the last growth
// ratio beyond it, where nq_count builds the frontier by device expansion.
uint32_t auto_depth(uint32_t n) {
    const uint64_t target = 1ull << 29, limit = 1ull << 32;
    const uint32_t cap = n > 4 ? n - 4 : 1;
    uint64_t prev = 0, f = 0;
    uint32_t k = 1;
    for (; k <= std::min<uint32_t>(cap, 8); ++k) {
        prev = f;
        if (frontier_fill(n, k, nullptr, nullptr, nullptr, nullptr, 0, &f, nullptr) != NQ_OK)
            return 1;
        if (f >= target) return k;
    }
    --k;                                    // deepest enumerated depth
    if (k < cap && prev > 0 && f > prev) {
        const double ratio = (double)f / (double)prev;
        double est = (double)f;
        while (k < cap && est < (double)target && est * ratio < (double)limit) {
            est *= ratio;
            ++k;
        }
    }
    return std::max<uint32_t>(1, k);
}

// The kings search's automatic depth: the shallowest whose host frontier has
// at least 2^22 entries (kept on the host, so at most 2^27), at most n - 2.
uint32_t kings_auto_depth(uint32_t n) {
    if (n <= 3) return n;
    uint32_t best = 1;
    for (uint32_t d = 1; d + 2 <= n; ++d) {
        uint64_t F = 0;
        if (frontier_fill(n, d, nullptr, nullptr, nullptr, nullptr, 0, &F, nullptr, true) != NQ_OK ||
            F > (1ull << 27))
            break;
        best = d;
        if (F >= (1ull << 22)) break;
    }
    return best;
}

uint32_t refill_default(const nq_opts* o) {
    return (o && o->refill_every) ? o->refill_every : 512u;
}

}  // namespace

// Runs the DFS over device-resident entries of one board size.
static int run_device(uint32_t n, const uint32_t* d_cols, const uint32_t* d_ld,
                      const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len,
                      uint64_t* d_counts, unsigned long long* d_total, uint32_t min_placed,
                      const nq_opts* opts, double* kernel_ms) {
    if (len == 0) {
        if (kernel_ms) *kernel_ms = 0.0;
        return NQ_OK;
    }
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    const uint32_t mode = opt_mode(opts);
    const uint32_t frames = std::max<uint32_t>(1, frames_needed(n, min_placed));
    LaunchCfg cfg;
    uint64_t* d_nodes = opts ? opts->d_nodes : nullptr;
    const bool kings = opts && (opts->flags & NQ_FLAG_KINGS);
    rc = plan_launch(dev, mode, opts ? opts->wg_size : 0, opts ? opts->waves_per_cu : 0, frames,
                     len, d_nodes != nullptr, leafctr_ok(n, min_placed), &cfg, false, kings, n);
    if (rc != NQ_OK) return rc;
    hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
    unsigned long long* head = nullptr;
    if (mode == NQ_MODE_PERSISTENT) NQ_HIP(hipMallocAsync((void**)&head, 8, s));
    DfsParams P{};
    P.cols = d_cols; P.ld = d_ld; P.rd = d_rd; P.weight = d_weight;
    P.counts = d_counts; P.totals = d_total; P.nodes = d_nodes; P.head = head;
    P.len = len; P.n = n; P.frames = frames; P.refill_every = refill_default(opts);
    P.idle_min = default_idle_min();
    P.claim = (opts && opts->claim) ? opts->claim : default_claim(len, cfg);
    P.reverse = (opts && (opts->flags & NQ_FLAG_FORWARD_ORDER)) ? 0u : 1u;
    P.wide = (opts && (opts->flags & NQ_FLAG_WIDE_TOTAL)) ? 1u : 0u;
    EventTimer t;
    if (kernel_ms) rc = t.start(s);
    if (rc == NQ_OK) rc = launch_dfs(cfg, P, s);
    if (rc == NQ_OK && kernel_ms) rc = t.stop(s, kernel_ms);
    if (head) {                                   // freed on every path past its allocation
        hipError_t e = hipFreeAsync(head, s);
        if (e != hipSuccess && rc == NQ_OK) { set_hip_error((int)e); rc = NQ_EDEVICE; }
    }
    return rc;
}


namespace {

// Allocates the arrays of a frontier of `len` entries (cols | ld | rd | weight)
// with room for `cap` >= len (the arrays are laid out for cap entries).
int alloc_frontier(uint64_t len, DeviceFrontier* f, uint64_t cap = 0) {
    cap = std::max(cap, len);
    const size_t o_ld = cap * 4, o_rd = 2 * cap * 4, o_w = 3 * cap * 4;
    DevBuf arr;
    int rc = arr.alloc(o_w + cap + 16);
    if (rc != NQ_OK) return rc;
    char* b = arr.as<char>();
    *f = DeviceFrontier();                        // frees what it held
    f->dev = arr.p;
    arr.p = nullptr;
    f->len = len;
    f->cap = cap;
    f->cols = reinterpret_cast<uint32_t*>(b);
    f->ld = reinterpret_cast<uint32_t*>(b + o_ld);
    f->rd = reinterpret_cast<uint32_t*>(b + o_rd);
    f->w = reinterpret_cast<uint8_t*>(b + o_w);
    return NQ_OK;
}

// A frontier of `len` entries in `f`, keeping f's arrays when they have room
// (contents lost); a new allocation gets 1/8 more room, so that the next
// chunks of a chunked count, a little larger or smaller, reuse it.
int reuse_frontier(uint64_t len, DeviceFrontier* f) {
    if (f->dev && f->cap >= len) {
        f->len = len;
        f->first_row.clear();
        return NQ_OK;
    }
    *f = DeviceFrontier();                        // free before the larger allocation
    return alloc_frontier(len, f, len + len / 8);
}

// The host frontier of depth `depth` (nq_frontier) uploaded to the device.
int host_frontier(uint32_t n, uint32_t depth, hipStream_t s, DeviceFrontier* out,
                  bool kings = false) {
    uint64_t F = 0;
    std::vector<uint64_t> first_row;
    int rc = frontier_fill(n, depth, nullptr, nullptr, nullptr, nullptr, 0, &F, nullptr, kings);
    if (rc != NQ_OK) return rc;
    std::vector<uint32_t> hc(F), hl(F), hr(F);
    std::vector<uint8_t> hw(F);
    rc = frontier_fill(n, depth, hc.data(), hl.data(), hr.data(), hw.data(), F, &F, &first_row,
                       kings);
    if (rc != NQ_OK) return rc;
    if ((rc = alloc_frontier(F, out)) != NQ_OK) return rc;
    if (F) {
        NQ_HIP(hipMemcpyAsync(out->cols, hc.data(), F * 4, hipMemcpyHostToDevice, s));
        NQ_HIP(hipMemcpyAsync(out->ld, hl.data(), F * 4, hipMemcpyHostToDevice, s));
        NQ_HIP(hipMemcpyAsync(out->rd, hr.data(), F * 4, hipMemcpyHostToDevice, s));
        NQ_HIP(hipMemcpyAsync(out->w, hw.data(), F, hipMemcpyHostToDevice, s));
    }
    NQ_HIP(hipStreamSynchronize(s));              // the host vectors die here
    out->first_row = std::move(first_row);
    return NQ_OK;
}

// `in` expanded by `rows` (1..3) on the device into `out`; the row-0 runs are
// carried over, and `offsets` (nullable) receives the index of the first child
// of every entry of `in` (offsets[in.len] = out->len).
// The frontier `rows` rows below `in`, in `out`.  With `keep` (chunked
// counts) out's arrays and the scan scratch *keep are reused when they have
// room, so that a count of many chunks does not allocate and free its
// largest buffers once per chunk (on this runtime such frees and
// allocations of several GB slow down after a few dozen, to 0.2-2 s each).
int expand_frontier(uint32_t n, const DeviceFrontier& in, uint32_t rows, hipStream_t s,
                    DeviceFrontier* out, std::vector<uint64_t>* offsets,
                    DevBuf* keep = nullptr) {
    TraceRange t("expand");
    if (in.len == 0) {                            // nothing to expand
        if (offsets) offsets->assign(1, 0);
        int rc0 = keep ? reuse_frontier(0, out) : alloc_frontier(0, out);
        out->first_row.assign(in.first_row.size(), 0);
        return rc0;
    }
    DevBuf local;
    DevBuf& scratch = keep ? *keep : local;
    int rc = keep ? scratch.ensure(expand_scratch_bytes(in.len))
                  : scratch.alloc(expand_scratch_bytes(in.len));
    if (rc != NQ_OK) return rc;
    uint64_t F = 0;
    rc = expand_device(n, rows, in.cols, in.ld, in.rd, in.w, in.len, nullptr, nullptr, nullptr,
                       nullptr, 0, &F, scratch.p, s);
    if (rc != NQ_OK) return rc;
    std::vector<uint64_t> first_row = in.first_row;
    const uint64_t* offs = scratch.as<uint64_t>() + (in.len + 1);
    if (offsets) {
        offsets->resize(in.len + 1);
        NQ_HIP(hipMemcpy(offsets->data(), offs, (in.len + 1) * 8, hipMemcpyDeviceToHost));
        for (auto& o : first_row) o = (*offsets)[o];
    } else {
        for (auto& o : first_row) {
            uint64_t v = 0;
            NQ_HIP(hipMemcpy(&v, offs + o, 8, hipMemcpyDeviceToHost));
            o = v;
        }
    }
    if ((rc = keep ? reuse_frontier(F, out) : alloc_frontier(F, out)) != NQ_OK) return rc;
    uint64_t got = 0;
    rc = expand_device(n, rows, in.cols, in.ld, in.rd, in.w, in.len, out->cols, out->ld, out->rd,
                       out->w, F, &got, scratch.p, s);
    if (rc != NQ_OK) return rc;
    NQ_HIP(hipStreamSynchronize(s));              // the scratch dies here
    out->first_row = std::move(first_row);
    return NQ_OK;
}

}  // namespace

DeviceFrontier::~DeviceFrontier() {
    if (dev) (void)hipFree(dev);
}

DeviceFrontier& DeviceFrontier::operator=(DeviceFrontier&& o) noexcept {
    if (this != &o) {
        if (dev) (void)hipFree(dev);
        dev = o.dev; len = o.len; cap = o.cap; cols = o.cols; ld = o.ld; rd = o.rd; w = o.w;
        first_row = std::move(o.first_row);
        o.dev = nullptr;
        o.len = 0;
        o.cap = 0;
    }
    return *this;
}

int build_device_frontier(uint32_t n, uint32_t depth, void* stream, DeviceFrontier* out) {
    if (!out || out->dev || depth > n) return NQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // Depth 5 on the host (3e5 entries at N = 20), the rest in device
    // expansions of up to three rows each.
    uint32_t have = depth >= 7 ? 5u : depth;
    DeviceFrontier cur;
    int rc = host_frontier(n, have, s, &cur);
    if (rc != NQ_OK) return rc;
    while (have < depth) {
        // equal steps (5 -> 7 -> 9, not 5 -> 8 -> 9): the last input stays small
        const uint32_t left = depth - have, steps = (left + 2) / 3;
        const uint32_t rows = (left + steps - 1) / steps;
        DeviceFrontier next;
        if ((rc = expand_frontier(n, cur, rows, s, &next, nullptr)) != NQ_OK) return rc;
        cur = std::move(next);
        have += rows;
    }
    *out = std::move(cur);
    return NQ_OK;
}

int build_device_frontier_at(uint32_t n, uint32_t host_depth, uint32_t rows, void* stream,
                             DeviceFrontier* out, std::vector<uint64_t>* offsets) {
    if (!out || out->dev || rows > 3 || host_depth + rows > n) return NQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    DeviceFrontier cur;
    int rc = host_frontier(n, host_depth, s, &cur);
    if (rc != NQ_OK) return rc;
    if (rows == 0) {
        if (offsets) offsets->clear();
        *out = std::move(cur);
        return NQ_OK;
    }
    DeviceFrontier next;
    if ((rc = expand_frontier(n, cur, rows, s, &next, offsets)) != NQ_OK) return rc;
    *out = std::move(next);
    return NQ_OK;
}

// Counts chunks first.. of the (n, depth) count: chunk i is the range
// [F*i/chunks, F*(i+1)/chunks) of the host frontier of host_depth, deepened
// on the device in equal steps of up to three rows and searched by one
// launch into a 128-bit device total.  At most max_run chunks (0 = all the
// rest); after each one on_chunk(chunks done, its weighted count as an
// unsigned __int128) is called, and a status other than NQ_OK from it stops
// the loop.  kernel_ms (nullable) accumulates the DFS kernel time.
template <class OnChunk>
int count_chunks(uint32_t n, const nq_opts& local, uint32_t depth, uint32_t host_depth,
                 uint32_t chunks, uint32_t first, uint32_t max_run, double* kernel_ms,
                 OnChunk&& on_chunk) {
    uint64_t Fh = 0;
    std::vector<uint32_t> hc, hl, hr;
    std::vector<uint8_t> hw;
    {
        TraceRange t("frontier");
        int rc = frontier_fill(n, host_depth, nullptr, nullptr, nullptr, nullptr, 0, &Fh, nullptr);
        if (rc != NQ_OK) return rc;
        hc.resize(Fh); hl.resize(Fh); hr.resize(Fh); hw.resize(Fh);
        if ((rc = frontier_fill(n, host_depth, hc.data(), hl.data(), hr.data(), hw.data(), Fh,
                                &Fh, nullptr)) != NQ_OK)
            return rc;
    }
    int rc = NQ_OK;
    hipStream_t s = (hipStream_t)local.stream;
    DevBuf tot;
    if ((rc = tot.alloc(16)) != NQ_OK) return rc;
    auto* d_total = tot.as<unsigned long long>();   // low word, high word
    nq_opts wide = local;
    wide.flags |= NQ_FLAG_WIDE_TOTAL;
    // Device buffers kept across chunks and grown when a chunk needs more:
    // the uploaded host range, two frontiers that the expansions alternate
    // between, and the expansion's scan scratch.
    DeviceFrontier up, pingpong[2];
    DevBuf scan;
    uint32_t ran = 0;
    for (uint32_t i = first; i < chunks && (max_run == 0 || ran < max_run); ++i, ++ran) {
        const uint64_t lo = Fh * i / chunks, hi = Fh * (i + 1) / chunks;
        unsigned __int128 part = 0;
        TraceRange chunk_range("chunk");
        if (hi > lo) {
            if ((rc = reuse_frontier(hi - lo, &up)) != NQ_OK) return rc;
            NQ_HIP(hipMemcpyAsync(up.cols, hc.data() + lo, (hi - lo) * 4, hipMemcpyHostToDevice, s));
            NQ_HIP(hipMemcpyAsync(up.ld, hl.data() + lo, (hi - lo) * 4, hipMemcpyHostToDevice, s));
            NQ_HIP(hipMemcpyAsync(up.rd, hr.data() + lo, (hi - lo) * 4, hipMemcpyHostToDevice, s));
            NQ_HIP(hipMemcpyAsync(up.w, hw.data() + lo, hi - lo, hipMemcpyHostToDevice, s));
            const DeviceFrontier* cur = &up;
            int which = 0;
            for (uint32_t have = host_depth; have < depth;) {
                const uint32_t left = depth - have, steps = (left + 2) / 3;
                const uint32_t rows = (left + steps - 1) / steps;
                DeviceFrontier* next = &pingpong[which];
                which ^= 1;
                if ((rc = expand_frontier(n, *cur, rows, s, next, nullptr, &scan)) != NQ_OK)
                    return rc;
                cur = next;
                have += rows;
            }
            double ms = 0.0;
            if ((rc = launch_zero_u64(d_total, 2, s)) != NQ_OK) return rc;
            if ((rc = run_device(n, cur->cols, cur->ld, cur->rd, cur->w, cur->len, nullptr, d_total,
                                 depth, &wide, kernel_ms ? &ms : nullptr)) != NQ_OK)
                return rc;
            uint64_t words[2] = {0, 0};
            NQ_HIP(hipMemcpyAsync(words, d_total, 16, hipMemcpyDeviceToHost, s));
            NQ_HIP(hipStreamSynchronize(s));
            part = ((unsigned __int128)words[1] << 64) | words[0];
            if (kernel_ms) *kernel_ms += ms;
        }
        if ((rc = on_chunk(i + 1, part)) != NQ_OK) return rc;
    }
    return NQ_OK;
}

int time_chunk(uint32_t n, uint32_t depth, uint32_t chunks, uint32_t index, const nq_opts& opts,
               double* ms, unsigned __int128* total) {
    if (n > NQ_MAX_N || chunks == 0 || index >= chunks || depth < kChunkHostDepth || depth > n)
        return NQ_EINVAL;
    nq_opts local = opts;
    local.depth = depth;
    local.counts_out = nullptr;
    local.d_nodes = nullptr;
    local.kernel_ms_out = nullptr;
    unsigned __int128 got = 0;
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = count_chunks(n, local, depth, kChunkHostDepth, chunks, index, 1, nullptr,
                                [&](uint32_t, unsigned __int128 part) {
                                    got = part;
                                    return (int)NQ_OK;
                                });
    const auto t1 = std::chrono::steady_clock::now();
    if (rc != NQ_OK) return rc;
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    *total = got;
    return NQ_OK;
}

}  // namespace nqi

using namespace nqi;

extern "C" const char* nq_strerror(int status) {
    switch (status) {
        case NQ_OK: return "ok";
        case NQ_EINVAL: return "invalid argument";
        case NQ_ERANGE: return "output buffer too small";
        case NQ_ENOMEM: return "out of memory";
        case NQ_EDEVICE: return "HIP runtime error";
        case NQ_EAGAIN: return "not finished yet";
        case NQ_EFULL: return "admission refused: no capacity";
        case NQ_ENOENT: return "unknown ticket";
        default: return "unknown status";
    }
}

extern "C" int nq_last_hip_error(void) { return g_last_hip_error; }

extern "C" int nq_set_loop_form(int form, int* previous) { return set_loop_form(form, previous); }

extern "C" int nq_expand(uint32_t n, uint32_t rows, const uint32_t* d_cols, const uint32_t* d_ld,
                         const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len,
                         uint32_t* d_ocols, uint32_t* d_old, uint32_t* d_ord, uint8_t* d_oweight,
                         uint64_t capacity, uint64_t* out_len, void* stream) {
    if (n < 1 || n > NQ_MAX_N_WIDE || rows < 1 || rows > 3 || !out_len) return NQ_EINVAL;
    if (len && (!d_cols || !d_ld || !d_rd)) return NQ_EINVAL;
    try {
        DevBuf scratch;
        int rc = scratch.alloc(expand_scratch_bytes(len));
        if (rc != NQ_OK) return rc;
        rc = expand_device(n, rows, d_cols, d_ld, d_rd, d_weight, len, d_ocols, d_old, d_ord,
                           d_oweight, capacity, out_len, scratch.p, stream);
        if (rc == NQ_OK && d_ocols) {
            // the scratch is freed on return: wait for the write pass
            hipError_t e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
        }
        return rc;
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_count_subproblems(uint32_t n, const uint32_t* d_cols, const uint32_t* d_ld,
                                    const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len,
                                    uint64_t* d_counts, uint64_t* d_total, const nq_opts* opts) {
    if (n < 1 || n > NQ_MAX_N_WIDE) return NQ_EINVAL;
    if (opts && (opts->flags & ~NQ_FLAGS_COUNT) != 0) return NQ_EINVAL;
    const uint32_t min_placed = opts ? std::min(opts->depth, n) : 0u;
    if (n > NQ_MAX_N) {
        // beyond 64-bit totals: a 128-bit d_total, and at most 20 rows below
        // every prefix so that each per-subproblem count stays below 20! < 2^62
        const bool wide = opts && (opts->flags & NQ_FLAG_WIDE_TOTAL);
        if ((d_total && !wide) || min_placed + kMaxRowsBelowWide < n) return NQ_EINVAL;
    }
    if (len == 0) return NQ_OK;
    if (!d_cols || !d_ld || !d_rd) return NQ_EINVAL;
    try {
        return run_device(n, d_cols, d_ld, d_rd, d_weight, len, d_counts,
                          reinterpret_cast<unsigned long long*>(d_total), min_placed, opts,
                          opts ? opts->kernel_ms_out : nullptr);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_count(uint32_t n, const nq_opts* opts_in, uint64_t* out_total) {
    if (n < 1 || n > NQ_MAX_N || !out_total) return NQ_EINVAL;
    if (opts_in && (opts_in->flags & ~NQ_FLAGS_COUNT) != 0) return NQ_EINVAL;
    if (opts_in && (opts_in->flags & NQ_FLAG_WIDE_TOTAL)) return NQ_EINVAL;  // no device total
    // Automatic depth: the autotuner's choice for this n if it ran, else the
    // frontier-size rule.  A tuned launch shape fills fields left at 0.
    nq_opts local{};
    if (opts_in) local = *opts_in;
    local.d_nodes = nullptr;          // per-entry nodes are a nq_count_subproblems output
    const nq_opts* opts = &local;
    const bool kings = (local.flags & NQ_FLAG_KINGS) != 0;
    // the number of king placements passes 2^64 at n = 22 (about n! / e^2)
    if (kings && n > kMaxKingsN) return NQ_EINVAL;
    uint32_t tuned_chunks = 0;                        // the tuner chose a chunked count
    if (local.depth == 0 && !kings) {
        nq_tuned t;
        if (tune_lookup(n, &t) == NQ_OK) {
            local.depth = t.depth;
            tuned_chunks = t.chunks;
            if (!local.wg_size) local.wg_size = t.wg_size;
            if (!local.waves_per_cu) local.waves_per_cu = t.waves_per_cu;
            if (!local.refill_every) local.refill_every = t.refill_every;
            if (!local.claim) local.claim = t.claim;
        }
    }
    const bool auto_pick = local.depth == 0;          // neither the caller nor the tuner chose
    const uint32_t depth = local.depth ? local.depth : kings ? kings_auto_depth(n) : auto_depth(n);
    if (depth > n) return NQ_EINVAL;
    const ChunkPlan* plan = chunk_plan(n);
    if (!kings && ((auto_pick && plan) || tuned_chunks) && !local.counts_out &&
        opt_mode(opts) == NQ_MODE_PERSISTENT) {
        // A whole frontier deep enough for these boards does not fit in device
        // memory; chunks of the depth-5 frontier deepened to the plan's (or the
        // tuner's) depth do (as nq_count_resumable, without a progress file).
        const uint32_t depth_c = tuned_chunks ? depth : plan->depth;
        const uint32_t chunks_c = tuned_chunks ? tuned_chunks : plan->chunks;
        if (depth_c < kChunkHostDepth) return NQ_EINVAL;
        try {
            TraceRange whole("nq_count (chunked)");
            uint64_t total = 0;
            double ms = 0.0;
            local.depth = depth_c;
            int rc = count_chunks(n, local, depth_c, kChunkHostDepth, chunks_c, 0, 0,
                                  opts_in && opts_in->kernel_ms_out ? &ms : nullptr,
                                  [&](uint32_t, unsigned __int128 part) {
                                      total += (uint64_t)part;    // Q(n <= 23) < 2^64
                                      return (int)NQ_OK;
                                  });
            if (rc != NQ_OK) return rc;
            if (opts_in && opts_in->kernel_ms_out) *opts_in->kernel_ms_out = ms;
            *out_total = total;
            return NQ_OK;
        } catch (const std::bad_alloc&) {
            return NQ_ENOMEM;
        } catch (...) {
            return NQ_EINVAL;
        }
    }
    try {
        TraceRange whole("nq_count");
        hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
        DeviceFrontier fr;
        // the kings frontier is built on the host only (nq_expand follows the
        // queens' recurrence)
        int rc;
        {
            TraceRange t("frontier");
            rc = kings ? host_frontier(n, depth, s, &fr, true) : build_device_frontier(n, depth, s, &fr);
        }
        if (rc != NQ_OK) return rc;
        const uint64_t F = fr.len;
        const std::vector<uint64_t>& first_row = fr.first_row;
        if (opts && opts->counts_out && opts->counts_capacity < F) return NQ_ERANGE;
        // counts (only when asked for) | total
        const bool want_counts = opts && opts->counts_out;
        DevBuf buf;
        const size_t off_tot = want_counts ? F * 8 : 0;
        if ((rc = buf.alloc(off_tot + 8)) != NQ_OK) return rc;
        char* b = buf.as<char>();
        auto* d_total = reinterpret_cast<unsigned long long*>(b + off_tot);
        uint64_t* d_counts = want_counts ? reinterpret_cast<uint64_t*>(b) : nullptr;
        if ((rc = launch_zero_u64(d_total, 1, s)) != NQ_OK) return rc;
        const uint32_t mode = opt_mode(opts);
        double ms = 0.0, ms_part = 0.0;
        roctxRangePushA("dfs launch");     // enqueue only: the launches are asynchronous
        if (mode == NQ_MODE_PLAIN) {
            // One launch per row-0 column (the form the paper's host driver uses
            // per GPU slice), each over its contiguous run of the frontier.
            for (size_t j = 0; j + 1 < first_row.size(); ++j) {
                const uint64_t lo = first_row[j], hi = first_row[j + 1];
                rc = run_device(n, fr.cols + lo, fr.ld + lo, fr.rd + lo, fr.w + lo, hi - lo,
                                d_counts ? d_counts + lo : nullptr, d_total, depth, opts,
                                opts && opts->kernel_ms_out ? &ms_part : nullptr);
                if (rc != NQ_OK) break;
                ms += ms_part;
            }
        } else {
            rc = run_device(n, fr.cols, fr.ld, fr.rd, fr.w, F, d_counts, d_total, depth, opts,
                            opts && opts->kernel_ms_out ? &ms : nullptr);
        }
        roctxRangePop();
        if (rc != NQ_OK) return rc;
        uint64_t total = 0;
        TraceRange result_range("dfs wait and result");
        NQ_HIP(hipMemcpyAsync(&total, d_total, 8, hipMemcpyDeviceToHost, s));
        if (want_counts && F)
            NQ_HIP(hipMemcpyAsync(opts->counts_out, d_counts, F * 8, hipMemcpyDeviceToHost, s));
        NQ_HIP(hipStreamSynchronize(s));
        if (want_counts)
            for (uint64_t i = 0; i < F; ++i)
                if (opts->counts_out[i] == kCountInvalid) return NQ_EINVAL;
        if (opts_in && opts_in->kernel_ms_out) *opts_in->kernel_ms_out = ms;
        *out_total = total;
        return NQ_OK;
    } catch (const std::bad_alloc&) {
        return NQ_ENOMEM;
    } catch (...) {
        return NQ_EINVAL;
    }
}

// ---- nq_count_resumable: a long count in chunks, with its progress in a file.

namespace {

constexpr uint32_t kResumeHostDepth = kChunkHostDepth;   // chunks are ranges of this host frontier
constexpr uint32_t kResumeChunks = 64;

struct Progress {
    uint32_t n = 0, depth = 0, host_depth = 0, chunks = 0, done = 0;
    unsigned __int128 total = 0;
};

// Decimal text of a 128-bit count.
std::string u128_text(unsigned __int128 v) {
    char buf[48];
    int i = sizeof buf - 1;
    buf[i] = 0;
    do {
        buf[--i] = (char)('0' + (int)(v % 10));
        v /= 10;
    } while (v != 0);
    return std::string(buf + i);
}

// Parses 1..39 decimal digits into *v; false on anything else or overflow.
bool u128_parse(const char* s, size_t len, unsigned __int128* v) {
    if (len == 0 || len > 39) return false;
    const unsigned __int128 max = ~(unsigned __int128)0;
    unsigned __int128 x = 0;
    for (size_t i = 0; i < len; ++i) {
        if (s[i] < '0' || s[i] > '9') return false;
        const unsigned d = (unsigned)(s[i] - '0');
        if (x > (max - d) / 10) return false;
        x = x * 10 + d;
    }
    *v = x;
    return true;
}

// FNV-1a (64-bit) of the record text: catches a torn or edited file.
uint64_t fnv1a64(const std::string& s) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 0x100000001b3ull;
    }
    return h;
}

std::string progress_body(const Progress& p) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "nq-progress 1 n=%u depth=%u host_depth=%u chunks=%u done=%u total=",
                  p.n, p.depth, p.host_depth, p.chunks, p.done);
    return buf + u128_text(p.total);
}

// NQ_OK with *exists = false when there is no file; NQ_EINVAL when the file
// cannot be read or is not one intact record.
int progress_read(const char* path, Progress* p, bool* exists) {
    *exists = false;
    FILE* f = std::fopen(path, "r");
    if (!f) return access(path, F_OK) == 0 ? NQ_EINVAL : NQ_OK;
    char line[256] = {};
    const bool got = std::fgets(line, sizeof line, f) != nullptr;
    std::fclose(f);
    if (!got) return NQ_EINVAL;
    unsigned n, depth, hd, chunks, done;
    unsigned long long check;
    int t0 = -1, t1 = -1;
    // the total is up to 128 bits: its digits are located by %n and parsed apart
    if (std::sscanf(line,
                    "nq-progress 1 n=%u depth=%u host_depth=%u chunks=%u done=%u total=%n%*[0-9]%n "
                    "check=%llx",
                    &n, &depth, &hd, &chunks, &done, &t0, &t1, &check) != 6 ||
        t0 < 0 || t1 <= t0)
        return NQ_EINVAL;
    Progress q;
    q.n = n; q.depth = depth; q.host_depth = hd; q.chunks = chunks; q.done = done;
    if (!u128_parse(line + t0, (size_t)(t1 - t0), &q.total)) return NQ_EINVAL;
    if (fnv1a64(progress_body(q)) != check || q.done > q.chunks) return NQ_EINVAL;
    *p = q;
    *exists = true;
    return NQ_OK;
}

// Writes the record to path.tmp, flushes it to the disk and renames it over
// path, so the file always holds one complete record.
int progress_write(const char* path, const Progress& p) {
    const std::string body = progress_body(p);
    char tail[40];
    std::snprintf(tail, sizeof tail, " check=%016llx\n", (unsigned long long)fnv1a64(body));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return NQ_EINVAL;
    bool ok = std::fputs((body + tail).c_str(), f) >= 0 && std::fflush(f) == 0 &&
              fsync(fileno(f)) == 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return NQ_EINVAL;
    // make the rename itself durable: flush the directory that holds the file
    const std::string full(path);
    const size_t slash = full.find_last_of('/');
    const std::string dir =
        slash == std::string::npos ? "." : (slash == 0 ? "/" : full.substr(0, slash));
    const int dfd = open(dir.c_str(), O_RDONLY | O_DIRECTORY);
    if (dfd >= 0) {
        (void)fsync(dfd);
        close(dfd);
    }
    return NQ_OK;
}

}  // namespace

// Both resumable entry points: n up to max_n, the total in 128 bits.
static int count_resumable(uint32_t n, const nq_opts* opts_in, const char* path, uint32_t chunks,
                           uint32_t max_chunks, uint32_t max_n, unsigned __int128* out_total,
                           uint32_t* out_done) {
    if (n < 1 || n > max_n || !path || !*path || !out_total || !out_done) return NQ_EINVAL;
    if (opts_in && (opts_in->flags & ~NQ_FLAGS_COUNT) != 0) return NQ_EINVAL;
    if (opts_in && (opts_in->counts_out || opts_in->d_nodes)) return NQ_EINVAL;
    if (opts_in && (opts_in->flags & NQ_FLAG_KINGS)) return NQ_EINVAL;
    nq_opts local{};
    if (opts_in) local = *opts_in;
    local.kernel_ms_out = nullptr;
    try {
        Progress old;
        bool exists = false;
        int rc = progress_read(path, &old, &exists);
        if (rc != NQ_OK) return rc;
        const uint32_t nchunks = chunks ? chunks : kResumeChunks;
        // The automatic depth must be the same in every process that works on
        // one file, so it never comes from this process's tuning results: the
        // depth of a record of the same count, else the chunk plan of n, else
        // the frontier-size rule (for boards beyond 28 at least n - 20 rows).
        uint32_t depth = local.depth;
        if (depth == 0) {
            if (exists && old.n == n && old.chunks == nchunks) {
                depth = old.depth;
            } else if (n > NQ_MAX_N) {
                depth = n - kMaxRowsBelowWide;            // 9..11 for 29..31
            } else {
                const ChunkPlan* plan = chunk_plan(n);
                depth = plan ? plan->depth : auto_depth(n);
            }
        }
        if (depth > n) return NQ_EINVAL;
        if (n > NQ_MAX_N && depth + kMaxRowsBelowWide < n) return NQ_EINVAL;
        local.depth = depth;
        Progress pr;
        pr.n = n;
        pr.depth = depth;
        pr.host_depth = std::min(depth, kResumeHostDepth);
        pr.chunks = nchunks;
        if (exists) {
            if (old.n != pr.n || old.depth != pr.depth || old.host_depth != pr.host_depth ||
                old.chunks != pr.chunks)
                return NQ_EINVAL;                       // the file of another count
            pr = old;
        }
        if (pr.done < pr.chunks) {
            rc = count_chunks(n, local, depth, pr.host_depth, pr.chunks, pr.done, max_chunks,
                              nullptr, [&](uint32_t done, unsigned __int128 part) {
                                  pr.total += part;
                                  pr.done = done;
                                  return progress_write(path, pr);
                              });
            if (rc != NQ_OK) return rc;
        }
        *out_done = pr.done;
        *out_total = pr.total;
        return pr.done == pr.chunks ? NQ_OK : NQ_EAGAIN;
    } catch (const std::bad_alloc&) {
        return NQ_ENOMEM;
    } catch (...) {
        return NQ_EINVAL;
    }
}

extern "C" int nq_count_resumable(uint32_t n, const nq_opts* opts, const char* path,
                                  uint32_t chunks, uint32_t max_chunks, uint64_t* out_total,
                                  uint32_t* out_done) {
    if (!out_total) return NQ_EINVAL;
    unsigned __int128 total = 0;
    const int rc = count_resumable(n, opts, path, chunks, max_chunks, NQ_MAX_N, &total, out_done);
    if (rc != NQ_OK && rc != NQ_EAGAIN) return rc;
    if ((total >> 64) != 0) return NQ_ERANGE;           // a wide record: *out_done is written
    *out_total = (uint64_t)total;
    return rc;
}

extern "C" int nq_count_resumable_wide(uint32_t n, const nq_opts* opts, const char* path,
                                       uint32_t chunks, uint32_t max_chunks, uint64_t* out_total,
                                       uint32_t* out_done) {
    if (!out_total) return NQ_EINVAL;
    unsigned __int128 total = 0;
    const int rc =
        count_resumable(n, opts, path, chunks, max_chunks, NQ_MAX_N_WIDE, &total, out_done);
    if (rc != NQ_OK && rc != NQ_EAGAIN) return rc;
    out_total[0] = (uint64_t)total;
    out_total[1] = (uint64_t)(total >> 64);
    return rc;
}
