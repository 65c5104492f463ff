// Serving loop: continuous batching of count requests on one GPU.
//
// Requests (a full count Q(n), or the weighted sum over a contiguous slice of
// a frontier) arrive at any time.  Every request is served out of a frontier
// kept in device memory: built once per (n, depth) and, for slices of a
// shallow frontier, pre-expanded by up to three rows on the device, so that a
// slice of a few thousand subtrees becomes a few hundred thousand smaller ones
// (children are contiguous and in order, so a slice maps to one contiguous
// range of the expanded frontier) and spreads over the whole GPU.  A scheduler
// thread admits requests in arrival order while request slots, work-ring space
// and the stack frames of the epoch kernel allow, copies their subproblems
// device-to-device into a ring, and launches a bounded "epoch": one persistent
// DFS launch over exactly the entries admitted since the previous epoch.  Epochs rotate over four streams, so new epochs are queued while
// older ones still run and their waves fill the CUs as the older epochs
// drain.  Every retired subproblem decrements its request's remaining counter
// on the device; the lane that retires the last one publishes the request's
// total to pinned host memory (value, then a generation flag), where the
// scheduler sees it without waiting for the epoch to end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "nq_internal.h"
#include "nq_trace.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum class ReqState { Pending, Admitted, Done };

struct Req {
    nq_request rq{};
    ReqState state = ReqState::Pending;
    int status = NQ_OK;
    uint64_t count = 0;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    uint32_t slot = 0, gen = 0;
    uint64_t ring_start = 0, ring_len = 0;
    uint32_t depth = 0;          // pre-placement depth (COUNT: chosen at submit)
    uint64_t entries = 0;        // subproblems of this request
};

// A frontier kept on the device: the (n, depth) frontier expanded by `rows`;
// entry i of the (n, depth) frontier owns entries [off[i], off[i + 1]) of `fr`
// (off empty when rows == 0: entry i is entry i).
struct Resident {
    nqi::DeviceFrontier fr;
    uint32_t rows = 0;
    uint64_t len = 0;                    // entries of the (n, depth) frontier
    uint64_t bytes = 0;
    std::vector<uint64_t> off;
    uint64_t first(uint64_t i) const { return rows ? off[i] : i; }
};

struct Epoch {
    hipEvent_t done = nullptr;
    uint32_t stream = 0;                   // index of its stream in nq_server::streams
    std::vector<nqi::SlotInit> inits;      // host staging kept alive until `done`
};

constexpr uint32_t kHeads = 64;
constexpr uint32_t kStreams = 4;             // epochs in flight at once (divides kHeads)
constexpr uint32_t kHeadStride = kHeads / kStreams;   // work heads of two streams: 128 B apart
// The latency lane: the last stream takes only epochs of quick requests
// (COUNTs of boards up to kQuickMaxN, at most about 1.3 ms alone on the whole
// GPU), so that a quick request never waits for a free stream behind epochs
// of N = 17, 18 counts or slices, which take 5 to 20 ms each.  Quick epochs
// take another free stream only while no other request waits; the others
// never take the last one.
constexpr uint32_t kQuickStream = kStreams - 1;
constexpr uint32_t kQuickMaxN = 16;
constexpr size_t kRingEntryBytes = 4 * 4 + 1;   // cols, ld, rd, inst + weight
constexpr uint64_t kCountEntries = 1u << 18;    // COUNT: shallowest depth with this many
constexpr uint64_t kSliceSplit = 1u << 16;      // SLICE residents: expand when a slice of
                                                // the whole frontier would have fewer

}  // namespace

struct nq_server {
    // configuration
    uint32_t max_frames = 14;
    uint32_t max_slots = 4096;
    uint64_t ring_cap = 0;
    uint64_t budget = 0;
    uint64_t resident_bytes = 0;
    nq_opts launch{};
    uint32_t cu_count = 0;
    nqi::DeviceInfo devinfo{};
    // Launch shape of an epoch whose deepest subproblem needs f stack frames
    // (planned on first use): the LDS stack, and so the waves per CU, is sized
    // for the requests in the epoch, not for the server's limit.  Index 1 of
    // the first dimension: the epoch's boards are small enough for the row
    // marker of the default step (largest board + f <= 30); index 0: any
    // board (the kernel then tests the last row with a popcount).
    nqi::LaunchCfg cfg_by_frames[2][NQ_MAX_N + 1] = {};
    bool cfg_ready[2][NQ_MAX_N + 1] = {};

    // device memory
    void* dev = nullptr;
    uint32_t *r_cols = nullptr, *r_ld = nullptr, *r_rd = nullptr, *r_inst = nullptr;
    uint8_t* r_w = nullptr;
    uint32_t *s_n = nullptr, *s_rem = nullptr, *s_gen = nullptr;
    unsigned long long* s_tot = nullptr;
    unsigned long long* heads = nullptr;
    nqi::SlotInit* d_init = nullptr;       // max_slots records per epoch stream
    unsigned long long *h_val = nullptr, *h_flag = nullptr;   // pinned, host view
    unsigned long long *d_val = nullptr, *d_flag = nullptr;   // device view
    hipStream_t streams[kStreams] = {};
    hipStream_t aux = nullptr;              // resident frontier builds
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Resident> resident;   // (n, depth, kind)

    // Request state shared with the callers' threads (guarded by mu).
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Req> reqs;
    bool stop = false;
    int fatal = NQ_OK;
    int fatal_hip = 0;            // hipError_t behind `fatal`, handed to the caller's thread

    // Device-side bookkeeping, touched by the scheduler thread only (so the
    // HIP calls that enqueue an epoch run without mu held).
    struct Admit {                          // a request on the device, in ring order
        uint64_t ticket, ring_start, ring_len;
        uint32_t slot, gen;
        bool done;
    };
    std::deque<Admit> admitted;
    std::vector<uint32_t> free_slots;
    std::vector<uint32_t> slot_gen;
    uint64_t next_ticket = 1;
    uint64_t ring_head = 0, ring_tail = 0;  // logical positions, tail - head in use
    uint64_t epoch_no = 0;
    bool round_robin = false;               // epoch i on stream i mod kStreams, busy or not
    bool reserve = false;                   // NQ_FLAG_SERVE_RESERVE: one large epoch at a
                                            // time, a wave per CU left for quick ones
    std::deque<Epoch> epochs;
    std::thread worker;
};

namespace nqi {

namespace {

// Smallest depth whose frontier has at least kCountEntries entries, and at
// least n - 11 (at most 9 stack frames per lane: the LDS-bound DFS keeps 16
// waves per CU, and a large board's subtrees stay a few thousand nodes, so
// one request's tail is short), within the server's stack budget (frames) and
// at most n - 4 (n - 2 for small boards).
uint32_t count_depth(uint32_t n, uint32_t max_frames) {
    if (n <= 3) return n;                       // tiny boards: full pre-placement
    const uint32_t hi = n > 6 ? n - 4 : n - 2;
    uint32_t lo = (n >= max_frames + 2) ? std::max<uint32_t>(1, n - 2 - max_frames) : 1u;
    if (n > 11 + lo) lo = std::min(hi, n - 11);
    for (uint32_t k = lo; k <= hi; ++k) {
        uint64_t f = 0;
        if (frontier_fill(n, k, nullptr, nullptr, nullptr, nullptr, 0, &f, nullptr) != NQ_OK)
            break;
        if (f >= kCountEntries) return k;
    }
    return std::max(lo, hi);
}

// The resident frontier serving (n, depth) requests of one kind, built on
// first use (on the server's own stream, so running epochs are not waited
// for).  COUNT residents are the plain frontier (its depth already gives
// kCountEntries subtrees).  SLICE residents of a frontier of at least
// kSliceSplit entries, where a slice is a small part of a large search, are
// expanded by three rows (two or one when fewer rows would be left below), as
// far as the resident budget allows.
int ensure_resident(nq_server* s, uint32_t n, uint32_t depth, uint32_t kind, Resident** out) {
    auto key = std::make_tuple(n, depth, kind);
    auto it = s->resident.find(key);
    if (it != s->resident.end()) {
        *out = &it->second;
        return NQ_OK;
    }
    uint64_t F = 0;
    int rc = frontier_fill(n, depth, nullptr, nullptr, nullptr, nullptr, 0, &F, nullptr);
    if (rc != NQ_OK) return rc;
    uint32_t rows = 0;
    if (kind == NQ_REQ_SLICE && depth >= 2 && F >= kSliceSplit)
        rows = (n >= depth + 13) ? 3u : (n >= depth + 10) ? 2u : (n >= depth + 7) ? 1u : 0u;
    const uint64_t avail = s->budget / 2 > s->resident_bytes ? s->budget / 2 - s->resident_bytes : 0;
    for (; rows > 0; --rows) {                   // the deepest expansion that fits
        uint64_t Fd = 0;
        if ((rc = frontier_fill(n, depth + rows, nullptr, nullptr, nullptr, nullptr, 0, &Fd,
                                nullptr)) != NQ_OK)
            return rc;
        if (Fd * 13 + (F + 1) * 8 <= avail) break;
    }
    Resident r;
    r.rows = rows;
    r.len = F;
    if (F * 13 > avail && rows == 0) return NQ_ENOMEM;
    rc = build_device_frontier_at(n, depth, rows, s->aux, &r.fr, rows ? &r.off : nullptr);
    if (rc != NQ_OK) return rc;
    r.bytes = r.fr.len * 13 + r.off.size() * 8;
    if (r.bytes > avail) return NQ_ENOMEM;
    s->resident_bytes += r.bytes;
    auto ins = s->resident.emplace(key, std::move(r));
    *out = &ins.first->second;
    return NQ_OK;
}

// Copies `len` entries into the ring at logical position `pos` (wrapping).
template <class CopyFn>
void ring_segments(const nq_server* s, uint64_t pos, uint64_t len, CopyFn&& fn) {
    uint64_t phys = pos % s->ring_cap, done = 0;
    while (done < len) {
        const uint64_t take = std::min(len - done, s->ring_cap - phys);
        fn(phys, done, take);
        done += take;
        phys = 0;
    }
}

// A pending request handed to the scheduler thread (copied out under mu).
struct Candidate {
    uint64_t ticket;
    nq_request rq;
    uint32_t depth;
};

// What admission decided for a candidate, applied to its Req under mu.
struct Outcome {
    uint64_t ticket;
    int status;                 // NQ_OK, or the error the request ends with
    bool admitted;              // on the device (else finished now with `count`)
    uint64_t count;
    uint64_t entries, ring_start, ring_len;
    uint32_t slot, gen;
    uint64_t t;
};

// Reads the published results of admitted requests, marks them done and frees
// their slots and ring space.  mu held (it writes Req records).
void collect(nq_server* s) {
    const uint64_t t = now_ns();
    for (auto& a : s->admitted) {
        if (a.done) continue;
        const unsigned long long flag = __atomic_load_n(&s->h_flag[a.slot], __ATOMIC_ACQUIRE);
        if (flag != a.gen) continue;
        auto it = s->reqs.find(a.ticket);              // present until done and polled
        if (it != s->reqs.end()) {
            Req& r = it->second;
            r.count = __atomic_load_n(&s->h_val[a.slot], __ATOMIC_ACQUIRE);
            r.t_done = t;
            r.state = ReqState::Done;
        }
        a.done = true;
        s->free_slots.push_back(a.slot);
    }
    // Ring space is reclaimed in admission order.
    while (!s->admitted.empty() && s->admitted.front().done) {
        s->ring_head = s->admitted.front().ring_start + s->admitted.front().ring_len;
        s->admitted.pop_front();
    }
    if (s->admitted.empty()) s->ring_head = s->ring_tail;
    s->cv.notify_all();
}

// Retires finished epochs' staging buffers (scheduler thread, mu not held).
// An epoch whose event reports a device error is retired too; the error is
// returned, to become the server's fatal status: its requests will never
// publish.
int retire_epochs(nq_server* s) {
    int err = 0;
    // every finished epoch, not only a prefix: quick epochs end behind a long
    // one on another stream, and the list stays as short as the work in flight
    for (auto it = s->epochs.begin(); it != s->epochs.end();) {
        const hipError_t q = hipEventQuery(it->done);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        if (q != hipSuccess && err == 0) err = (int)q;
        (void)hipEventDestroy(it->done);
        it = s->epochs.erase(it);
    }
    return err;
}

bool quick_request(const nq_request& rq) {
    return rq.kind == NQ_REQ_COUNT && rq.n <= kQuickMaxN;
}

// The stream for the next epoch: one with no epoch in flight, so that an
// epoch never waits in stream order behind another (a short epoch queued
// behind an N = 18 count would wait for all of it), or -1 when every stream
// the epoch may take is busy (the candidates then wait in the queue, and the
// next epoch takes all that arrived meanwhile).  A quick epoch tries the
// latency lane first, and the other streams only when `lane_only` is false
// (no other request waits for them, so quick ones cannot starve them).  With
// `reserve` (NQ_FLAG_SERVE_RESERVE) other epochs take only the first stream,
// one at a time, and quick ones the lane and the two streams between.  With
// `round_robin` (NQ_SERVE_ROUND_ROBIN=1 in the environment, for measurement)
// epoch i goes to stream i mod kStreams, busy or not, whatever its requests.
int pick_stream(nq_server* s, bool quick, bool lane_only) {
    if (s->round_robin) return (int)(s->epoch_no % kStreams);
    bool busy[kStreams] = {};
    for (const Epoch& ep : s->epochs)
        if (!busy[ep.stream] && hipEventQuery(ep.done) == hipErrorNotReady) busy[ep.stream] = true;
    if (quick && !busy[kQuickStream]) return (int)kQuickStream;
    if (s->reserve) {
        if (!quick) return busy[0] ? -1 : 0;
        for (uint32_t k = 1; k + 1 < kStreams; ++k)
            if (!busy[k]) return (int)k;
        return -1;
    }
    if (quick && lane_only) return -1;
    for (uint32_t i = 0; i < kStreams - 1; ++i) {
        const uint32_t k = (uint32_t)((s->epoch_no + i) % (kStreams - 1));
        if (!busy[k]) return (int)k;
    }
    return -1;
}

// Admits candidates of one class (quick or not) in arrival order while
// request slots and ring space allow and launches one epoch over them
// (scheduler thread, mu not held: resident frontier builds and the enqueued
// copies and launch do not block submitters).  Quick requests go first when
// the latency lane (or, with no other request waiting, another stream) is
// free for them: they may overtake older requests of the other class, never
// one of their own.  decided[i] is set for every candidate admitted or
// finished; the others stay queued.
int admit_and_launch(nq_server* s, const std::vector<Candidate>& cand, std::vector<Outcome>* out,
                     std::vector<char>* decided) {
    decided->assign(cand.size(), 0);
    if (cand.empty() || s->free_slots.empty()) return NQ_OK;
    bool any_quick = false, any_other = false;
    for (const Candidate& c : cand) (quick_request(c.rq) ? any_quick : any_other) = true;
    const bool split = !s->round_robin;                   // round robin: one class
    int sidx = -1;
    bool quick_epoch = any_quick;
    if (any_quick) sidx = pick_stream(s, true, any_other);
    if (sidx < 0 && any_other) {
        sidx = pick_stream(s, false, false);
        quick_epoch = false;
    }
    if (sidx < 0) return NQ_OK;                           // every stream busy: wait
    TraceRange t("epoch");
    Epoch ep;
    ep.stream = (uint32_t)sidx;
    const uint64_t epoch_start = s->ring_tail;
    uint32_t frames = 0;                                  // deepest stack of the epoch
    // Whether every request of the epoch fits the default step's row marker
    // (board + its stack frames <= 30).  An epoch keeps to one kind: a run
    // of small requests is not made to test its last row by popcount because
    // a large one arrived among them; the large one starts the next epoch.
    bool small_epoch = true;
    struct Copy { const Resident* res; uint64_t src, pos, len; uint32_t slot; };
    std::vector<Copy> copies;
    size_t idx = 0;
    for (; idx < cand.size() && !s->free_slots.empty(); ++idx) {
        const Candidate& c = cand[idx];
        if (split && quick_request(c.rq) != quick_epoch) continue;   // the other class's epoch
        auto finish = [&](int status, uint64_t count) {
            const uint64_t now = now_ns();
            out->push_back({c.ticket, status, false, count, 0, 0, 0, 0, 0, now});
            (*decided)[idx] = 1;
        };
        Resident* res = nullptr;
        int rc = ensure_resident(s, c.rq.n, c.depth, c.rq.kind, &res);
        if (rc != NQ_OK) { finish(rc, 0); continue; }
        uint64_t lo = 0, hi = res->len;                   // entries of the (n, depth) frontier
        if (c.rq.kind == NQ_REQ_SLICE) {
            if (c.rq.start > res->len || c.rq.len > res->len - c.rq.start) {
                finish(NQ_EINVAL, 0);
                continue;
            }
            lo = c.rq.start;
            hi = c.rq.start + c.rq.len;
        }
        const uint64_t src = res->first(lo);
        const uint64_t F = res->first(hi) - src;          // subproblems in the ring
        if (F > s->ring_cap) { finish(NQ_ENOMEM, 0); continue; }  // can never fit
        if (s->ring_tail + F - s->ring_head > s->ring_cap) break;   // wait for space
        if (F == 0) { finish(NQ_OK, 0); continue; }       // nothing to search
        const uint32_t fr = frames_needed(c.rq.n, c.depth + res->rows);
        const bool small = c.rq.n + fr <= 30u;
        if (!copies.empty() && small != small_epoch) break;   // the next epoch takes it
        small_epoch = small;
        const uint32_t slot = s->free_slots.back();
        s->free_slots.pop_back();
        const uint32_t gen = ++s->slot_gen[slot];
        const uint64_t start = s->ring_tail;
        s->ring_tail += F;
        frames = std::max(frames, fr);
        ep.inits.push_back({slot, c.rq.n, (uint32_t)F, gen});
        copies.push_back({res, src, start, F, slot});
        out->push_back({c.ticket, NQ_OK, true, 0, F, start, F, slot, gen, now_ns()});
        (*decided)[idx] = 1;
        s->admitted.push_back({c.ticket, start, F, slot, gen, false});
    }
    if (copies.empty()) return NQ_OK;
    const uint64_t n_entries = s->ring_tail - epoch_start;
    hipStream_t st = s->streams[sidx];
    hipError_t e = hipSuccess;
    // 1. slot records, 2. every request's entries (device to device out of its
    // resident frontier) and instance ids, in ring order.
    const size_t init_off = (size_t)sidx * s->max_slots;
    nqi::SlotInit* d_init = s->d_init + init_off;
    if ((e = hipMemcpyAsync(d_init, ep.inits.data(), ep.inits.size() * sizeof(SlotInit),
                            hipMemcpyHostToDevice, st)) != hipSuccess) {
        set_hip_error(e);
        return NQ_EDEVICE;
    }
    int rc = launch_slot_init(d_init, (uint32_t)ep.inits.size(), s->s_n, s->s_rem, s->s_tot,
                              s->s_gen, st);
    if (rc != NQ_OK) return rc;
    for (const Copy& cp : copies) {
        const DeviceFrontier& fr = cp.res->fr;
        ring_segments(s, cp.pos, cp.len, [&](uint64_t phys, uint64_t off, uint64_t len) {
            if (e != hipSuccess || rc != NQ_OK) return;
            const uint64_t from = cp.src + off;
            if ((e = hipMemcpyAsync(s->r_cols + phys, fr.cols + from, len * 4,
                                    hipMemcpyDeviceToDevice, st)) != hipSuccess) return;
            if ((e = hipMemcpyAsync(s->r_ld + phys, fr.ld + from, len * 4,
                                    hipMemcpyDeviceToDevice, st)) != hipSuccess) return;
            if ((e = hipMemcpyAsync(s->r_rd + phys, fr.rd + from, len * 4,
                                    hipMemcpyDeviceToDevice, st)) != hipSuccess) return;
            if ((e = hipMemcpyAsync(s->r_w + phys, fr.w + from, len, hipMemcpyDeviceToDevice,
                                    st)) != hipSuccess) return;
            rc = launch_fill_u32(s->r_inst + phys, cp.slot, len, st);
        });
    }
    if (rc != NQ_OK) return rc;
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    // 5. the epoch: one persistent launch over [epoch_start, ring_tail).
    DfsParams P{};
    P.cols = s->r_cols; P.ld = s->r_ld; P.rd = s->r_rd; P.weight = s->r_w;
    P.inst = s->r_inst; P.inst_n = s->s_n; P.ninst = s->max_slots;
    P.totals = s->s_tot;
    P.head = s->heads + (size_t)sidx * kHeadStride;        // one head per stream, in its order
    P.len = n_entries;
    P.frames = frames;
    P.refill_every = s->launch.refill_every ? s->launch.refill_every : 512u;
    P.idle_min = default_idle_min();
    P.reverse = 0;                                      // arrival order
    P.base = epoch_start % s->ring_cap;
    P.wrap = s->ring_cap;
    P.remaining = s->s_rem;
    P.inst_gen = s->s_gen;
    P.host_val = s->d_val;
    P.host_flag = s->d_flag;
    // plan_launch keeps the marker when its largest board + frames <= 30;
    // here each request was checked against its own frames above
    const int small = small_epoch ? 1 : 0;
    if (!s->cfg_ready[small][frames]) {
        if ((rc = plan_launch(s->devinfo, NQ_MODE_PERSISTENT, s->launch.wg_size,
                              s->launch.waves_per_cu, frames, 1, false, true,
                              &s->cfg_by_frames[small][frames], true, false,
                              small ? 30u - frames : NQ_MAX_N_WIDE)) != NQ_OK)
            return rc;
        s->cfg_ready[small][frames] = true;
    }
    LaunchCfg cfg = s->cfg_by_frames[small][frames];
    const uint64_t waves = (n_entries + 63) / 64;
    const uint64_t per_wg = cfg.wg_size / 64u;
    if (s->reserve && !quick_epoch && split) {
        // one resident wave per CU fewer than the LDS allows: room for quick epochs
        const uint32_t per_cu = cfg.grid / s->cu_count;  // resident workgroups per CU
        if (per_cu > 1) cfg.grid = (per_cu - 1) * s->cu_count;
    }
    cfg.grid = (uint32_t)std::min<uint64_t>(cfg.grid, (waves + per_wg - 1) / per_wg);
    P.claim = default_claim(n_entries, cfg);
    if ((rc = launch_dfs(cfg, P, st)) != NQ_OK) return rc;
    if ((e = hipEventCreateWithFlags(&ep.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventRecord(ep.done, st)) != hipSuccess) {
        set_hip_error(e);
        return NQ_EDEVICE;
    }
    s->epochs.push_back(std::move(ep));
    ++s->epoch_no;
    return NQ_OK;
}

// Applies admission outcomes and returns undecided candidates to the front of
// the queue in their order (or drops them when the server is being
// destroyed, as the queue itself was).  mu held.
void apply(nq_server* s, const std::vector<Candidate>& cand, const std::vector<Outcome>& out,
           const std::vector<char>& decided) {
    for (const Outcome& o : out) {
        auto it = s->reqs.find(o.ticket);
        if (it == s->reqs.end()) continue;
        Req& r = it->second;
        r.status = o.status;
        r.t_admit = o.t;
        if (o.admitted) {
            r.state = ReqState::Admitted;
            r.slot = o.slot;
            r.gen = o.gen;
            r.ring_start = o.ring_start;
            r.ring_len = o.ring_len;
            r.entries = o.entries;
        } else {
            r.count = o.count;
            r.t_done = o.t;
            r.state = ReqState::Done;
        }
    }
    for (size_t i = cand.size(); i-- > 0;) {
        if (i < decided.size() && decided[i]) continue;
        if (s->stop)
            s->reqs.erase(cand[i].ticket);
        else
            s->pending.push_front(cand[i].ticket);
    }
    s->cv.notify_all();
}

void worker_main(nq_server* s) {
    std::vector<Candidate> cand;
    std::vector<Outcome> out;
    std::vector<char> decided;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        cand.clear();
        out.clear();
        decided.clear();
        int rc = NQ_OK, hip = 0;
        try {
            collect(s);
            // The oldest pending requests, as many as there are free slots,
            // leave the queue while the device work is enqueued unlocked.
            if (s->fatal == NQ_OK) {
                const size_t take = std::min(s->pending.size(), s->free_slots.size());
                cand.reserve(take);
                out.reserve(take);
                for (size_t i = 0; i < take; ++i) {
                    const uint64_t t = s->pending.front();
                    const Req& r = s->reqs.at(t);
                    cand.push_back({t, r.rq, r.depth});
                    s->pending.pop_front();
                }
            }
            lk.unlock();
            if (const int ev = retire_epochs(s)) {
                rc = NQ_EDEVICE;
                hip = ev;
            } else if (!cand.empty()) {
                rc = admit_and_launch(s, cand, &out, &decided);
                if (rc != NQ_OK) hip = nq_last_hip_error();   // set on this (the worker) thread
            }
        } catch (...) {                 // a host allocation failed: stop admitting
            rc = NQ_ENOMEM;
            hip = 0;
        }
        if (!lk.owns_lock()) lk.lock();
        apply(s, cand, out, decided);
        if (rc != NQ_OK && s->fatal == NQ_OK) {
            s->fatal = rc;
            s->fatal_hip = hip;
            s->cv.notify_all();
        }
        // After a fatal error nothing admitted is waited for: its results
        // will not come, and pollers see the error instead.
        const bool busy = s->fatal == NQ_OK && (!s->admitted.empty() || !s->epochs.empty());
        if (s->stop && !busy) break;
        if (busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            // (after a fatal error pending requests are never admitted)
            s->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
                return s->stop || (s->fatal == NQ_OK && !s->pending.empty());
            });
        }
    }
}

void destroy_all(nq_server* s) {
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamSynchronize(st);
    if (s->aux) (void)hipStreamSynchronize(s->aux);
    for (auto& ep : s->epochs)
        if (ep.done) (void)hipEventDestroy(ep.done);
    if (s->dev) (void)hipFree(s->dev);
    if (s->h_val) (void)hipHostFree(s->h_val);
    if (s->h_flag) (void)hipHostFree(s->h_flag);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    s->resident.clear();
    if (s->aux) (void)hipStreamDestroy(s->aux);
    delete s;
}

}  // namespace

int serve_create(const nq_opts* opts, uint64_t hbm_budget, nq_server** out) {
    if (!out) return NQ_EINVAL;
    if (opts && (opts->flags & ~NQ_FLAGS_ALL) != 0) return NQ_EINVAL;
    // queens only; request totals are 64-bit (every board <= 28)
    if (opts && (opts->flags & (NQ_FLAG_KINGS | NQ_FLAG_WIDE_TOTAL))) return NQ_EINVAL;
    nq_server* s = new (std::nothrow) nq_server();
    if (!s) return NQ_ENOMEM;
    if (opts) s->launch = *opts;
    if (const char* rr = std::getenv("NQ_SERVE_ROUND_ROBIN")) s->round_robin = rr[0] == '1';
    s->reserve = opts && (opts->flags & NQ_FLAG_SERVE_RESERVE);
    s->budget = hbm_budget ? hbm_budget : (8ull << 30);
    // Frames: requests whose subproblems need more are refused at submit.
    s->max_frames = (opts && opts->depth) ? opts->depth : 14u;
    if (s->max_frames > NQ_MAX_N - 2) {                  // deeper than any board needs
        delete s;
        return NQ_EINVAL;
    }
    // Half of the budget is the work ring, the other half resident frontiers.
    s->ring_cap = std::min<uint64_t>(1ull << 31,
                                     std::max<uint64_t>(1u << 16, (s->budget / 2) / kRingEntryBytes));
    s->free_slots.reserve(s->max_slots);
    for (uint32_t i = 0; i < s->max_slots; ++i) s->free_slots.push_back(s->max_slots - 1 - i);
    s->slot_gen.assign(s->max_slots, 0);
    hipError_t e;
    auto fail = [&](int rc) {
        destroy_all(s);
        return rc;
    };
    int rc = device_info(&s->devinfo);
    if (rc != NQ_OK) return fail(rc);
    s->cu_count = (uint32_t)s->devinfo.cu_count;
    // The largest epoch must fit: planned here so that a bad launch option is
    // refused at creation.
    if ((rc = plan_launch(s->devinfo, NQ_MODE_PERSISTENT, s->launch.wg_size,
                          s->launch.waves_per_cu, s->max_frames, 1, false, true,
                          &s->cfg_by_frames[0][s->max_frames], true)) != NQ_OK)
        return fail(rc);
    s->cfg_ready[0][s->max_frames] = true;
    const uint64_t R = s->ring_cap, S = s->max_slots;
    const size_t o_ld = R * 4, o_rd = R * 8, o_inst = R * 12, o_w = R * 16;
    const size_t o_sn = (o_w + R + 255) / 256 * 256, o_rem = o_sn + S * 4, o_gen = o_rem + S * 4;
    const size_t o_tot = (o_gen + S * 4 + 255) / 256 * 256, o_heads = o_tot + S * 8;
    const size_t o_init = o_heads + kHeads * 8, bytes = o_init + kStreams * S * sizeof(SlotInit);
    if ((e = hipMalloc(&s->dev, bytes)) != hipSuccess) {
        set_hip_error(e);
        return fail(e == hipErrorOutOfMemory ? NQ_ENOMEM : NQ_EDEVICE);
    }
    char* b = static_cast<char*>(s->dev);
    s->r_cols = reinterpret_cast<uint32_t*>(b);
    s->r_ld = reinterpret_cast<uint32_t*>(b + o_ld);
    s->r_rd = reinterpret_cast<uint32_t*>(b + o_rd);
    s->r_inst = reinterpret_cast<uint32_t*>(b + o_inst);
    s->r_w = reinterpret_cast<uint8_t*>(b + o_w);
    s->s_n = reinterpret_cast<uint32_t*>(b + o_sn);
    s->s_rem = reinterpret_cast<uint32_t*>(b + o_rem);
    s->s_gen = reinterpret_cast<uint32_t*>(b + o_gen);
    s->s_tot = reinterpret_cast<unsigned long long*>(b + o_tot);
    s->heads = reinterpret_cast<unsigned long long*>(b + o_heads);
    s->d_init = reinterpret_cast<SlotInit*>(b + o_init);
    const unsigned host_flags = hipHostMallocMapped | hipHostMallocCoherent;
    if ((e = hipHostMalloc((void**)&s->h_val, S * 8, host_flags)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->h_flag, S * 8, host_flags)) != hipSuccess) {
        set_hip_error(e);
        return fail(NQ_ENOMEM);
    }
    std::memset(s->h_val, 0, S * 8);
    std::memset(s->h_flag, 0, S * 8);
    if ((e = hipHostGetDevicePointer((void**)&s->d_val, s->h_val, 0)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&s->d_flag, s->h_flag, 0)) != hipSuccess) {
        set_hip_error(e);
        return fail(NQ_EDEVICE);
    }
    for (auto& st : s->streams)
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
            set_hip_error(e);
            return fail(NQ_EDEVICE);
        }
    if ((e = hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking)) != hipSuccess) {
        set_hip_error(e);
        return fail(NQ_EDEVICE);
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        return fail(NQ_ENOMEM);
    }
    *out = s;
    return NQ_OK;
}

// The server's fatal status, with its HIP error made visible to
// nq_last_hip_error() on the calling thread (the worker thread met it).
int fatal_status(const nq_server* s) {
    set_hip_error(s->fatal_hip);
    return s->fatal;
}

int serve_submit(nq_server* s, const nq_request* rq, uint64_t* ticket) {
    if (!s || !rq || !ticket) return NQ_EINVAL;
    if (rq->n < 1 || rq->n > NQ_MAX_N || rq->reserved != 0) return NQ_EINVAL;
    Req r;
    r.rq = *rq;
    if (rq->kind == NQ_REQ_COUNT) {
        r.depth = rq->depth ? rq->depth : count_depth(rq->n, s->max_frames);
        if (r.depth > rq->n) return NQ_EINVAL;
    } else if (rq->kind == NQ_REQ_SLICE) {
        if (rq->depth < 1 || rq->depth > rq->n) return NQ_EINVAL;
        if (rq->start + rq->len < rq->start) return NQ_EINVAL;
        r.depth = rq->depth;
    } else {
        return NQ_EINVAL;
    }
    if (frames_needed(rq->n, r.depth) > s->max_frames) return NQ_EINVAL;   // LDS footprint
    if (!leafctr_ok(rq->n, r.depth)) return NQ_EINVAL;                   // row counter range
    r.t_submit = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != NQ_OK) return fatal_status(s);
    if (s->pending.size() >= 65536) return NQ_EFULL;
    const uint64_t t = s->next_ticket++;
    s->reqs.emplace(t, r);
    s->pending.push_back(t);
    *ticket = t;
    s->cv.notify_all();
    return NQ_OK;
}

int serve_poll(nq_server* s, uint64_t ticket, nq_result* out, uint64_t wait_ns) {
    if (!s || !out) return NQ_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return NQ_ENOENT;
    if (it->second.state != ReqState::Done && wait_ns) {
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(wait_ns);
        s->cv.wait_until(lk, deadline, [&] {
            const auto j = s->reqs.find(ticket);   // another poller may take it
            return s->fatal != NQ_OK || j == s->reqs.end() || j->second.state == ReqState::Done;
        });
        it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return NQ_ENOENT;
    }
    const Req& r = it->second;
    if (r.state != ReqState::Done) return s->fatal != NQ_OK ? fatal_status(s) : NQ_EAGAIN;
    out->status = r.status;
    out->reserved = 0;
    out->count = r.count;
    out->entries = r.entries;
    out->t_submit_ns = r.t_submit;
    out->t_admit_ns = r.t_admit;
    out->t_done_ns = r.t_done;
    s->reqs.erase(it);
    return NQ_OK;
}

int serve_destroy(nq_server* s) {
    if (!s) return NQ_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // requests never admitted are dropped
        for (uint64_t t : s->pending) s->reqs.erase(t);
        s->pending.clear();
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    const int fatal = s->fatal != NQ_OK ? fatal_status(s) : NQ_OK;
    destroy_all(s);
    return fatal;
}

}  // namespace nqi

extern "C" int nq_serve_create(const nq_opts* opts, uint64_t hbm_budget_bytes, nq_server** out) {
    try {
        return nqi::serve_create(opts, hbm_budget_bytes, out);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_serve_submit(nq_server* s, const nq_request* req, uint64_t* out_ticket) {
    try {
        return nqi::serve_submit(s, req, out_ticket);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_serve_poll(nq_server* s, uint64_t ticket, nq_result* out) {
    try {
        return nqi::serve_poll(s, ticket, out, 0);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_serve_wait(nq_server* s, uint64_t ticket, nq_result* out, uint64_t timeout_ns) {
    try {
        return nqi::serve_poll(s, ticket, out, timeout_ns ? timeout_ns : 1);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_serve_destroy(nq_server* s) {
    try {
        return nqi::serve_destroy(s);
    } catch (...) {
        return NQ_EDEVICE;            // the worker thread could not be joined
    }
}
