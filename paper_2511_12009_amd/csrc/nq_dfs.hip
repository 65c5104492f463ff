// DFS kernels for gfx950 (CDNA4, wave64).
//
// One lane of a 64-wide wavefront owns one subproblem at a time and searches
// its subtree with the iterative DFS of Algorithm 2 (Section 2), using the
// merged last-row step of Algorithm 3 (Section 3.2.3 / Section 4.3): the free
// squares of row N-1 are counted with a popcount and never pushed.
//
// Lane state.  The frame being expanded -- (cols, ld, rd, avail) -- lives in
// VGPRs.  Ancestors that still have untried columns are kept in LDS; an
// ancestor with no untried column is never stored, so a pop always lands on a
// frame with work and every loop trip places exactly one queen (one DFS node).
//
// LDS layout (the bank-conflict-free stack of Section 3.1, re-derived for a
// 64-lane wave and 16-byte frames): wave w of a workgroup owns S * 64 * 16
// bytes, S = the stack's frames plus, in every form but the default one, a
// sentinel slot; slot f of lane l is the 16-byte frame at index
// (w * S + f) * 64 + l, slot 0 holding the lane's sentinel where there is one.
// A wave-wide ds_write_b128 / ds_read_b128 touches one 16-byte slot per lane,
// and the slot's bank offset depends on l only (64 * 16 bytes is a multiple of
// every bank-row size), so lanes at different depths never collide.
//
// Scheduling.  Plain mode: lane i of the grid takes entry i and idles once its
// subtree is done.  Persistent mode: a resident grid; a wave visits the
// scheduler every `refill_every` DFS steps, or earlier once `idle_min` of its
// lanes are idle.  A visit retires finished lanes, then hands its idle lanes
// entries by rank (mbcnt): first from the wave's own block of claimed entries,
// then from a fresh block of at least `claim` entries taken with one atomic add
// on a global head.  The idle lanes therefore read consecutive entries with
// coalesced loads, and the head sees one atomic per block rather than one per
// visit.  By default entries are claimed from the end of the frontier down:
// subtrees below the later row-0 columns are the larger ones (the per-GPU times
// of Section 4.5 grow with the position in the frontier), and starting them
// first shortens the tail of the launch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>

#include "nq_internal.h"
#include "nq_wave.h"

namespace nqi {

// Default inner-loop form of the DFS kernels (see nq_dfs_kernel).
constexpr int kDefaultLoop = 7;
constexpr int kLoopForms = 8;          // forms 0..7
// LDS frames per lane that a form needs beyond N - 2 - placed.
constexpr uint32_t kFormExtraFrames[kLoopForms] = {0, 0, 0, 1, 1, 1, 1, 1};
// Sentinel slots per lane below its stack.  Form 7 parks a finished lane in
// registers instead, which leaves each wave 1 KB more room for other waves.
constexpr uint32_t kFormSentinel[kLoopForms] = {1, 1, 1, 1, 1, 1, 1, 0};


// Serving: the wave's retirements, added to their requests.  A request's total
// and remaining count are only touched by device-scope atomics; the lane whose
// subtraction takes the remaining count to zero publishes the total to host
// memory: value first, then the generation flag, each a system-scope store,
// so a host that sees the flag also sees the value.
//
// Ordering without cache maintenance: device-scope atomics are performed at
// one point for all CUs, and a flush waits for its addition to the total to
// return before it issues its subtraction, so when the subtractions reach zero
// every addition has been performed and the finishing lane's atomic read of
// the total sees them all.  (A device-scope fence here would write back and
// invalidate the L2 of the wave's XCD.)
//
// Each atomic pair makes the wave wait for a round trip to that point, so a
// wave keeps what its lanes retire for one request (wave-uniform: slot, sum,
// entries) and flushes it when a retirement of another request arrives, after
// kRetireHold scheduler visits, or when the wave ends; the lanes of a wave
// mostly hold consecutive entries of one request, so most visits only add to
// the held sum.
constexpr uint32_t kNoSlot = 0xffffffffu;
constexpr uint32_t kRetireHold = 8;

struct RetireHold {
    uint32_t slot = kNoSlot;     // request slot held (wave-uniform), kNoSlot = none
    uint32_t entries = 0;        // entries retired and not yet subtracted
    uint32_t visits = 0;         // scheduler visits since the first held retirement
    uint64_t sum = 0;            // weighted count not yet added
};

// Adds the held retirements to their request (lane 0 issues the atomics).
__device__ __forceinline__ void retire_flush(RetireHold& h, uint32_t* remaining,
                                             unsigned long long* totals, const uint32_t* gen,
                                             unsigned long long* host_val,
                                             unsigned long long* host_flag, uint32_t lane) {
    if (h.slot == kNoSlot) return;
    if (lane == 0) {
        const uint32_t s0 = h.slot;
        if (h.sum != 0) {
            const unsigned long long was = __hip_atomic_fetch_add(
                &totals[s0], (unsigned long long)h.sum, __ATOMIC_RELAXED,
                __HIP_MEMORY_SCOPE_AGENT);
            asm volatile("" : : "v"(was) : "memory");       // returned: performed
        }
        const uint32_t before = __hip_atomic_fetch_sub(&remaining[s0], h.entries,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before == h.entries) {
            const unsigned long long t = __hip_atomic_fetch_add(
                &totals[s0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&host_val[s0], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host_flag[s0], (unsigned long long)gen[s0], __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    h.slot = kNoSlot;
    h.entries = 0;
    h.visits = 0;
    h.sum = 0;
}

// One scheduler visit's retirements: `retiring` lanes pass their request slot
// `s` and weighted count `val`; every lane of the wave calls it.  The lanes of
// one request are summed with a wave reduction and added to the held
// retirements (flushing those first when they belong to another request).
__device__ __forceinline__ void retire_to_requests(RetireHold& h, uint32_t* remaining,
                                                   unsigned long long* totals,
                                                   const uint32_t* gen,
                                                   unsigned long long* host_val,
                                                   unsigned long long* host_flag, bool retiring,
                                                   uint32_t s, uint64_t val, uint32_t lane) {
    uint64_t pend = __builtin_amdgcn_ballot_w64(retiring);
    while (pend != 0) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint32_t s0 = __builtin_amdgcn_readfirstlane((uint32_t)__shfl((int)s, leader, 64));
        const bool mine = retiring && s == s0;
        const uint64_t grp = __builtin_amdgcn_ballot_w64(mine);
        uint64_t add = mine ? val : 0u;
        for (int off = 32; off > 0; off >>= 1) add += shfl_xor_u64(add, off);
        if (h.slot != s0)
            retire_flush(h, remaining, totals, gen, host_val, host_flag, lane);
        h.slot = s0;
        h.entries += (uint32_t)__popcll(grp);
        h.sum += add;
        pend &= ~grp;
    }
    if (h.slot != kNoSlot && ++h.visits >= kRetireHold)
        retire_flush(h, remaining, totals, gen, host_val, host_flag, lane);
}

// Per-lane state of the search.  `top` and `floor` are LDS byte addresses in
// the lane's column of the wave's stack region; the frame at `floor` is a
// sentinel (cols = all 32 bits set, avail = 0).  Popping it leaves the lane in
// a state in which every later step is a no-op: no free column, no free square
// below (cols + step keeps every column bit set, whatever the step), no leaf
// (bit 31 clear after the wrap-around), and the stack pointer pinned at the
// sentinel.  So "avail == 0 after a step" means "subtree finished", with no
// per-lane loop exit.  A lane whose entry needs no search parks in the same
// state.
//
// Leaf test.  With LEAFCTR the bits of `cols` above the board hold a row
// counter, advanced by the same add that places the queen; it is started so
// that bit 31 becomes set exactly when the queen just placed fills row N-2 (the
// next row is the last one).  The test is then a sign check instead of a
// popcount.  It needs N - 1 - placed <= 2^(31 - N) (always true for N <= 26);
// otherwise the popcount form of Algorithm 3 is used.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// cols of a parked or finished lane (see the kernel comment).
constexpr uint32_t kParked = 0xffffffffu;
typedef __attribute__((address_space(3))) u32x4 lds_frame;

// A frame addressed by its absolute LDS byte address.
__device__ __forceinline__ lds_frame* frame_at(int32_t addr) {
    return (lds_frame*)(uintptr_t)(uint32_t)addr;
}

// One 32-bit word of the LDS stack by its absolute byte address.
__device__ __forceinline__ __attribute__((address_space(3))) uint32_t* word_at(int32_t addr) {
    return (__attribute__((address_space(3))) uint32_t*)(uintptr_t)(uint32_t)addr;
}

// Exec-masked helpers for the hand-scheduled loops (forms 1 and 2).  Each block
// switches exec to the given lane mask, does its LDS access and stack-pointer
// update, and restores exec before the block ends.  The SALU instructions in a
// block overwrite SCC, so every such block lists it as clobbered (otherwise
// the compiler may keep a loop-exit compare in SCC across the block).

// Push: frame -> [top + 1024], top += 1024 for the lanes in `m`.
__device__ __forceinline__ void isa_push(u32x4 st, int32_t& top, uint64_t m) {
    uint64_t sv;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m]\n\t"
        "ds_write_b128 %[top], %[st] offset:1024\n\t"
        "v_add_u32 %[top], 0x400, %[top]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [top] "+v"(top), [sv] "=&s"(sv)
        : [m] "s"(m), [st] "v"(st)
        : "memory", "scc");
}

// Pop: frame <- [top], top = max(top - 1024, floor) for the lanes in `m`; the
// loaded frame is waited for before the block ends.
__device__ __forceinline__ void isa_pop(u32x4& st, int32_t& top, int32_t floor, uint64_t m) {
    uint64_t sv;
    int32_t t;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m]\n\t"
        "ds_read_b128 %[st], %[top]\n\t"
        "v_add_u32 %[t], 0xfffffc00, %[top]\n\t"
        "v_max_i32 %[top], %[t], %[fl]\n\t"
        "s_mov_b64 exec, %[sv]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [st] "+v"(st), [top] "+v"(top), [sv] "=&s"(sv), [t] "=&v"(t)
        : [m] "s"(m), [fl] "v"(floor)
        : "memory", "scc");
}

// p = lowest set bit of v; v loses it (in place, so the loop-carried register
// of v is also the one the pop writes).
__device__ __forceinline__ void isa_take_lowest(uint32_t& v, uint32_t& p) {
    uint32_t neg;
    asm("v_sub_u32 %[n], 0, %[v]\n\t"
        "v_and_b32 %[p], %[v], %[n]\n\t"
        "v_xor_b32 %[v], %[v], %[p]"
        : [v] "+v"(v), [p] "=&v"(p), [n] "=&v"(neg));
}

// Forms 6 and 7's push: every lane writes its frame to [top + 1024], the slot
// above its stack, which holds nothing (the lanes that do not push overwrite
// free space).  No exec mask.
__device__ __forceinline__ void isa_store_above(u32x4 st, int32_t top) {
    asm volatile("ds_write_b128 %[top], %[st] offset:1024"
                 : : [top] "v"(top), [st] "v"(st) : "memory");
}

// Lanes with a != 0, from a itself (one compare; the compiler would rather
// recompute the OR of a's three sources, one instruction more).
__device__ __forceinline__ uint64_t isa_nonzero(uint32_t a) {
    uint64_t m;
    asm("v_cmp_ne_u32 %0, 0, %1" : "=s"(m) : "v"(a));
    return m;
}

// Select: d = m ? a : d per lane (v_cndmask with an SGPR lane mask).
__device__ __forceinline__ uint32_t isa_sel(uint64_t m, uint32_t a, uint32_t d) {
    asm("v_cndmask_b32 %0, %0, %1, %2" : "+v"(d) : "v"(a), "s"(m));
    return d;
}
__device__ __forceinline__ uint32_t isa_sel_u(uint64_t m, uint32_t a, uint32_t d) {
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(d), "v"(a), "s"(m));
    return r;
}
__device__ __forceinline__ int32_t isa_sel_i(uint64_t m, int32_t a, int32_t d) {
    int32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(d), "v"(a), "s"(m));
    return r;
}

// sum += 1 for the lanes in `m` (carry-in add).
__device__ __forceinline__ void isa_count(uint32_t& sum, uint64_t m) {
    uint64_t junk;
    asm("v_addc_co_u32 %0, %1, %0, 0, %2" : "+v"(sum), "=s"(junk) : "s"(m));
}

// Negated untried set w = -avail: p = lowest untried column, w becomes
// -(avail - p) in place, zm = lanes whose untried set is now empty (the carry
// out of w + p).  The mask leaves the block in an SGPR pair and is only read by
// SALU code.
__device__ __forceinline__ void isa_take_neg(uint32_t& w, uint32_t& p, uint64_t& zm) {
    uint32_t t;
    asm("v_sub_u32 %[t], 0, %[w]\n\t"
        "v_and_b32 %[p], %[w], %[t]\n\t"
        "v_add_co_u32 %[w], %[z], %[w], %[p]"
        : [w] "+v"(w), [p] "=&v"(p), [t] "=&v"(t), [z] "=&s"(zm));
}

// Returns -a; am = lanes with a != 0 (the borrow of 0 - a), read by SALU
// code only.
__device__ __forceinline__ uint32_t isa_neg_any(uint32_t a, uint64_t& am) {
    uint32_t n;
    asm("v_sub_co_u32 %0, %1, 0, %2" : "=v"(n), "=s"(am) : "v"(a));
    return n;
}

// Form 3's first instructions: p = lowest untried column of w, w loses it (in
// place), and alive = lanes whose w was not empty (the borrow of 0 - w), read
// by SALU code only.
__device__ __forceinline__ void isa_take_alive(uint32_t& w, uint32_t& p, uint64_t& alive) {
    uint32_t neg;
    asm("v_sub_co_u32 %[n], %[al], 0, %[w]\n\t"
        "v_and_b32 %[p], %[w], %[n]\n\t"
        "v_xor_b32 %[w], %[w], %[p]"
        : [w] "+v"(w), [p] "=&v"(p), [n] "=&v"(neg), [al] "=&s"(alive));
}

// Form 3's pop: frame <- [top], top -= 1024 for the lanes in `m`, with no
// clamp (a lane pops only while it has work, so it pops its sentinel at most
// once); the loaded frame is waited for before the block ends.
__device__ __forceinline__ void isa_pop_free(u32x4& st, int32_t& top, uint64_t m) {
    uint64_t sv;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m]\n\t"
        "ds_read_b128 %[st], %[top]\n\t"
        "v_add_u32 %[top], 0xfffffc00, %[top]\n\t"
        "s_mov_b64 exec, %[sv]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [st] "+v"(st), [top] "+v"(top), [sv] "=&s"(sv)
        : [m] "s"(m)
        : "memory", "scc");
}

// One step's stack and frame update for form 2: lanes in `pm` store the frame
// at [top + 1024] and advance top, lanes in `dm` take the child frame `ch`
// (four v_cndmask), lanes in `qm` reload the frame at [top] and step top back.
// The three masks are disjoint.  No clamp: a lane that has popped its sentinel
// is parked and its masks stay empty until it takes a new entry.
__device__ __forceinline__ void isa_step128(u32x4& st, u32x4 ch, int32_t& top, uint64_t pm,
                                            uint64_t dm, uint64_t qm) {
    uint64_t sv;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[pm]\n\t"
        "ds_write_b128 %[top], %[st] offset:1024\n\t"
        "v_add_u32 %[top], 0x400, %[top]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [top] "+v"(top), [sv] "=&s"(sv)
        : [pm] "s"(pm), [st] "v"(st)
        : "memory", "scc");
    st.x = isa_sel(dm, ch.x, st.x);
    st.y = isa_sel(dm, ch.y, st.y);
    st.z = isa_sel(dm, ch.z, st.z);
    st.w = isa_sel(dm, ch.w, st.w);
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[qm]\n\t"
        "ds_read_b128 %[st], %[top]\n\t"
        "v_add_u32 %[top], 0xfffffc00, %[top]\n\t"
        "s_mov_b64 exec, %[sv]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [st] "+v"(st), [top] "+v"(top), [sv] "=&s"(sv)
        : [qm] "s"(qm)
        : "memory", "scc");
}

// LOOP selects the inner-loop form: 0 = plain C++ (the compiler places the
// exec masks), 1 = hand-placed exec masks, 2 = as 1 with the untried set kept
// negated so that two lane masks come from carries, 3 = the step without
// selects, 6 = form 3 with a push that needs no exec mask, 7 = form 6 without
// the sentinel slot (the default; see below).  Two
// more forms exist to measure the paper's own design choices: 4 keeps the
// frame being expanded in the LDS stack too (read every step, its untried set
// written back: Algorithm 2 as the paper prints it, with the last-row step of
// Algorithm 3) and 5 is form 0 without the last-row step (the last row is
// searched like any other).  Both need one LDS frame more per lane, which the
// launcher adds to P.frames (kFormExtraFrames).  SERVE
// (persistent launches of the serving loop, P.remaining set) compiles in the
// per-request retirement; it is a template flag so that the scheduler visit
// of every other launch carries none of its code.  KINGS runs the second
// search (n kings, one per row and column): the same stack, scheduler and
// leaf test, with the next row's attacked squares taken from the placed king
// alone (no diagonals carried down); it exists for forms 1 and 7, form 7 with
// the popcount leaf test only (the kings' rd is recomputed from the king just
// placed, so it cannot carry the row marker).
template <bool PERSISTENT, bool STATS, bool LEAFCTR, int LOOP, bool SERVE, bool KINGS = false>
__global__ __launch_bounds__(1024) void nq_dfs_kernel(DfsParams P) {
    static_assert(!KINGS || LOOP == 1 || (LOOP == 7 && !LEAFCTR),
                  "the kings search runs in form 1, or in form 7 with the popcount leaf test");
    constexpr bool F3 = LOOP == 3 || LOOP >= 6;      // the step without selects
    constexpr bool SENT = kFormSentinel[LOOP] != 0u;
    extern __shared__ uint4 lds_stack[];
    const int32_t lds = (int32_t)(uint32_t)(uintptr_t)(lds_frame*)lds_stack;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    // Slot 0 of the lane: its sentinel, or (form 6) its first frame; an empty
    // stack has `top` one slot below it.
    const int32_t floor =
        lds + (int32_t)(((wave * (P.frames + kFormSentinel[LOOP])) * 64u + lane) * 16u);
    const int32_t empty_top = SENT ? floor : floor - 1024;
    int32_t top = empty_top;
    if (SENT) *frame_at(floor) = u32x4{kParked, 0u, 0u, 0u};

    uint32_t c = kParked, l = 0, r = 0, v = 0, last = 0, nm1 = 0, step_k = 0;
    uint32_t leaf_lim = 0;                // form 3 with LEAFCTR: rd below this = leaf
    uint64_t idx = 0;
    uint32_t sum32 = 0, steps32 = 0;
    uint64_t sum64 = 0, steps64 = 0;
    uint64_t wtotal = 0;                  // weighted total, single-instance launches
    uint64_t wtotal_hi = 0;               // its carries (128-bit totals, P.wide)
    uint32_t acc_s = 0u;                  // batches: instance of the lane's pending sum
    uint64_t acc_v = 0;                   // batches: weighted sum not yet added
    RetireHold held;                      // serving: retirements not yet added
    bool has_task = false;                // holds an entry not yet retired
    bool exhausted = !PERSISTENT;         // no entries left to claim (wave-uniform)
    bool claimed_all = false;             // head has passed the end (wave-uniform)
    uint64_t qlo = 0, qhi = 0;            // claimed entries not yet taken (wave-uniform)

    // Takes entry `i`: loads its triple, writes the sentinel and settles the
    // cases that need no search (a full board, the last row, no free square).
    auto take = [&](uint64_t i) {
        if (PERSISTENT && P.reverse) i = P.len - 1 - i;
        if (P.wrap) {
            i += P.base;
            if (i >= P.wrap) i -= P.wrap;
        }
        idx = i;
        uint32_t n = P.n;
        bool bad_inst = false;
        if (P.inst) {
            const uint32_t s = P.inst[i];
            bad_inst = s >= P.ninst;
            n = bad_inst ? 1u : P.inst_n[s];
        }
        last = (1u << n) - 1u;
        nm1 = n - 1u;
        c = P.cols[i] & last;
        l = P.ld[i] & last;
        r = P.rd[i] & last;
        v = 0u;
        top = empty_top;
        sum32 = 0; sum64 = 0; steps32 = 0; steps64 = 0;
        has_task = true;
        const uint32_t placed = __popc(c);
        const uint32_t avail = last & ~(c | l | r);
        step_k = LEAFCTR ? (1u << n) : 0u;
        if (SENT) *frame_at(floor) = u32x4{kParked, 0u, 0u, 0u};
        if (bad_inst || n < 1u || n > NQ_MAX_N_WIDE) {
            sum64 = kCountInvalid;        // instance id or board size out of range
        } else if (placed >= nm1) {
            sum32 = (placed == n) ? 1u : __popc(avail);
        } else if (n - 2u - placed > P.frames - kFormExtraFrames[LOOP] ||
                   (LEAFCTR && !F3 && nm1 - placed > (1u << (31u - n))) ||
                   (LEAFCTR && F3 && 2u * n - 1u - placed > 31u)) {
            sum64 = kCountInvalid;        // does not fit this launch's stack or counter
        } else if (avail != 0u) {
            v = avail;
            if (F3) {
                // forms 3, 6 and 7: the columns off the board count as taken,
                // so the free squares of the next row are one 3-input NOR; with
                // LEAFCTR a marker bit rides in rd, one place lower per row,
                // and reaches bit n exactly in the frames of the last row
                c |= ~last;
                if (LEAFCTR) {
                    r |= 1u << (2u * n - 1u - placed);
                    leaf_lim = 2u << n;
                }
            } else if (LEAFCTR) {
                c |= ((1u << (31u - n)) - (nm1 - placed)) << n;
            }
        }
        if (v == 0u) c = kParked;         // nothing to search: park like a finished lane
    };

    if (!PERSISTENT) {
        const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (i < P.len) take(i);
    }

    for (;;) {
        // ---- scheduler visit: flush counters, retire finished lanes, refill.
        sum64 += sum32; sum32 = 0;
        if (STATS) { steps64 += steps32; steps32 = 0; }
        bool req_retire = false;          // serving: this lane retires an entry now
        uint32_t req_slot = 0u;
        uint64_t req_val = 0u;
        if (has_task && v == 0u) {
            const bool ok = sum64 != kCountInvalid;
            if (P.counts) P.counts[idx] = sum64;
            if (STATS) P.nodes[idx] = steps64;
            const uint32_t s = P.inst ? P.inst[idx] : 0u;
            const bool inst_ok = !P.inst || s < P.ninst;
            if (P.totals && ok && sum64 != 0) {
                const uint64_t w = P.weight ? (uint64_t)P.weight[idx] : 1u;
                if (!P.inst) {
                    const uint64_t add = w * sum64;
                    wtotal += add;
                    wtotal_hi += (wtotal < add) ? 1u : 0u;
                } else if (SERVE) {
                    req_val = w * sum64;          // serving: added per wave below
                } else {
                    // batches: a lane's consecutive entries mostly belong to one
                    // instance; add to its total when the instance changes
                    if (s != acc_s) {
                        if (acc_v) atomicAdd(&P.totals[acc_s], (unsigned long long)acc_v);
                        acc_s = s;
                        acc_v = 0;
                    }
                    acc_v += w * sum64;
                }
            }
            req_retire = SERVE && inst_ok;
            req_slot = s;
            has_task = false;
        }
        if (SERVE)
            retire_to_requests(held, P.remaining, P.totals, P.inst_gen, P.host_val, P.host_flag,
                               req_retire, req_slot, req_val, lane);
        if (PERSISTENT && !exhausted)
            refill_idle_lanes(qlo, qhi, claimed_all, exhausted, has_task, lane, P.head, P.len,
                              P.claim, take);
        if (!__any(v != 0u)) {
            if (exhausted && !__any(has_task)) break;
            continue;
        }

        // ---- DFS steps (Algorithm 2 with the Algorithm 3 last-row step).
        // The frame is kept as one 4-vector so that push and pop move it with
        // a single ds_write_b128 / ds_read_b128 and no register shuffling.
        u32x4 st = {c, l, r, v};
        // Steps run in chunks (64 steps in form 1, 32 in form 2).  After a
        // chunk a wave returns to the scheduler early when all its lanes have
        // finished (avail == 0 after a step) or, in persistent mode, once
        // `idle_min` of them have, so a finished lane waits for at most one
        // chunk instead of `refill_every` steps; a chunk's end check costs two
        // ballots, which 64-step chunks pay half as often as 32-step ones
        // (N = 20 at k = 9: 995 against 1004 ms; 16 steps: 1021, 128: 995,
        // 256: 1005).  The trip counts are wave-uniform; readfirstlane keeps
        // them in SGPRs.
        auto chunk_done = [&](uint32_t avail) {
            const uint32_t idle = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(avail == 0u));
            const uint32_t lanes = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(true));
            return idle == lanes ||
                   (PERSISTENT && P.idle_min && !exhausted && idle >= P.idle_min);
        };
        if (LOOP == 0) {
        for (uint32_t it = 0; it < P.refill_every; ++it) {
            const uint32_t p = st.w & (0u - st.w);    // lowest untried column
            st.w ^= p;
            // p is free in this frame, so OR and ADD agree on c, l and r.
            const uint32_t nc = LEAFCTR ? st.x + p + step_k : (st.x | p);
            const uint32_t nl = (st.y + p) << 1;
            const uint32_t nr = (st.z + p) >> 1;
            const uint32_t a = last & ~(nc | nl | nr); // free squares of the next row
            if (STATS) steps32 += (p != 0u);
            const bool leaf = LEAFCTR ? (int32_t)nc < 0 : __popc(nc) == nm1;
            const bool any = a != 0u;
            sum32 += (leaf && any) ? 1u : 0u;         // the last row has one column left
            const bool desc = any && !leaf;
            if (desc && st.w != 0u) {                 // keep the parent only if it has work
                top += 1024;
                *frame_at(top) = st;
            }
            st.x = desc ? nc : st.x;
            st.y = desc ? nl : st.y;
            st.z = desc ? nr : st.z;
            st.w = desc ? a : st.w;
            if (st.w == 0u) {                         // frame exhausted: pop
                st = *frame_at(top);
                top = max(top - 1024, floor);
            }
        }
        } else if (LOOP == 1) {
        // The lane masks live in SGPR pairs; the push, the selects, the pop
        // and the leaf count use them directly.
        uint32_t chunks = __builtin_amdgcn_readfirstlane((P.refill_every + 63u) / 64u);
        for (;;) {
            uint32_t trips = 64u;
            do {
                // p = lowest untried column; the untried set keeps its register.
                uint32_t p, rest = st.w;
                isa_take_lowest(rest, p);
                const uint32_t nc = LEAFCTR ? st.x + p + step_k : (st.x | p);
                const uint32_t nl = KINGS ? (p << 1) : (st.y + p) << 1;
                const uint32_t nr = KINGS ? (p >> 1) : (st.z + p) >> 1;
                const uint32_t a = last & ~(nc | nl | nr);
                if (STATS) steps32 += (p != 0u);
                const uint64_t leafm = __builtin_amdgcn_ballot_w64(
                    LEAFCTR ? (int32_t)nc < 0 : __popc(nc) == nm1);
                const uint64_t anym = __builtin_amdgcn_ballot_w64(a != 0u);
                const uint64_t restm = __builtin_amdgcn_ballot_w64(rest != 0u);
                const uint64_t descm = anym & ~leafm;
                isa_count(sum32, anym & leafm);
                st.w = rest;
                isa_push(st, top, descm & restm);
                st.x = isa_sel(descm, nc, st.x);
                st.y = isa_sel(descm, nl, st.y);
                st.z = isa_sel(descm, nr, st.z);
                st.w = isa_sel(descm, a, st.w);
                // After the select, avail == 0 exactly when the lane did not
                // descend (a descent has a != 0) and had no untried column left.
                isa_pop(st, top, floor, ~(descm | restm));
                trips = __builtin_amdgcn_readfirstlane(trips - 1u);
            } while (trips != 0u);
            chunks = __builtin_amdgcn_readfirstlane(chunks - 1u);
            if (chunks == 0u || chunk_done(st.w)) break;
        }
        } else if (LOOP == 3 || LOOP >= 6) {
        // Form 3: no selects.  Each step pushes the frame being expanded when
        // it still has an untried column, computes the child into the other
        // register frame, and pops when the child is not searched (no free
        // square, or a leaf): a descent leaves the child in place, and a dead
        // child or a leaf is replaced by the frame just pushed (or, when that
        // had nothing left, by the nearest ancestor with work).  Lanes pop
        // only while they had an untried column, so the stack pointer needs no
        // clamp.  The frame at row N-2 is pushed before its leaf children are
        // counted: one LDS frame more than form 1.  Two register frames
        // alternate (two steps per trip), so the child is written without
        // moves and can be computed while the parent is being pushed.
        //
        // Form 6 is form 3 with a push that needs no exec mask.  At the start
        // of a step a lane's stack holds at most the frames of the rows above
        // the one being expanded, so the slot above its top is free and inside
        // its column of the stack (the frame of row N-2, the deepest one
        // pushed, is popped in the step that pushes it): every lane writes its
        // frame there, and only the lanes with untried columns left advance
        // `top`.  A pop reads from `top + 1024` in those lanes (a select made
        // before the child is known) and from `top` in the others.  Two SALU
        // instructions fewer per step than form 3, one VALU instruction more;
        // the free squares are tested for zero directly (one compare instead
        // of the OR of their three sources and a compare), and a loop trip
        // runs four steps instead of two.
        //
        // Form 7 (the default) is form 6 without the sentinel slot: 1 KB of
        // LDS per wave less (10 instead of 11 KB at N = 20, depth 9: 16
        // resident waves per CU instead of 14).  A lane whose search ends
        // (no untried column left, the child not searched, the stack empty)
        // pops the slot above its empty stack, which holds the frame it has
        // just written (no untried column: the `max` below keeps the address
        // there), and a lane without an untried column takes every column as
        // occupied, so its children have no free square and it never pushes,
        // pops or counts again.  One select and one max per step more than
        // form 6.
        constexpr bool NOSENT = LOOP == 7;
        constexpr bool UPUSH = LOOP == 6 || LOOP == 7;
        auto step3 = [&](u32x4& A, u32x4& B) {
            uint32_t p, rest = A.w;
            uint64_t alive;
            isa_take_alive(rest, p, alive);           // the untried rest keeps A.w's register
            A.w = rest;
            const uint64_t restm = __builtin_amdgcn_ballot_w64(A.w != 0u);
            int32_t from = top;                       // forms 6 and 7: where a pop reads
            if (NOSENT) {
                // a lane without work computes a child with every column taken
                // (no free square), and a pop from an empty stack reads the
                // slot just written (its frame, with no untried column)
                A.x = isa_sel_u(alive, A.x, ~0u);
                from = isa_sel_i(restm, top + 1024, max(top, floor));
            } else if (UPUSH) {
                from = isa_sel_i(restm, top + 1024, top);
            }
            B.x = A.x + p;                            // p is free: + is |
            B.y = KINGS ? p << 1 : (A.y + p) << 1;
            B.z = KINGS ? p >> 1 : (A.z + p) >> 1;
            B.w = ~(B.x | B.y | B.z);                 // off-board columns are set in B.x
            const uint64_t leafm = __builtin_amdgcn_ballot_w64(
                LEAFCTR ? B.z < leaf_lim : __popc(B.x) == 31u);
            const uint64_t anym = UPUSH ? isa_nonzero(B.w) : __builtin_amdgcn_ballot_w64(B.w != 0u);
            if (STATS) isa_count(steps32, alive);
            isa_count(sum32, anym & leafm);
            if (UPUSH) isa_store_above(A, top); else isa_push(A, top, restm);
            isa_pop_free(B, UPUSH ? from : top, alive & ~(anym & ~leafm));
            if (UPUSH) top = from;
        };
        uint32_t chunks = __builtin_amdgcn_readfirstlane((P.refill_every + 63u) / 64u);
        u32x4 other;
        for (;;) {
            uint32_t trips = UPUSH ? 16u : 32u;       // 64 steps per chunk
            do {
                step3(st, other);
                step3(other, st);
                if (UPUSH) {                          // four steps per trip
                    step3(st, other);
                    step3(other, st);
                }
                trips = __builtin_amdgcn_readfirstlane(trips - 1u);
            } while (trips != 0u);
            chunks = __builtin_amdgcn_readfirstlane(chunks - 1u);
            if (chunks == 0u || chunk_done(st.w)) break;
        }
        } else if (LOOP == 4) {
        // The paper's loop as printed: the frame being expanded is the top
        // of the LDS stack, read at every step, with its untried set written
        // back; a child is pushed on top of it; an exhausted frame is popped
        // at the next step.  Registers carry no frame between scheduler
        // visits: a new entry is pushed when the lane enters, and the lane's
        // `v` is 1 while its stack holds a frame.
        if (st.w != 0u && top == floor) {
            top += 1024;
            *frame_at(top) = st;
        }
        for (uint32_t it = 0; it < P.refill_every; ++it) {
            const u32x4 f = *frame_at(top);
            const uint32_t p = f.w & (0u - f.w);
            if (p == 0u) {                            // exhausted (or the sentinel)
                top = max(top - 1024, floor);
            } else {
                *(word_at(top) + 3) = f.w ^ p;
                const uint32_t nc = LEAFCTR ? f.x + p + step_k : (f.x | p);
                const uint32_t nl = (f.y + p) << 1;
                const uint32_t nr = (f.z + p) >> 1;
                const uint32_t a = last & ~(nc | nl | nr);
                if (STATS) steps32 += 1u;
                const bool leaf = LEAFCTR ? (int32_t)nc < 0 : __popc(nc) == nm1;
                if (leaf) {
                    sum32 += (a != 0u) ? 1u : 0u;
                } else if (a != 0u) {
                    top += 1024;
                    *frame_at(top) = u32x4{nc, nl, nr, a};
                }
            }
        }
        st.w = (top != floor) ? 1u : 0u;
        } else if (LOOP == 5) {
        // Form 0 without the last-row step: a queen placed in row N-2 is a
        // frame like any other, and a solution is counted when the last row
        // gets its queen (the board is full).  Placements in the last row are
        // not DFS nodes (they are the solutions), so STATS leaves them out.
        for (uint32_t it = 0; it < P.refill_every; ++it) {
            const uint32_t p = st.w & (0u - st.w);
            st.w ^= p;
            const uint32_t nc = LEAFCTR ? st.x + p + step_k : (st.x | p);
            const uint32_t nl = (st.y + p) << 1;
            const uint32_t nr = (st.z + p) >> 1;
            const uint32_t a = last & ~(nc | nl | nr);
            const bool full = p != 0u && (nc & last) == last;
            if (STATS) steps32 += (p != 0u && !full);
            sum32 += full ? 1u : 0u;
            const bool desc = a != 0u;                // never on a full board
            if (desc && st.w != 0u) {
                top += 1024;
                *frame_at(top) = st;
            }
            st.x = desc ? nc : st.x;
            st.y = desc ? nl : st.y;
            st.z = desc ? nr : st.z;
            st.w = desc ? a : st.w;
            if (st.w == 0u) {
                st = *frame_at(top);
                top = max(top - 1024, floor);
            }
        }
        } else {
        // Form 2.  The frame keeps the untried set negated, w = -avail (mod
        // 2^32), so that two lane masks come out of carries instead of
        // compares: p = w & -w is the lowest untried column, and w + p =
        // -(avail - p) carries out exactly when that column was the last one;
        // the child's w = 0 - a borrows exactly when a != 0.  A parked lane has
        // w = 0: p = 0, no carry, no free square, so it neither pushes,
        // descends nor pops, and its stack pointer needs no clamp.
        uint32_t chunks = __builtin_amdgcn_readfirstlane((P.refill_every + 31u) / 32u);
        st.w = 0u - st.w;
        for (;;) {
            uint32_t trips = 32u;
            do {
                uint32_t w = st.w, p;
                uint64_t zm;
                isa_take_neg(w, p, zm);
                const uint32_t nc = LEAFCTR ? st.x + p + step_k : (st.x | p);
                const uint32_t nl = (st.y + p) << 1;
                const uint32_t nr = (st.z + p) >> 1;
                uint64_t anym;
                const uint32_t na = isa_neg_any(last & ~(nc | nl | nr), anym);
                if (STATS) steps32 += (p != 0u);
                const uint64_t leafm = __builtin_amdgcn_ballot_w64(
                    LEAFCTR ? (int32_t)nc < 0 : __popc(nc) == nm1);
                const uint64_t descm = anym & ~leafm;
                isa_count(sum32, anym & leafm);
                st.w = w;
                isa_step128(st, u32x4{nc, nl, nr, na}, top, descm & ~zm, descm,
                            zm & ~descm);
                trips = __builtin_amdgcn_readfirstlane(trips - 1u);
            } while (trips != 0u);
            chunks = __builtin_amdgcn_readfirstlane(chunks - 1u);
            if (chunks == 0u || chunk_done(st.w)) break;
        }
        st.w = 0u - st.w;
        }
        c = st.x; l = st.y; r = st.z; v = st.w;
    }

    if (SERVE) retire_flush(held, P.remaining, P.totals, P.inst_gen, P.host_val, P.host_flag, lane);
    if (!SERVE && P.totals && P.inst && acc_v)
        atomicAdd(&P.totals[acc_s], (unsigned long long)acc_v);
    if (P.totals && !P.inst) {
        // 128-bit wave sum (the high word holds the carries; it stays 0 unless
        // one wave's share exceeds 2^64, possible only for boards beyond 28)
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t lo = shfl_xor_u64(wtotal, off);
            wtotal_hi += shfl_xor_u64(wtotal_hi, off);
            wtotal += lo;
            wtotal_hi += (wtotal < lo) ? 1u : 0u;
        }
        if (lane == 0 && (wtotal | wtotal_hi) != 0) {
            const unsigned long long before =
                atomicAdd(&P.totals[0], (unsigned long long)wtotal);
            if (P.wide) {
                const uint64_t carry = wtotal_hi + ((before + wtotal < before) ? 1u : 0u);
                if (carry) atomicAdd(&P.totals[1], (unsigned long long)carry);
            }
        }
    }
}

__global__ void nq_slot_init_kernel(const SlotInit* recs, uint32_t count, uint32_t* inst_n,
                                    uint32_t* remaining, unsigned long long* totals,
                                    uint32_t* gen) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const SlotInit r = recs[i];
        inst_n[r.slot] = r.n;
        remaining[r.slot] = r.entries;
        totals[r.slot] = 0ull;
        gen[r.slot] = r.gen;
    }
}

__global__ void nq_zero_u64_kernel(unsigned long long* dst, uint64_t count) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = 0ull;
}

__global__ void nq_fill_u32_kernel(uint32_t* dst, uint32_t value, uint64_t count) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = value;
}

template <bool PERSISTENT, bool STATS, bool LEAFCTR, int LOOP, bool SERVE = false,
          bool KINGS = false>
static const void* kernel_ptr() {
    return reinterpret_cast<const void*>(
        &nq_dfs_kernel<PERSISTENT, STATS, LEAFCTR, LOOP, SERVE, KINGS>);
}

// The kings search: form 1 (with or without the row counter) or form 7 (the
// popcount leaf test only), no serving.
static const void* select_kings_kernel(int form, uint32_t mode, bool stats, bool leafctr) {
    if (form == 7) {
        if (leafctr) return nullptr;
        if (mode == NQ_MODE_PERSISTENT)
            return stats ? kernel_ptr<true, true, false, 7, false, true>()
                         : kernel_ptr<true, false, false, 7, false, true>();
        return stats ? kernel_ptr<false, true, false, 7, false, true>()
                     : kernel_ptr<false, false, false, 7, false, true>();
    }
    if (form != 1) return nullptr;
    if (mode == NQ_MODE_PERSISTENT) {
        if (stats)
            return leafctr ? kernel_ptr<true, true, true, 1, false, true>()
                           : kernel_ptr<true, true, false, 1, false, true>();
        return leafctr ? kernel_ptr<true, false, true, 1, false, true>()
                       : kernel_ptr<true, false, false, 1, false, true>();
    }
    if (stats)
        return leafctr ? kernel_ptr<false, true, true, 1, false, true>()
                       : kernel_ptr<false, true, false, 1, false, true>();
    return leafctr ? kernel_ptr<false, false, true, 1, false, true>()
                   : kernel_ptr<false, false, false, 1, false, true>();
}

// The kernel for a launch shape; serving launches exist only as persistent,
// no-statistics kernels, with the row counter except in form 3 (nullptr
// otherwise).
template <int LOOP>
static const void* select_kernel_loop(uint32_t mode, bool stats, bool leafctr, bool serve) {
    const bool pers = mode == NQ_MODE_PERSISTENT;
    if (serve) {
        if (!pers || stats) return nullptr;
        if (leafctr) return kernel_ptr<true, false, true, LOOP, true>();
        return (LOOP == 3 || LOOP >= 6) ? kernel_ptr<true, false, false, LOOP, true>() : nullptr;
    }
    if (pers) {
        if (stats)
            return leafctr ? kernel_ptr<true, true, true, LOOP>() : kernel_ptr<true, true, false, LOOP>();
        return leafctr ? kernel_ptr<true, false, true, LOOP>() : kernel_ptr<true, false, false, LOOP>();
    }
    if (stats)
        return leafctr ? kernel_ptr<false, true, true, LOOP>() : kernel_ptr<false, true, false, LOOP>();
    return leafctr ? kernel_ptr<false, false, true, LOOP>() : kernel_ptr<false, false, false, LOOP>();
}

// Inner-loop form of the launches planned from now on: NQ_DFS_LOOP=0..7 in the
// environment overrides the default, and set_loop_form (nq_set_loop_form) sets
// it at run time (for measurements of the forms against each other).
static std::atomic<int> g_loop_form{-1};

static int loop_form() {
    int f = g_loop_form.load(std::memory_order_relaxed);
    if (f >= 0) return f;
    const char* e = std::getenv("NQ_DFS_LOOP");
    f = kDefaultLoop;
    if (e && e[0] >= '0' && e[0] <= '7' && e[1] == 0) f = e[0] - '0';
    int expect = -1;
    g_loop_form.compare_exchange_strong(expect, f);
    return g_loop_form.load(std::memory_order_relaxed);
}

int set_loop_form(int form, int* previous) {
    if (form < -1 || form >= kLoopForms) return NQ_EINVAL;
    if (previous) *previous = loop_form();
    g_loop_form.store(form, std::memory_order_relaxed);   // -1: read again on next use
    return NQ_OK;
}

uint32_t default_claim(uint64_t len, const LaunchCfg& cfg) {
    static const long env = [] {
        const char* e = std::getenv("NQ_CLAIM");
        if (e && *e) {
            const long x = std::strtol(e, nullptr, 10);
            if (x >= 0 && x <= 4096) return x;
        }
        return -1l;
    }();
    if (env >= 0) return (uint32_t)env;
    // A block of up to 256 entries per atomic, but no more than 1/16 of a
    // wave's share of the frontier, so small launches still spread over every
    // resident wave (0 = each refill claims exactly its idle lanes).
    const uint64_t waves = (uint64_t)cfg.grid * (cfg.wg_size / 64u);
    return (uint32_t)std::min<uint64_t>(256, waves ? len / (waves * 16) : 0);
}

uint32_t default_idle_min() {
    static const uint32_t v = [] {
        const char* e = std::getenv("NQ_IDLE_MIN");
        if (e && *e) {
            const long x = std::strtol(e, nullptr, 10);
            if (x >= 0 && x <= 64) return (uint32_t)x;
        }
        return 4u;
    }();
    return v;
}

static const void* select_kernel(int form, uint32_t mode, bool stats, bool leafctr, bool serve,
                                 bool kings) {
    if (kings) return serve ? nullptr : select_kings_kernel(form, mode, stats, leafctr);
    switch (form) {
        case 0: return select_kernel_loop<0>(mode, stats, leafctr, serve);
        case 1: return select_kernel_loop<1>(mode, stats, leafctr, serve);
        case 2: return select_kernel_loop<2>(mode, stats, leafctr, serve);
        case 3: return select_kernel_loop<3>(mode, stats, leafctr, serve);
        case 4: return select_kernel_loop<4>(mode, stats, leafctr, serve);
        case 5: return select_kernel_loop<5>(mode, stats, leafctr, serve);
        case 6: return select_kernel_loop<6>(mode, stats, leafctr, serve);
        case 7: return select_kernel_loop<7>(mode, stats, leafctr, serve);
        default: return nullptr;
    }
}

int device_info(DeviceInfo* out) {
    static thread_local DeviceInfo cache[64];
    static thread_local bool have[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    if (dev >= 0 && dev < 64 && have[dev]) { *out = cache[dev]; return NQ_OK; }
    DeviceInfo d{};
    d.device = dev;
    int v = 0;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
        set_hip_error(e); return NQ_EDEVICE;
    }
    d.cu_count = v;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) !=
        hipSuccess) {
        set_hip_error(e); return NQ_EDEVICE;
    }
    d.lds_per_cu = v;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) !=
        hipSuccess) {
        set_hip_error(e); return NQ_EDEVICE;
    }
    d.lds_per_block = v;
    d.max_waves_per_cu = 32;
    if (dev >= 0 && dev < 64) { cache[dev] = d; have[dev] = true; }
    *out = d;
    return NQ_OK;
}

int plan_launch(const DeviceInfo& dev, uint32_t mode, uint32_t wg_size, uint32_t waves_per_cu,
                uint32_t frames, uint64_t len, bool stats, bool leafctr, LaunchCfg* cfg,
                bool serve, bool kings, uint32_t max_n) {
    if (mode != NQ_MODE_PLAIN && mode != NQ_MODE_PERSISTENT) return NQ_EINVAL;
    // the kings search runs form 1 when the queens run form 1, else form 7
    // with the popcount leaf test (its rd carries no marker)
    const int form = kings ? (loop_form() == 1 ? 1 : 7) : loop_form();
    // form 3's marker starts at bit 2n - 1 - placed = n + 1 + (frames of the
    // entry): it fits in 32 bits for every entry when max_n + frames <= 30
    if (form == 3 || form >= 6) leafctr = leafctr && max_n + frames <= 30u && !kings;
    frames += kFormExtraFrames[form];
    if (wg_size == 0) {
        // Plain: up to 4 waves per workgroup, as many as the LDS stacks allow.
        const uint64_t per_wave = 64ull * (frames + kFormSentinel[form]) * 16u;
        const uint64_t fit = per_wave ? (uint64_t)dev.lds_per_block / per_wave : 4;
        wg_size = (mode == NQ_MODE_PLAIN) ? 64u * (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4, fit))
                                          : 64u;
    }
    if (wg_size % 64u != 0 || wg_size > 1024u) return NQ_EINVAL;
    // The frames, and (all forms but 6) one sentinel frame per lane below them.
    const uint64_t lds = (uint64_t)wg_size * (frames + kFormSentinel[form]) * 16u;
    if (lds > (uint64_t)dev.lds_per_block) return NQ_EINVAL;
    cfg->mode = mode;
    cfg->wg_size = wg_size;
    cfg->lds_bytes = (uint32_t)lds;
    cfg->stats = stats;
    cfg->leafctr = leafctr;
    cfg->serve = serve;
    cfg->form = form;
    cfg->kings = kings;
    const void* fn = select_kernel(form, mode, stats, leafctr, serve, kings);
    if (!fn) return NQ_EINVAL;
    if (mode == NQ_MODE_PLAIN) {
        const uint64_t g = (len + wg_size - 1) / wg_size;
        if (g > 0x7fffffffull) return NQ_EINVAL;
        cfg->grid = (uint32_t)g;
        return NQ_OK;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, fn, (int)wg_size, (size_t)lds);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    if (per_cu < 1) return NQ_EINVAL;
    if (waves_per_cu) {
        const uint32_t want = std::max(1u, waves_per_cu / (wg_size / 64u));
        per_cu = std::min(per_cu, (int)want);
    }
    cfg->grid = (uint32_t)per_cu * (uint32_t)dev.cu_count;
    return NQ_OK;
}

int launch_zero_u64(unsigned long long* dst, uint64_t count, void* stream) {
    if (count == 0) return NQ_OK;
    const uint32_t block = 256;
    const uint64_t grid = (count + block - 1) / block;
    hipLaunchKernelGGL(nq_zero_u64_kernel, dim3((uint32_t)grid), dim3(block), 0,
                       (hipStream_t)stream, dst, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    return NQ_OK;
}

int launch_fill_u32(uint32_t* dst, uint32_t value, uint64_t count, void* stream) {
    if (count == 0) return NQ_OK;
    const uint32_t block = 256;
    const uint64_t grid = (count + block - 1) / block;
    if (grid > 0x7fffffffull) return NQ_EINVAL;
    hipLaunchKernelGGL(nq_fill_u32_kernel, dim3((uint32_t)grid), dim3(block), 0,
                       (hipStream_t)stream, dst, value, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    return NQ_OK;
}

int launch_slot_init(const SlotInit* recs, uint32_t count, uint32_t* inst_n, uint32_t* remaining,
                     unsigned long long* totals, uint32_t* gen, void* stream) {
    if (count == 0) return NQ_OK;
    const uint32_t block = 256;
    hipLaunchKernelGGL(nq_slot_init_kernel, dim3((count + block - 1) / block), dim3(block), 0,
                       (hipStream_t)stream, recs, count, inst_n, remaining, totals, gen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    return NQ_OK;
}

int launch_dfs(const LaunchCfg& cfg, const DfsParams& P, void* stream) {
    if (P.len == 0 || cfg.grid == 0) return NQ_OK;
    hipStream_t s = (hipStream_t)stream;
    // A serving launch (P.remaining set) needs a launch shape planned for it,
    // and the LDS planned must hold the stacks of the form it was planned for.
    if (cfg.serve != (P.remaining != nullptr)) return NQ_EINVAL;
    if (cfg.form < 0 || cfg.form >= kLoopForms) return NQ_EINVAL;
    const void* fn = select_kernel(cfg.form, cfg.mode, cfg.stats, cfg.leafctr, cfg.serve,
                                   cfg.kings);
    if (!fn) return NQ_EINVAL;
    DfsParams Q = P;
    Q.frames += kFormExtraFrames[cfg.form];
    if ((uint64_t)cfg.lds_bytes <
        (uint64_t)cfg.wg_size * (Q.frames + kFormSentinel[cfg.form]) * 16u)
        return NQ_EINVAL;
    if (cfg.mode == NQ_MODE_PERSISTENT) {
        int rc = launch_zero_u64(P.head, 1, stream);
        if (rc != NQ_OK) return rc;
    }
    const dim3 grid(cfg.grid), block(cfg.wg_size);
    void* args[] = {&Q};
    hipError_t le = hipLaunchKernel(fn, grid, block, args, cfg.lds_bytes, s);
    if (le != hipSuccess) { set_hip_error(le); return NQ_EDEVICE; }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    return NQ_OK;
}

}  // namespace nqi
