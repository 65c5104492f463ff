// Third search on the lane-stack engine: the permanent of a 0/1 matrix,
// i.e. the number of permutations s of 0..n-1 with a[r][s(r)] = 1 for every
// row r, counted by a depth-first search over the rows.
//
// The paper's conclusion names combinatorial permutation problems among the
// searches its method carries over to (many subproblems, an iterative form
// with a stack, frames of more than one word).  This search differs from the
// queens in the two places that the conclusion leaves open:
//   * the frame is two words, (used columns, untried columns of the row being
//     filled), 8 bytes: the stack is the same lane-interleaved LDS layout with
//     an 8-byte slot, frame f of lane l of wave w at
//     ((w * (frames + 1) + f) * 64 + l) * 8, so a wave-wide ds_write_b64 /
//     ds_read_b64 touches 512 consecutive bytes whatever the lanes' depths;
//   * the leaf rule: the last two rows are never entered.  When the row about
//     to be filled is row n - 2, two columns x, y are left, and the lane adds
//     the completions in closed form, [a(n-2, x) a(n-1, y)] + [a(n-2, y)
//     a(n-1, x)] (0, 1 or 2), where the queens' last-row step adds one when
//     the last row has a free square.
// The next row's allowed columns depend on the row, which differs from lane
// to lane: the matrix's rows sit in LDS and a lane reads the word of its row
// (the row is the popcount of the used columns).
//
// Scheduling is the queens kernel's (nq_wave.h): plain launches take one
// entry per lane; persistent launches keep a resident grid whose waves visit
// a scheduler every `refill_every` steps (or once `idle_min` lanes are idle),
// retire finished lanes, and hand idle lanes entries by rank from a block
// claimed with one atomic add on a global head.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <new>
#include <vector>

#include "nq_internal.h"
#include "nq_trace.h"
#include "nq_wave.h"

namespace nqi {

namespace {

constexpr uint32_t kPermParked = 0xffffffffu;     // sentinel: all columns used, nothing untried
// Step 2 keeps the row of a frame's children in bits 27..31 of its used
// columns (boards have at most 20 columns, bits 20..26 stay zero), so that
// bits 25..31 are the byte offset of that row's allowed columns in a table
// of 32 rows, one per LDS bank.  Its sentinel has every column used and row
// 31; the row of a parked lane's child wraps through 0..31, all inside the
// table, and a parked lane reading row r reads the word of the live lanes
// at row r (a 64-row table put rows r and r + 32 in one bank: 1.5 % of the
// LDS instructions conflicted).
constexpr uint32_t kPermRowShift = 27;
constexpr uint32_t kPermRowOne = 1u << kPermRowShift;
constexpr uint32_t kPermParked2 = 0xf80fffffu;
constexpr uint32_t kPermTableRows = 34;
constexpr uint32_t kPermFrameBytes = 8;

struct PermParams {
    const uint32_t* cols;        // used columns of each entry (device)
    uint64_t* counts;            // nullable: count per entry
    unsigned long long* total;   // nullable: accumulated total
    uint64_t* nodes;             // stats kernels: DFS steps per entry
    unsigned long long* head;    // persistent kernels: next unclaimed entry
    uint64_t len;
    uint32_t n;
    uint32_t frames;             // LDS frames per lane
    uint32_t refill_every;
    uint32_t idle_min;
    uint32_t claim;
    uint32_t rows[32];           // row r's allowed columns (bit c)
};

// A frame: (used columns, untried columns), one 8-byte LDS slot.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u32x2 lds_frame2;

__device__ __forceinline__ lds_frame2* frame2_at(int32_t addr) {
    return (lds_frame2*)(uintptr_t)(uint32_t)addr;
}

// Completions of the last two rows when `left` holds the two unused columns
// {x, y} and ra, rb are the allowed columns of rows n-2 and n-1: the number
// of ways to give x and y to the two rows, [x in ra][y in rb] + [y in ra][x
// in rb] = popc(A & swap(B)) with A = ra & left, B = rb & left, where swap
// exchanges x and y: B itself when it holds both or neither, else left ^ B.
__device__ __forceinline__ uint32_t two_rows(uint32_t left, uint32_t ra, uint32_t rb) {
    const uint32_t a = ra & left, b = rb & left;
    const uint32_t swapped = (__popc(b) == 1u) ? (b ^ left) : b;
    return __popc(a & swapped);
}

// The hand-scheduled step (STEP 1) moves frames with these blocks; each one
// that switches exec declares SCC clobbered (its SALU instructions write it).

// p = lowest untried column of w, w loses it (in place), alive = lanes whose w
// was not empty (the borrow of 0 - w).
__device__ __forceinline__ void perm_take(uint32_t& w, uint32_t& p, uint64_t& alive) {
    uint32_t neg;
    asm("v_sub_co_u32 %[n], %[al], 0, %[w]\n\t"
        "v_and_b32 %[p], %[w], %[n]\n\t"
        "v_xor_b32 %[w], %[w], %[p]"
        : [w] "+v"(w), [p] "=&v"(p), [n] "=&v"(neg), [al] "=&s"(alive));
}

// Lanes with a != 0 (one compare).
__device__ __forceinline__ uint64_t perm_nonzero(uint32_t a) {
    uint64_t m;
    asm("v_cmp_ne_u32 %0, 0, %1" : "=s"(m) : "v"(a));
    return m;
}

// m ? a : d per lane.
__device__ __forceinline__ int32_t perm_sel(uint64_t m, int32_t a, int32_t d) {
    int32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(d), "v"(a), "s"(m));
    return r;
}

// a + b + c in one instruction (the compiler splits it otherwise).
__device__ __forceinline__ uint32_t perm_add3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// Every lane writes its frame to the slot above its stack top (free space in
// the lanes that do not push).  No exec mask.
__device__ __forceinline__ void perm_store_above(u32x2 f, int32_t top) {
    asm volatile("ds_write_b64 %[top], %[f] offset:512" : : [top] "v"(top), [f] "v"(f) : "memory");
}

// Pop for the lanes in m: frame <- [from], from -= one slot; waited for.
__device__ __forceinline__ void perm_pop(u32x2& f, int32_t& from, uint64_t m) {
    uint64_t sv;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m]\n\t"
        "ds_read_b64 %[f], %[from]\n\t"
        "v_add_u32 %[from], 0xfffffe00, %[from]\n\t"
        "s_mov_b64 exec, %[sv]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [f] "+v"(f), [from] "+v"(from), [sv] "=&s"(sv)
        : [m] "s"(m)
        : "memory", "scc");
}

// For the lanes in m, sum += the completions of the last two rows (two_rows
// below): B = rb & left; swapped = left ^ B when B holds one of the two
// columns, else B; sum += popc(ra & swapped) (swapped lies inside left).
__device__ __forceinline__ void perm_leaf(uint32_t& sum, uint32_t left, uint32_t ra,
                                          uint32_t rb, uint64_t m) {
    uint64_t sv;
    uint32_t b, t, u;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m]\n\t"
        "v_and_b32 %[b], %[rb], %[left]\n\t"
        "v_bcnt_u32_b32 %[t], %[b], 0\n\t"
        "v_cmp_eq_u32 vcc, 1, %[t]\n\t"
        "v_cndmask_b32 %[u], 0, %[left], vcc\n\t"
        "v_bitop3_b32 %[t], %[u], %[ra], %[b] bitop3:0x48\n\t"   // ra & (u ^ b)
        "v_bcnt_u32_b32 %[sum], %[t], %[sum]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [sum] "+v"(sum), [sv] "=&s"(sv), [b] "=&v"(b), [t] "=&v"(t), [u] "=&v"(u)
        : [m] "s"(m), [left] "v"(left), [ra] "v"(ra), [rb] "v"(rb)
        : "vcc", "scc");
}

// STEP selects the inner loop: 0 = the step in plain C++ (the compiler places
// the exec masks and selects), 1 = hand-scheduled (the default): two register
// frames alternate, the child is computed into the other one, every lane
// writes its frame to the free slot above its stack (the lanes with an
// untried column left advance the stack pointer), and a lane whose child is
// not searched (no allowed column, or the last two rows reached) pops, which
// returns the frame just written when it had an untried column left; the
// next row's allowed columns are read from LDS before the child is known (the
// child's row is one more than the frame's), and the last two rows'
// completions are counted under an exec mask.  Step 2 (the default) is step
// 1 with the children's row carried in the high bits of the used columns
// (kPermRowShift): the row's allowed columns are read at that byte offset
// and the leaf test compares the word, where step 1 counts the used columns
// twice (for the address and for the test).  Steps 1 and 2 need one frame
// more per lane (the frame of row n - 3 is written before its leaves are
// counted).
template <bool PERSISTENT, bool STATS, int STEP>
__global__ __launch_bounds__(1024) void nq_perm_kernel(PermParams P) {
    constexpr uint32_t extra = STEP >= 1 ? 1u : 0u;
    constexpr uint32_t parked = STEP == 2 ? kPermParked2 : kPermParked;
    extern __shared__ u32x2 perm_stack[];
    // the matrix's rows, then rows that allow nothing: rows 32 and 33 are the
    // "next row" of a parked lane in steps 0 and 1 (its used set has all 32
    // bits), any of rows 0..31 that of a parked lane in step 2
    __shared__ uint32_t mrows[kPermTableRows];
    if (threadIdx.x < kPermTableRows)
        mrows[threadIdx.x] = threadIdx.x < P.n ? P.rows[threadIdx.x] : 0u;
    __syncthreads();
    const uint32_t lds = (uint32_t)(uintptr_t)(lds_frame2*)perm_stack;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    // Stack addresses are signed: LDS offsets are far below 2^31, and popping
    // the sentinel computes floor - stride, which max() takes back to floor.
    const int32_t floor =
        (int32_t)(lds + ((wave * (P.frames + 1u)) * 64u + lane) * kPermFrameBytes);
    const int32_t stride = (int32_t)(64u * kPermFrameBytes);
    const uint32_t n = P.n;
    const uint32_t board = (n >= 32u) ? 0xffffffffu : ((1u << n) - 1u);
    // the last two rows' allowed columns (wave-uniform)
    const uint32_t ra = n >= 2u ? mrows[n - 2u] : 0u, rb = mrows[(n - 1u) & 31u];
    const uint32_t leaf_row = n - 2u;     // reached with the last two rows left (n >= 3)
    int32_t top = floor;
    *frame2_at(floor) = u32x2{parked, 0u};

    uint32_t c = parked, v = 0u;
    uint64_t idx = 0, sum = 0, steps = 0, wtotal = 0;
    uint32_t sum32 = 0;                   // leaves since the last scheduler visit
    bool has_task = false;
    bool exhausted = !PERSISTENT;
    bool claimed_all = false;
    uint64_t qlo = 0, qhi = 0;

    // Takes entry i: its used columns, the sentinel, and the cases that need
    // no search (at most two rows left, or a row with no allowed column).
    auto take = [&](uint64_t i) {
        idx = i;
        has_task = true;
        top = floor;
        sum = 0;
        steps = 0;
        *frame2_at(floor) = u32x2{parked, 0u};
        c = P.cols[i] & board;
        v = 0u;
        const uint32_t placed = __popc(c);
        if (placed >= n) {
            sum = 1;                                   // a complete permutation
        } else if (placed + 1u == n) {
            sum = __popc(rb & ~c & board);             // the last row
        } else if (placed + 2u == n) {
            sum = two_rows(~c & board, ra, rb);        // the last two rows
        } else if (n - 3u - placed > P.frames - extra) {
            sum = kCountInvalid;                       // does not fit this launch's stack
        } else {
            v = mrows[placed] & ~c & board;
            if (STEP == 2) c |= (placed + 1u) << kPermRowShift;   // the children's row
        }
        if (v == 0u) c = parked;
    };

    if (!PERSISTENT) {
        const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (i < P.len) take(i);
    }

    for (;;) {
        // ---- scheduler visit: retire finished lanes, refill idle ones.
        sum += sum32;                     // at most 2 per step: no 32-bit overflow
        sum32 = 0;
        if (has_task && v == 0u) {
            if (P.counts) P.counts[idx] = sum;
            if (STATS) P.nodes[idx] = steps;
            if (sum != kCountInvalid) wtotal += sum;
            has_task = false;
        }
        if (PERSISTENT && !exhausted)
            refill_idle_lanes(qlo, qhi, claimed_all, exhausted, has_task, lane, P.head, P.len,
                              P.claim, take);
        if (!__any(v != 0u)) {
            if (exhausted && !__any(has_task)) break;
            continue;
        }
        // ---- DFS steps: place the lowest untried column of the current row.
        // A parked lane (sentinel popped) has every column used and nothing
        // untried: p = 0, its "next row" is 32 (33 in step 1; in step 2 one
        // of rows 0..31, one more each step), which gives it no unused
        // allowed column, so no descent (and no count: it is not
        // alive); in step 0 its pops read the sentinel again (top stays at
        // floor), in steps 1 and 2 it does not pop.  A board of n <= 2 never
        // gets here (its entries are settled when taken), so leaf_row never
        // wraps into use.
        if (STEP >= 1) {
            const uint32_t leaf_word = leaf_row << kPermRowShift;   // step 2's leaf test
            auto step = [&](u32x2& A, u32x2& B) {
                const uint32_t row = STEP == 2 ? 0u : __popc(A.x) + 1u;   // the child's row
                const uint32_t mrow =
                    STEP == 2 ? *reinterpret_cast<const uint32_t*>(
                                    reinterpret_cast<const char*>(mrows) + (A.x >> 25))
                              : mrows[row];
                uint32_t p, rest = A.y;
                uint64_t alive;
                perm_take(rest, p, alive);
                A.y = rest;
                const uint64_t restm = __builtin_amdgcn_ballot_w64(rest != 0u);
                int32_t from = perm_sel(restm, top + stride, top);   // where a pop reads
                // p is unused, so + is |; step 2 computes the unused and the
                // allowed unused columns from A.x and p, off the add's path
                B.x = STEP == 2 ? perm_add3(A.x, p, kPermRowOne) : (A.x | p);
                const uint32_t left = STEP == 2 ? board & ~(A.x | p) : board & ~B.x;
                B.y = STEP == 2 ? mrow & ~(A.x | p) : mrow & left;   // a row lies in the board
                // step 2: a live frame's children are at most at the leaf row
                const uint64_t leafm = __builtin_amdgcn_ballot_w64(
                    STEP == 2 ? A.x >= leaf_word : row == leaf_row);
                const uint64_t anym = perm_nonzero(B.y);
                if (STATS) steps += (p != 0u) ? 1u : 0u;
                perm_leaf(sum32, left, ra, rb, leafm & alive);
                perm_store_above(A, top);
                perm_pop(B, from, alive & ~(anym & ~leafm));
                top = from;
            };
            u32x2 st = {c, v}, other;
            for (uint32_t it = 0; it < P.refill_every; it += 32u) {
                for (int s = 0; s < 8; ++s) {
                    step(st, other);
                    step(other, st);
                    step(st, other);
                    step(other, st);
                }
                const uint64_t idle = __ballot(st.y == 0u);
                const uint32_t lanes = (uint32_t)__popcll(__ballot(true));
                const uint32_t nidle = (uint32_t)__popcll(idle);
                if (nidle == lanes || (PERSISTENT && !exhausted && nidle >= P.idle_min)) break;
            }
            c = st.x;
            v = st.y;
            continue;
        }
        for (uint32_t it = 0; it < P.refill_every; it += 32u) {
            for (int s = 0; s < 32; ++s) {
                const uint32_t p = v & (0u - v);
                v ^= p;
                const uint32_t nc = c | p;
                const uint32_t row = __popc(nc);       // the row to fill next (32: parked)
                const uint32_t left = ~nc & board;     // unused columns
                const uint32_t a = mrows[row] & left;
                const bool leaf = row == leaf_row;     // the last two rows are left
                if (STATS) steps += (p != 0u) ? 1u : 0u;
                if (leaf && p != 0u) sum32 += two_rows(left, ra, rb);
                const bool desc = a != 0u && !leaf;
                if (desc && v != 0u) {                 // keep the frame if it has work
                    top += stride;
                    *frame2_at(top) = u32x2{c, v};
                }
                c = desc ? nc : c;
                v = desc ? a : v;
                if (v == 0u) {                         // exhausted: pop
                    const u32x2 f = *frame2_at(top);
                    c = f.x;
                    v = f.y;
                    // unsigned addresses: never step below the sentinel
                    top = max(top - stride, floor);
                }
            }
            const uint64_t idle = __ballot(v == 0u);
            const uint32_t lanes = (uint32_t)__popcll(__ballot(true));
            const uint32_t nidle = (uint32_t)__popcll(idle);
            if (nidle == lanes || (PERSISTENT && !exhausted && nidle >= P.idle_min)) break;
        }
    }
    if (P.total) {
        for (int off = 32; off > 0; off >>= 1) wtotal += shfl_xor_u64(wtotal, off);
        if (lane == 0 && wtotal != 0) atomicAdd(P.total, (unsigned long long)wtotal);
    }
}

template <int STEP>
const void* perm_kernel_step(bool persistent, bool stats) {
    if (persistent)
        return stats ? reinterpret_cast<const void*>(&nq_perm_kernel<true, true, STEP>)
                     : reinterpret_cast<const void*>(&nq_perm_kernel<true, false, STEP>);
    return stats ? reinterpret_cast<const void*>(&nq_perm_kernel<false, true, STEP>)
                 : reinterpret_cast<const void*>(&nq_perm_kernel<false, false, STEP>);
}

// The inner loop of the launches from now on: NQ_PERM_STEP=0 or 1 in the
// environment selects the plain C++ step or the hand-scheduled step without
// the row field (for measurement), otherwise step 2; nq_perm_set_step sets it
// at run time.
std::atomic<int> g_perm_step{-1};

int perm_step() {
    int st = g_perm_step.load(std::memory_order_relaxed);
    if (st >= 0) return st;
    const char* e = std::getenv("NQ_PERM_STEP");
    st = (e && (e[0] == '0' || e[0] == '1') && e[1] == 0) ? e[0] - '0' : 2;
    int expect = -1;
    g_perm_step.compare_exchange_strong(expect, st);
    return g_perm_step.load(std::memory_order_relaxed);
}

const void* perm_kernel(bool persistent, bool stats, int step) {
    return step == 2   ? perm_kernel_step<2>(persistent, stats)
           : step == 1 ? perm_kernel_step<1>(persistent, stats)
                       : perm_kernel_step<0>(persistent, stats);
}

// Rows of an n x n matrix: every bit is a column of the board.
bool rows_ok(uint32_t n, const uint32_t* rows) {
    if (n < 1 || n > NQ_PERM_MAX_N || !rows) return false;
    const uint32_t board = (1u << n) - 1u;
    for (uint32_t r = 0; r < n; ++r)
        if (rows[r] & ~board) return false;
    return true;
}

// Depth-first enumeration of the prefixes of length `depth`, lexicographic
// (row 0's column ascending, then row 1's, ...).
struct PermFrontier {
    uint32_t n, depth;
    const uint32_t* rows;
    uint32_t* out;
    uint64_t cap, len;
    void walk(uint32_t row, uint32_t used) {
        if (row == depth) {
            if (out && len < cap) out[len] = used;
            ++len;
            return;
        }
        uint32_t a = rows[row] & ~used;
        while (a) {
            const uint32_t p = a & (0u - a);
            a ^= p;
            walk(row + 1, used | p);
        }
    }
};

// The automatic depth: the shallowest with at least 2^20 entries, at most
// n - 2 and with at most 2^26 entries (the frontier is built on the host).
uint32_t perm_auto_depth(uint32_t n, const uint32_t* rows) {
    if (n <= 2) return n;
    uint32_t best = 1;
    for (uint32_t d = 1; d + 2 <= n; ++d) {
        PermFrontier f{n, d, rows, nullptr, 0, 0};
        f.walk(0, 0u);
        if (f.len > (1ull << 26)) break;
        best = d;
        if (f.len >= (1ull << 20)) break;
    }
    return best;
}

int perm_run(uint32_t n, const uint32_t* rows, const uint32_t* d_cols, uint64_t len,
             uint32_t depth, uint64_t* d_counts, unsigned long long* d_total,
             const nq_opts* opts) {
    if (len == 0) {
        if (opts && opts->kernel_ms_out) *opts->kernel_ms_out = 0.0;
        return NQ_OK;
    }
    const uint32_t mode = (opts && opts->mode) ? opts->mode : (uint32_t)NQ_MODE_PERSISTENT;
    if (mode != NQ_MODE_PLAIN && mode != NQ_MODE_PERSISTENT) return NQ_EINVAL;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    // frames for rows depth..n-4 (the current frame is in registers and the
    // last two rows are never entered), plus steps 1 and 2's frame of row n - 3
    const int step = perm_step();
    const uint32_t frames = std::max<uint32_t>(1, n >= depth + 3u ? n - 3u - depth : 0u) +
                            (step >= 1 ? 1u : 0u);
    uint32_t wg = opts && opts->wg_size ? opts->wg_size : 64u;
    if (wg % 64u != 0 || wg > 1024u) return NQ_EINVAL;
    const uint64_t lds = (uint64_t)wg * (frames + 1u) * kPermFrameBytes;
    if (lds + kPermTableRows * 4u > (uint64_t)dev.lds_per_block) return NQ_EINVAL;   // + the matrix
    const bool stats = opts && opts->d_nodes;
    const void* fn = perm_kernel(mode == NQ_MODE_PERSISTENT, stats, step);
    uint32_t grid = 0;
    if (mode == NQ_MODE_PLAIN) {
        const uint64_t g = (len + wg - 1) / wg;
        if (g > 0x7fffffffull) return NQ_EINVAL;
        grid = (uint32_t)g;
    } else {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)wg,
                                                                    (size_t)lds);
        if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
        if (per_cu < 1) return NQ_EINVAL;
        if (opts && opts->waves_per_cu)
            per_cu = std::min(per_cu, (int)std::max(1u, opts->waves_per_cu / (wg / 64u)));
        grid = (uint32_t)per_cu * (uint32_t)dev.cu_count;
    }
    PermParams P{};
    P.cols = d_cols;
    P.counts = d_counts;
    P.total = d_total;
    P.nodes = stats ? opts->d_nodes : nullptr;
    P.len = len;
    P.n = n;
    P.frames = frames;
    // a lane adds at most two leaves per step to its 32-bit count between
    // scheduler visits, so the visits stay well under 2^31 steps apart
    P.refill_every = (opts && opts->refill_every) ? std::min(opts->refill_every, 1u << 30) : 512u;
    P.idle_min = default_idle_min();
    {
        const uint64_t waves = (uint64_t)grid * (wg / 64u);
        P.claim = (opts && opts->claim) ? opts->claim
                                        : (uint32_t)std::min<uint64_t>(256, len / (waves * 16));
    }
    for (uint32_t r = 0; r < n; ++r) P.rows[r] = rows[r];
    hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
    hipError_t e;
    unsigned long long* head = nullptr;
    if (mode == NQ_MODE_PERSISTENT) {
        if ((e = hipMallocAsync((void**)&head, 8, s)) != hipSuccess) {
            set_hip_error(e);
            return NQ_EDEVICE;
        }
        rc = launch_zero_u64(head, 1, s);
    }
    P.head = head;
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = opts && opts->kernel_ms_out;
    if (rc == NQ_OK && timed) {
        if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess ||
            (e = hipEventRecord(a, s)) != hipSuccess) {
            set_hip_error(e);
            rc = NQ_EDEVICE;
        }
    }
    if (rc == NQ_OK) {
        void* args[] = {&P};
        e = hipLaunchKernel(fn, dim3(grid), dim3(wg), args, (size_t)lds, s);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) { set_hip_error(e); rc = NQ_EDEVICE; }
    }
    if (rc == NQ_OK && timed) {
        float f = 0.f;
        if ((e = hipEventRecord(b, s)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
            (e = hipEventElapsedTime(&f, a, b)) != hipSuccess) {
            set_hip_error(e);
            rc = NQ_EDEVICE;
        } else {
            *opts->kernel_ms_out = f;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (head) {
        e = hipFreeAsync(head, s);
        if (e != hipSuccess && rc == NQ_OK) { set_hip_error(e); rc = NQ_EDEVICE; }
    }
    return rc;
}

}  // namespace

}  // namespace nqi

using namespace nqi;

extern "C" int nq_perm_set_step(int step, int* previous) {
    if (step < -1 || step > 2) return NQ_EINVAL;
    if (previous) *previous = nqi::perm_step();
    nqi::g_perm_step.store(step, std::memory_order_relaxed);   // -1: read again on next use
    return NQ_OK;
}

extern "C" int nq_perm_frontier(uint32_t n, const uint32_t* rows, uint32_t depth, uint32_t* cols,
                                uint64_t capacity, uint64_t* out_len) {
    if (!rows_ok(n, rows) || depth > n || !out_len) return NQ_EINVAL;
    try {
        const bool fill = cols != nullptr && capacity != 0;   // else a size query
        PermFrontier f{n, depth, rows, fill ? cols : nullptr, fill ? capacity : 0, 0};
        f.walk(0, 0u);
        *out_len = f.len;
        return (fill && f.len > capacity) ? NQ_ERANGE : NQ_OK;
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_perm_count_subproblems(uint32_t n, const uint32_t* rows, const uint32_t* d_cols,
                                         uint64_t len, uint32_t depth, uint64_t* d_counts,
                                         unsigned long long* d_total, const nq_opts* opts) {
    if (!rows_ok(n, rows) || depth > n || (len > 0 && !d_cols)) return NQ_EINVAL;
    if (opts && opts->flags != 0) return NQ_EINVAL;
    try {
        TraceRange t("perm dfs");
        return perm_run(n, rows, d_cols, len, depth, d_counts, d_total, opts);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_perm_count(uint32_t n, const uint32_t* rows, const nq_opts* opts,
                             uint64_t* out_total) {
    if (!rows_ok(n, rows) || !out_total) return NQ_EINVAL;
    if (opts && (opts->flags != 0 || opts->counts_out || opts->d_nodes)) return NQ_EINVAL;
    const uint32_t depth = (opts && opts->depth) ? opts->depth : perm_auto_depth(n, rows);
    if (depth > n) return NQ_EINVAL;
    try {
        TraceRange whole("nq_perm_count");
        PermFrontier f{n, depth, rows, nullptr, 0, 0};
        f.walk(0, 0u);
        std::vector<uint32_t> h(f.len);
        f.out = h.data();
        f.cap = f.len;
        f.len = 0;
        f.walk(0, 0u);
        hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
        uint32_t* d_cols = nullptr;
        unsigned long long* d_total = nullptr;
        hipError_t e;
        const size_t bytes = ((h.size() * 4 + 255) / 256) * 256 + 256;
        if ((e = hipMalloc((void**)&d_cols, bytes)) != hipSuccess) {
            set_hip_error(e);
            return e == hipErrorOutOfMemory ? NQ_ENOMEM : NQ_EDEVICE;
        }
        d_total = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(d_cols) + bytes - 256);
        int rc = NQ_OK;
        if (!h.empty() && (e = hipMemcpyAsync(d_cols, h.data(), h.size() * 4,
                                              hipMemcpyHostToDevice, s)) != hipSuccess) {
            set_hip_error(e);
            rc = NQ_EDEVICE;
        }
        if (rc == NQ_OK) rc = launch_zero_u64(d_total, 1, s);
        if (rc == NQ_OK) rc = perm_run(n, rows, d_cols, h.size(), depth, nullptr, d_total, opts);
        unsigned long long t = 0;
        if (rc == NQ_OK) {
            if ((e = hipMemcpyAsync(&t, d_total, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess) {
                set_hip_error(e);
                rc = NQ_EDEVICE;
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(d_cols);
        if (rc != NQ_OK) return rc;
        *out_total = t;
        return NQ_OK;
    } catch (const std::bad_alloc&) {
        return NQ_ENOMEM;
    } catch (...) {
        return NQ_EINVAL;
    }
}
