// The DFS kernels' parameters and launch shape: everything host code hands
// to nq_dfs_kernel.  Kept apart from the host-side declarations so that a
// record of the kernel's counters can name exactly the sources its code is
// built from.
#pragma once

#include <cstdint>

namespace nqi {

// Arguments of the DFS kernels (passed by value).
struct DfsParams {
    const uint32_t* cols;           // Somers triples, device
    const uint32_t* ld;
    const uint32_t* rd;
    const uint8_t* weight;          // nullable: weight 1
    const uint32_t* inst;           // nullable: every entry belongs to instance 0
    const uint32_t* inst_n;         // board size per instance (when inst != nullptr)
    uint64_t* counts;               // nullable: unweighted count per entry
    unsigned long long* totals;     // nullable: weighted total per instance (accumulated)
    uint64_t* nodes;                // stats kernels only: DFS steps per entry
    unsigned long long* head;       // persistent kernels: next unclaimed entry
    uint64_t len;                   // entries
    uint32_t n;                     // board size when inst == nullptr
    uint32_t frames;                // LDS stack frames per lane
    uint32_t refill_every;          // DFS steps between scheduler visits
    uint32_t reverse;               // persistent: claim entries from the last one down
    uint32_t wide;                  // totals[0..1] is one 128-bit total (low word first),
                                    // increased with carry (single-instance launches only)
    // Serving (all null / 0 otherwise).  Entries live in a ring: logical entry
    // i is physical (base + i) mod wrap.  The entries of one instance that a
    // wave retires together are added to totals[inst] and subtracted from
    // remaining[inst] at once; the subtraction that takes it to zero publishes
    // the instance's total to host-visible memory: host_val[inst] = total, then
    // host_flag[inst] = inst_gen[inst].
    uint64_t base;
    uint64_t wrap;
    uint32_t ninst;                 // instances (slots) when inst != nullptr: ids >= ninst
                                    // are never used to index (the entry is rejected)
    uint32_t idle_min;              // persistent: visit the scheduler early once this many
                                    // lanes of a wave are idle (0 = every refill_every steps)
    uint32_t claim;                 // persistent: entries a wave claims per atomic on head
                                    // (at least what its idle lanes need); the surplus is
                                    // handed out at the wave's later visits
    uint32_t* remaining;
    const uint32_t* inst_gen;
    unsigned long long* host_val;
    unsigned long long* host_flag;
};

// One request slot initialisation (serving): slot id, board size, entries,
// generation.  Applied by a kernel before the epoch that uses the slot.
struct SlotInit {
    uint32_t slot;
    uint32_t n;
    uint32_t entries;
    uint32_t gen;
};

// Count reported for an entry that needs more stack frames than the launch has.
constexpr uint64_t kCountInvalid = ~0ull;

struct LaunchCfg {
    uint32_t mode;          // NQ_MODE_PLAIN or NQ_MODE_PERSISTENT
    uint32_t wg_size;       // threads per workgroup
    uint32_t grid;          // workgroups
    uint32_t lds_bytes;     // dynamic LDS per workgroup
    bool stats;             // count DFS steps per entry
    bool leafctr;           // row counter in the high bits of cols (form 3: marker in rd)
    bool serve;             // serving epoch: per-request retirement (P.remaining set)
    int form;               // inner-loop form the launch was planned for
    bool kings;             // the kings search (NQ_FLAG_KINGS)
};

}  // namespace nqi
