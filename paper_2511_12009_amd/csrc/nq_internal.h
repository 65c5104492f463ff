// Internal declarations shared by the host-side translation units of libnq.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/nq.h"
#include "nq_kernel.h"

namespace nqi {

// One starting point of the frontier enumeration: the Somers triple after the
// first `row` rows, the rows still to place before the frontier depth, the
// weight every entry below it carries, its row-0 column, and the search (the
// kings search keeps only the last king's neighbours in ld / rd).
struct Root {
    uint32_t cols, ld, rd;
    int row;
    int rows_left;
    uint8_t weight;
    uint32_t first_col;
    bool kings;
};

std::vector<Root> frontier_roots(uint32_t n, uint32_t depth, bool kings = false);
uint64_t root_size(uint32_t n, const Root& rt);
std::vector<uint64_t> root_offsets(uint32_t n, const std::vector<Root>& roots);

// nq_frontier's body.  `first_row_offsets`, when set, receives the start of
// each row-0 column's run of entries followed by the total.
int frontier_fill(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld, uint32_t* rd,
                  uint8_t* weight, uint64_t capacity, uint64_t* out_len,
                  std::vector<uint64_t>* first_row_offsets, bool kings = false);

// Sets the inner-loop form of the DFS launches planned from now on (-1 = the
// default); *previous (nullable) receives the form in use.  NQ_EINVAL for an
// unknown form.
int set_loop_form(int form, int* previous);

// True when the row-counter form of the leaf test holds for every entry of an
// n board with at least `min_placed` queens placed: the counter needs
// n - 1 - placed <= 2^(31 - n).
inline bool leafctr_ok(uint32_t n, uint32_t min_placed) {
    if (n > 30) return false;
    const uint32_t rows = (n > min_placed + 1) ? n - 1 - min_placed : 0u;
    return rows <= (1u << (31u - n));
}

// Device properties used for launch shapes.
struct DeviceInfo {
    int device;
    int cu_count;
    int lds_per_cu;
    int lds_per_block;
    int max_waves_per_cu;
};

int device_info(DeviceInfo* out);

// Fills `cfg` for `len` entries of boards of at most `max_n` columns needing
// `frames` frames per lane (before the extra frames of the inner-loop form);
// `leafctr` says whether form 1's row counter fits every entry, and the
// launch uses the row counter (or form 3's marker) only where it fits;
// `serve` plans a serving epoch (persistent, no statistics), `kings` a launch
// of the kings search (inner-loop form 1).
int plan_launch(const DeviceInfo& dev, uint32_t mode, uint32_t wg_size, uint32_t waves_per_cu,
                uint32_t frames, uint64_t len, bool stats, bool leafctr, LaunchCfg* cfg,
                bool serve = false, bool kings = false, uint32_t max_n = NQ_MAX_N_WIDE);

// Enqueues the DFS kernel (and, for the persistent mode, the zeroing of
// *P.head) on `stream`.  Returns NQ_OK or NQ_EDEVICE.
int launch_dfs(const LaunchCfg& cfg, const DfsParams& P, void* stream);

// Enqueues the slot initialisations recs[0..count) (device array) on `stream`:
// inst_n[slot] = n, remaining[slot] = entries, totals[slot] = 0, gen[slot] = gen.
int launch_slot_init(const SlotInit* recs, uint32_t count, uint32_t* inst_n, uint32_t* remaining,
                     unsigned long long* totals, uint32_t* gen, void* stream);

// Enqueues dst[0..count) = 0 with a kernel (no memset node in captured graphs).
int launch_zero_u64(unsigned long long* dst, uint64_t count, void* stream);
// Enqueues dst[0..count) = value with a kernel.
int launch_fill_u32(uint32_t* dst, uint32_t value, uint64_t count, void* stream);

// Device frontier expansion (nq_expand.hip): scratch size for `len` parents,
// and the expansion itself; *out_len gets the child count (the call waits on
// the stream for it).  With null outputs only the size is computed; the scan
// offsets stay in the scratch at uint64 index len + 1 + i.
size_t expand_scratch_bytes(uint64_t len);
int expand_device(uint32_t n, uint32_t rows, const uint32_t* cols, const uint32_t* ld,
                  const uint32_t* rd, const uint8_t* w, uint64_t len, uint32_t* ocols,
                  uint32_t* old, uint32_t* ord, uint8_t* ow, uint64_t cap, uint64_t* out_len,
                  void* scratch, void* stream);

// Tuning results remembered for this process (nq_autotune), by device and n.
int tune_lookup(uint32_t n, nq_tuned* out);

// Chunked counts: chunk i of `chunks` is the range [F*i/chunks, F*(i+1)/chunks)
// of the host frontier of depth kChunkHostDepth (F entries), deepened on the
// device to the count's depth.
constexpr uint32_t kChunkHostDepth = 5;
// Boards whose automatic count runs in chunks, with the measured plan.
struct ChunkPlan { uint32_t n, depth, chunks; };
const ChunkPlan* chunk_plan(uint32_t n);   // nullptr: the whole frontier
// Counts chunk `index` of `chunks` at `depth` (persistent launch, launch
// fields of opts) and reports its wall time (host frontier, expansion, DFS,
// result) and weighted count.
int time_chunk(uint32_t n, uint32_t depth, uint32_t chunks, uint32_t index, const nq_opts& opts,
               double* ms, unsigned __int128* total);

// Lanes of a persistent wave that must be idle before it visits the scheduler
// between chunks of steps (NQ_IDLE_MIN in the environment overrides, for
// measurements).
uint32_t default_idle_min();
// Entries per work-head claim for a persistent launch over `len` entries
// (NQ_CLAIM in the environment overrides, for measurements).
uint32_t default_claim(uint64_t len, const LaunchCfg& cfg);

// Records a failing hipError_t for nq_last_hip_error().
void set_hip_error(int err);

// The frontier of (n, depth) resident in device memory, in one allocation
// cols | ld | rd | weight (frontier order), plus the start of every row-0 run
// (then len).  Built on the host (frontier_fill) at a shallow depth and, for
// depth >= 7, deepened on the device by up to two rows (expand_device), so
// that frontiers of 10^9 entries never pass through host memory.
struct DeviceFrontier {
    void* dev = nullptr;
    uint64_t len = 0;
    uint64_t cap = 0;               // entries the arrays are laid out for (>= len)
    uint32_t* cols = nullptr;
    uint32_t* ld = nullptr;
    uint32_t* rd = nullptr;
    uint8_t* w = nullptr;
    std::vector<uint64_t> first_row;
    DeviceFrontier() = default;
    DeviceFrontier(const DeviceFrontier&) = delete;
    DeviceFrontier& operator=(const DeviceFrontier&) = delete;
    DeviceFrontier(DeviceFrontier&& o) noexcept
        : dev(o.dev), len(o.len), cap(o.cap), cols(o.cols), ld(o.ld), rd(o.rd), w(o.w),
          first_row(std::move(o.first_row)) {
        o.dev = nullptr;
    }
    DeviceFrontier& operator=(DeviceFrontier&& o) noexcept;   // frees what it held
    ~DeviceFrontier();
};
// Builds it on `stream` and waits for it.  NQ_ENOMEM when it does not fit.
int build_device_frontier(uint32_t n, uint32_t depth, void* stream, DeviceFrontier* out);
// The same from an explicit split: the host frontier of depth host_depth,
// expanded by `rows` (0..3) on the device.  With `offsets` non-null and rows > 0
// it also receives, for every host-depth entry i, the index of its first child
// (offsets[F_host] = len), so that entries [a, b) of the host-depth frontier
// correspond to [offsets[a], offsets[b]) of the built one.
int build_device_frontier_at(uint32_t n, uint32_t host_depth, uint32_t rows, void* stream,
                             DeviceFrontier* out, std::vector<uint64_t>* offsets);

// Frames per lane needed by a subproblem with `placed` queens on an n board.
inline uint32_t frames_needed(uint32_t n, uint32_t placed) {
    return (n >= placed + 2) ? (n - 2 - placed) : 0u;
}

}  // namespace nqi
