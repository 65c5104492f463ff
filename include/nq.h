/*
 * libnq -- exact N-Queens solution counting on AMD Instinct MI355X (gfx950).
 *
 * The method (Yao & Li, "High-Performance N-Queens Solver on GPU: Iterative DFS
 * with Zero Bank Conflicts"):
 *   - Section 1: the board is split into independent subtrees by pre-placing the
 *     queens of the first k rows.  Only the first half of row 0 is enumerated
 *     (mirror symmetry, weight 2); for odd N the centre column of row 0 is added
 *     with the row-1 queen restricted to the first N/2 - 1 columns (weight 2).
 *     The solution count is the weighted sum of the subtrees' leaf counts.
 *   - Section 2, Algorithm 1: a subproblem is the Somers triple (cols, ld, rd) of
 *     32-bit masks; placing bit p does cols |= p, ld = (ld | p) << 1,
 *     rd = (rd | p) >> 1, and the free squares of the next row are
 *     last & ~(cols | ld | rd) with last = 2^N - 1.
 *   - Section 2, Algorithm 2, and Section 3.2.3 / Algorithm 3: each subtree is
 *     searched by an iterative DFS with an explicit stack of (cols, ld, rd,
 *     avail) frames; the last row is never pushed, its free squares are counted.
 *   - Section 4.5: N = 28 is the last size whose count fits in 64 bits; larger
 *     boards need wider totals.
 *
 * Conventions for every entry point:
 *   - Return value: NQ_OK (0) or a negative NQ_E* status.  Nothing throws, aborts
 *     or exits.  Outputs are written through pointers and only on NQ_OK, except
 *     where a function says otherwise (nq_frontier with NQ_ERANGE,
 *     nq_count_resumable with NQ_EAGAIN).
 *   - Bit j of a mask stands for column j.  Valid board sizes: 1 <= n <= 28
 *     (NQ_MAX_N); larger n is NQ_EINVAL, except where a function accepts boards
 *     up to NQ_MAX_N_WIDE (31, the widest board whose masks fit in 32 bits):
 *     nq_frontier, nq_kings_frontier, nq_frontier_runs, nq_expand,
 *     nq_count_subproblems (with 128-bit totals) and nq_count_resumable_wide.
 *   - Counts are exact uint64.  Per-subproblem counts are UNWEIGHTED; totals are
 *     weighted by the symmetry weights.
 *   - Host buffers are owned by the caller.  Device buffers passed in are owned
 *     by the caller and must stay valid until the work on the given stream ends.
 *   - A HIP failure returns NQ_EDEVICE; nq_last_hip_error() gives the hipError_t
 *     of the failing call on the calling thread.
 *   - Calls on distinct streams may run concurrently.  A server handle is
 *     internally locked.
 */
#ifndef NQ_H_
#define NQ_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NQ_MAX_N 28
#define NQ_MAX_N_WIDE 31

enum nq_status {
    NQ_OK = 0,
    NQ_EINVAL = -1,   /* invalid argument                                        */
    NQ_ERANGE = -2,   /* output buffer too small; *out_len holds the needed size  */
    NQ_ENOMEM = -3,   /* host or device allocation failed, or over a memory cap   */
    NQ_EDEVICE = -4,  /* a HIP call failed; see nq_last_hip_error()              */
    NQ_EAGAIN = -5,   /* nq_serve_poll: not finished yet; nq_count_resumable:
                         chunks remain (call again)                               */
    NQ_EFULL = -6,    /* nq_serve_submit: admission refused, retry later          */
    NQ_ENOENT = -7    /* unknown ticket                                           */
};

/* Static, human-readable text for a status code (never NULL). */
const char* nq_strerror(int status);

/* hipError_t of the last failing HIP call made by this library on this thread. */
int nq_last_hip_error(void);

/*
 * nq_frontier -- the pre-placed subproblems of Section 1 / Algorithm 1.
 *
 * Enumerates every legal placement of queens in rows 0..depth-1 of an n x n
 * board under the symmetry rule above, in lexicographic order of the columns
 * (c_0, ..., c_{depth-1}), and writes each as the Somers triple it leaves for
 * row `depth`:
 *   cols[i] = columns taken, ld[i] and rd[i] = squares of row `depth` attacked
 *   along the two diagonals (ld masked to n bits), weight[i] = 2, except 1 for
 *   depth == 0 (the empty board) and for the odd-n centre entry when depth == 1.
 * Entries whose row `depth` has no free square are kept (their count is 0).
 *
 * n in [1, 31], depth in [0, n].  Size query: if cols, ld or rd is NULL, or
 * capacity == 0, only *out_len = F is written and NQ_OK returned.  Otherwise
 * the arrays (length >= capacity; weight may be NULL) are filled; if
 * capacity < F the first `capacity` entries are written, *out_len = F and
 * NQ_ERANGE is returned.  Host memory only; thread-safe.
 */
int nq_frontier(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld, uint32_t* rd,
                uint8_t* weight, uint64_t capacity, uint64_t* out_len);

/*
 * nq_kings_frontier -- nq_frontier for the kings search (NQ_FLAG_KINGS): every
 * placement of one king per row in rows 0..depth-1, distinct columns, no two
 * kings of adjacent rows in adjacent columns, under the same symmetry rule
 * (mirror image s -> n-1-s; for odd n the centre column of row 0 with row 1 in
 * [0, n/2 - 2], the centre's neighbours being excluded by the rule itself) and
 * in the same order, weights and calling convention.  ld[i] / rd[i] hold the
 * square right / left of the king of row depth-1 (masked to n bits).
 */
int nq_kings_frontier(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld, uint32_t* rd,
                      uint8_t* weight, uint64_t capacity, uint64_t* out_len);

/*
 * nq_frontier_runs -- where each row-0 column's entries start in the frontier.
 *
 * The frontier of (n, depth) is ordered by the row-0 column first, so the
 * entries of each row-0 column (and, for odd n, of the centre column) form one
 * contiguous run.  Writes the start offset of every run followed by F, i.e.
 * runs + 1 values, into offsets (capacity >= runs + 1) and *out_runs = runs.
 * With offsets == NULL only *out_runs is written.  n in [1, 31], depth in
 * [1, n]; host only.
 */
int nq_frontier_runs(uint32_t n, uint32_t depth, uint64_t* offsets, uint32_t capacity,
                     uint32_t* out_runs);

/*
 * nq_expand -- the frontier `rows` rows deeper, computed on the device.
 *
 * Algorithm 1 continued on the GPU: for len device-resident subproblems
 * (d_cols, d_ld, d_rd; d_weight nullable) of an n board, writes every placement
 * of rows (1..3) more queens below each of them, as Somers triples of the
 * deeper row, into d_ocols, d_old, d_ord (d_oweight nullable; children inherit
 * their parent's weight, 1 when d_weight is NULL).  Order: all children of entry
 * 0 (lowest column first), then entry 1, ...; expanding nq_frontier(n, k) gives
 * nq_frontier(n, k + rows) exactly when k >= 2 or n is even.  (For odd n at
 * k = 1 the centre entry has weight 1 and an unrestricted row 1; its children
 * keep weight 1, which gives the same weighted count as the deeper frontier,
 * whose centre entries restrict row 1 and carry weight 2.)  With d_ocols, d_old or d_ord NULL only
 * *out_len (the number of children) is computed; capacity < *out_len is
 * NQ_ERANGE.  n in [1, 31].  The call allocates scratch device memory and waits on `stream`
 * (hipStream_t or NULL) for the size and, when writing, for the result.
 */
int nq_expand(uint32_t n, uint32_t rows, const uint32_t* d_cols, const uint32_t* d_ld,
              const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len, uint32_t* d_ocols,
              uint32_t* d_old, uint32_t* d_ord, uint8_t* d_oweight, uint64_t capacity,
              uint64_t* out_len, void* stream);

/* Scheduling modes of the DFS kernels. */
enum nq_mode {
    NQ_MODE_AUTO = 0,        /* persistent                                            */
    NQ_MODE_PLAIN = 1,       /* one lane per subproblem, grid = ceil(F / wg_size)     */
    NQ_MODE_PERSISTENT = 2   /* resident grid, lanes refilled from an atomic queue    */
};

/* Option flags. */
enum nq_flags {
    /* Persistent mode hands entries out in frontier order instead of the
     * default reverse order (the last row-0 columns carry the largest subtrees,
     * Section 4.5, so reverse order starts the longest work first). */
    NQ_FLAG_FORWARD_ORDER = 1u,
    /* nq_count / nq_count_subproblems: count n non-attacking KINGS, one per row
     * and column, instead of queens (the second depth-first search run on the
     * same lane stack; the paper's conclusion names permutation searches as
     * candidates for its method).  A king attacks only the adjacent row, so the
     * Somers triple of an entry is (columns taken, the square right of the last
     * king, the square left of it), as nq_kings_frontier writes it.  It runs
     * the step of inner-loop form 1 while nq_set_loop_form selects form 1, and
     * the step of form 7 with the popcount leaf test under every other form;
     * batches, servers and resumable counts refuse the flag (NQ_EINVAL). */
    NQ_FLAG_KINGS = 2u,
    /* nq_count_subproblems: d_total is uint64[2], a 128-bit total (low word
     * first) increased with carry.  Required when n > 28 and d_total is set:
     * Q(29) already exceeds 2^64 (Section 4.5). */
    NQ_FLAG_WIDE_TOTAL = 4u,
    /* nq_serve_create only (the counting entry points refuse it): favour the
     * latency of quick requests (COUNTs of boards up to 16) over throughput.
     * At most one epoch of other requests runs at a time, with one resident
     * wave per CU fewer than its LDS stack allows, so that an epoch of quick
     * requests always finds room on every CU.  Measured on a mix of COUNT
     * N = 10..18 and N = 21 slices: the quick COUNTs' p99 at 200 requests per
     * second 8-13 ms instead of 26-53 ms, 15-31 ms instead of 146-194 ms
     * beyond saturation, for 8 % less throughput at saturation and longer
     * waits of the other requests. */
    NQ_FLAG_SERVE_RESERVE = 8u
};
#define NQ_FLAGS_ALL 15u
/* The flags nq_count, nq_count_subproblems(_noalloc), the batch and the
 * resumable entry points accept; any other bit is NQ_EINVAL there. */
#define NQ_FLAGS_COUNT 7u

/*
 * Options shared by the counting entry points.  A NULL options pointer, or a
 * zero field, means "automatic".
 */
typedef struct nq_opts {
    uint32_t depth;          /* pre-placed rows k (nq_count / nq_count_batch); 0 = auto */
    uint32_t mode;           /* enum nq_mode                                           */
    uint32_t wg_size;        /* threads per workgroup, multiple of 64, <= 1024         */
    uint32_t waves_per_cu;   /* persistent grid: resident waves per CU (0 = max fit)   */
    uint32_t refill_every;   /* DFS steps between refill checks (0 = default)          */
    uint32_t flags;          /* NQ_FLAG_* bits; unknown bits are NQ_EINVAL             */
    void* stream;            /* hipStream_t to run on; NULL = the null stream          */
    uint64_t* counts_out;    /* nq_count: optional host buffer, F unweighted counts    */
    uint64_t counts_capacity;/* length of counts_out                                   */
    double* kernel_ms_out;   /* optional: device time of the DFS kernel(s), HIP events;
                                setting it makes the call wait for the kernel         */
    uint64_t* d_nodes;       /* nq_count_subproblems only, optional device uint64[len]:
                                DFS nodes of each subproblem (queens placed in rows
                                placed..n-2); selects the node-counting kernel        */
    uint32_t claim;          /* persistent mode: entries a wave takes from the shared
                                work head per atomic add (0 = default); what its idle
                                lanes do not need yet feeds its later refills         */
} nq_opts;

/*
 * nq_count -- Q(n): the number of ways to place n non-attacking queens.
 *
 * Builds the frontier of depth opts->depth (on the host, nq_frontier; for depth
 * >= 7 the depth-5 one on the host, deepened on the device by nq_expand in
 * steps of at most three rows) in
 * device memory owned by the library, runs the DFS kernels (Algorithm 2 with
 * the last-row step of Algorithm 3, one subproblem per lane) and returns the
 * weighted total in *out_total.  Synchronous: returns after the result is on the
 * host.  If opts->counts_out is set, it receives the per-subproblem counts in
 * frontier order (NQ_ERANGE if counts_capacity < F).  n in [1, 28].
 * opts->depth == 0 selects the depth nq_autotune found for n in this process,
 * else the shallowest depth whose frontier has at least 2^29 entries (at most
 * n - 4, and under 2^32 entries); for n = 21, 22 and 23, whose best depth
 * has a frontier too large (or not worth building whole), the automatic count
 * runs in chunks of the depth-5 frontier deepened on the device (n = 21: 16
 * chunks to depth 10; 22 and 23: 64 chunks to depth 11), as
 * nq_count_resumable does without a file (persistent mode, no per-entry
 * counts).  With NQ_FLAG_KINGS the kings frontier
 * (nq_kings_frontier) is built on the host only, at opts->depth or by default
 * the shallowest depth with at least 2^22 entries (at most n - 2 and 2^27
 * entries); the number of king placements passes 2^64 at n = 22, so with
 * that flag n > 21 is NQ_EINVAL.  NQ_FLAG_WIDE_TOTAL is NQ_EINVAL here.
 */
int nq_count(uint32_t n, const nq_opts* opts, uint64_t* out_total);

/*
 * nq_count_subproblems -- count the subtrees of caller-provided subproblems.
 *
 * Device pointers: d_cols, d_ld, d_rd (uint32[len], Somers triples for an
 * n x n board, bit j = column j; bits >= n are ignored), d_weight (uint8[len]
 * or NULL for weight 1), d_counts (uint64[len] or NULL) receives each
 * subproblem's unweighted leaf count, d_total (one uint64 or NULL) is
 * INCREASED by sum(weight * count) -- the caller zeroes it.  The queens already
 * placed are the set bits of cols, so a triple with popcount(cols) = n counts 1,
 * with n - 1 counts its free squares of the last row, and one with no free
 * square counts 0.  opts->depth promises that every triple has at least that
 * many queens placed; it sizes the LDS stack (n - 2 - depth frames per lane).
 * A triple with fewer queens is not searched: its d_counts entry is set to
 * UINT64_MAX and it adds nothing to d_total.  Asynchronous on opts->stream
 * (unless kernel_ms_out is set); len == 0 launches nothing.  n may be up to
 * NQ_MAX_N_WIDE (31); for n > 28 opts->depth must be at least n - 20 (at most
 * 20 rows below every prefix, so a per-subproblem count stays below 20! <
 * 2^62) and a non-NULL d_total needs NQ_FLAG_WIDE_TOTAL.  With
 * NQ_FLAG_KINGS the triples are kings-search triples (nq_kings_frontier: ld /
 * rd hold only the squares beside the last king) and the counts are king
 * placements; the same rules for full, last-row and dead entries apply.
 */
int nq_count_subproblems(uint32_t n, const uint32_t* d_cols, const uint32_t* d_ld,
                         const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len,
                         uint64_t* d_counts, uint64_t* d_total, const nq_opts* opts);

/*
 * nq_count_subproblems_noalloc -- nq_count_subproblems for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.
 *
 * Same arguments, layouts, ownership and results as nq_count_subproblems.  The
 * persistent scheduler's 64-bit work head, the only device memory the DFS
 * kernels need beyond the caller's buffers, lives in a 256-byte device array
 * of the library (one per GPU, held until the process ends; the head uses its
 * first 8 bytes, and no input size changes that), zeroed by a kernel before
 * each launch.  The call allocates nothing, never synchronizes and records no
 * memset.  opts->kernel_ms_out must be NULL (timing would create events):
 * NQ_EINVAL otherwise.  The first call on a device looks up the array's
 * device address.  Calls that overlap on one GPU (on different streams or
 * threads) share the array and race on the head: the caller serializes them.
 */
int nq_count_subproblems_noalloc(uint32_t n, const uint32_t* d_cols, const uint32_t* d_ld,
                                 const uint32_t* d_rd, const uint8_t* d_weight, uint64_t len,
                                 uint64_t* d_counts, uint64_t* d_total, const nq_opts* opts);

/*
 * nq_count_batch -- many independent counts in one persistent launch.
 *
 * For each instance i < ninst, builds the frontier of ns[i] (depth from
 * depths[i] when depths != NULL, else opts->depth or automatic), concatenates
 * them with per-entry instance ids, runs one persistent DFS launch (captured
 * and replayed as a HIP graph) and writes Q(ns[i]) to out_totals[i].
 * Synchronous.  Every ns[i] in [1, 28]; ninst == 0 does nothing.
 */
int nq_count_batch(uint32_t ninst, const uint32_t* ns, const uint32_t* depths,
                   const nq_opts* opts, uint64_t* out_totals);

/*
 * nq_count_resumable -- Q(n) as a sequence of chunks whose progress is kept in
 * a file, so that a long count that stops (a lost job, a time limit) resumes
 * where it stopped instead of starting over.  The paper runs N = 27 for months
 * and names fault tolerance as future work (Section 6); subproblems are
 * independent (Section 1), so a chunk's weighted count never changes and can
 * be recorded once it is done.
 *
 * The host frontier of depth min(depth, 5) (nq_frontier order) is cut into
 * `chunks` contiguous ranges (0 = 64); range i covers entries
 * [F*i/chunks, F*(i+1)/chunks).  Each range is deepened on the device to the
 * count's depth (opts->depth; 0 = as nq_count chooses) and searched by one
 * launch (opts->mode etc. as for nq_count).  After every range the file at
 * `path` is replaced (written to path.tmp, flushed, renamed) by one text line:
 *   nq-progress 1 n=.. depth=.. host_depth=.. chunks=.. done=.. total=.. check=..
 * (total = the weighted count of the ranges done; check = FNV-1a 64 of the text
 * before " check=").  A call that finds a record of the same n, depth, host
 * depth and chunks continues after its last range; a record of another count,
 * or a file that is not one intact record, is NQ_EINVAL (and left as it is).
 * At most max_chunks ranges are counted per call (0 = all).  Returns NQ_OK with
 * *out_total = Q(n) when every range is done, NQ_EAGAIN with the partial total
 * while ranges remain; *out_done = ranges done.  opts->counts_out and
 * opts->d_nodes must be NULL.  NQ_EINVAL also when the file cannot be written.
 * With opts->depth == 0 the depth is that of an existing record of the same n
 * and chunk count, else the one nq_count's automatic chunked count uses for n,
 * else nq_count's frontier-size rule; never a tuning result, so that every
 * process that continues a file picks the same depth.  n in [1, 28]; a total
 * of 2^64 or more (possible only for files written by nq_count_resumable_wide)
 * is NQ_ERANGE, with *out_done written and *out_total untouched.
 * Synchronous; one call at a time per file.
 */
int nq_count_resumable(uint32_t n, const nq_opts* opts, const char* path, uint32_t chunks,
                       uint32_t max_chunks, uint64_t* out_total, uint32_t* out_done);

/*
 * nq_count_resumable_wide -- nq_count_resumable with a 128-bit total, for
 * boards beyond the 64-bit limit of Section 4.5 (N = 28 is the last count
 * that fits in int64).  n in [1, 31] (NQ_MAX_N_WIDE); for n > 28 the depth
 * (opts->depth, or the automatic one) must be at least n - 20, which keeps
 * every per-subproblem count below 2^62.  Each range is counted with a
 * 128-bit device total (NQ_FLAG_WIDE_TOTAL), the ranges are added in 128 bits
 * on the host (the automatic depth of a board beyond 28 is n - 20), and the
 * record's total= field holds the 128-bit decimal value.
 * out_total[0] receives the low and out_total[1] the high 64 bits.  Everything
 * else is as nq_count_resumable, and both read and write the same records.
 */
int nq_count_resumable_wide(uint32_t n, const nq_opts* opts, const char* path, uint32_t chunks,
                            uint32_t max_chunks, uint64_t* out_total, uint32_t* out_done);

/*
 * nq_autotune -- measure the best pre-placement depth and launch shape for n.
 *
 * Times complete persistent counts of n on the current device: every depth in
 * [depth_lo, depth_hi] (0, 0 = max(1, n - 14) .. +4) twice with the default
 * launch shape, then, at the best depth, workgroup sizes of 64, 128 and 256
 * threads, a few resident-wave counts per CU, scheduler-visit intervals and
 * claim block sizes (entries a wave takes from the shared work head per
 * atomic: the persistent scheduler's queue depth), each axis starting from the
 * best so far, until budget_ms of device time is spent (0 = 60 s).
 * The paper tunes the pre-placed rows and the block and stack size by hand
 * (Section 4.1 Table 3, Section 4.2 Table 4).  Every trial must produce the
 * same count (else NQ_EDEVICE).  The winner is written to *out and remembered
 * for this process and device: nq_count with opts->depth == 0 then uses its
 * depth and every launch field the caller left at 0.  n in [4, 28].
 * Boards whose automatic count runs in chunks (n = 21, 22, 23: a whole count
 * takes 9 s to 13 min) are tuned on one chunk instead: the middle chunk of
 * the count's chunk plan (16 chunks for 21, 64 for 22 and 23) at every depth
 * in [depth_lo, depth_hi] (0, 0 = the plan's depth - 1 .. + 1; at least 5)
 * with the default launch shape, timed in wall-clock time (host frontier,
 * device expansion, DFS, result); out->chunks = the plan's chunk count,
 * out->count = that chunk's count (every depth must agree on it), and
 * nq_count then runs its chunked count at the tuned depth.
 */
typedef struct nq_tuned {
    uint32_t depth;          /* pre-placed rows                                  */
    uint32_t waves_per_cu;   /* 0 = as many as the LDS stacks allow              */
    uint32_t refill_every;   /* DFS steps between scheduler visits               */
    uint32_t trials;         /* timed counts made                                */
    double ms;               /* best device time of one count                    */
    uint64_t count;          /* the count every trial agreed on                  */
    uint32_t claim;          /* entries per work-head claim (0 = size default)   */
    uint32_t wg_size;        /* threads per workgroup (0 = the default, 64)      */
    uint32_t chunks;         /* 0 = one launch over the whole frontier; else the
                                count runs in this many chunks of the depth-5
                                frontier (n = 21..23)                           */
    uint32_t reserved;       /* 0                                                */
} nq_tuned;
int nq_autotune(uint32_t n, uint32_t depth_lo, uint32_t depth_hi, double budget_ms,
                nq_tuned* out);

/*
 * nq_autotune_trials -- nq_autotune that also reports every trial: trials[i]
 * (caller-owned, `capacity` entries) receives the i-th timed count's depth,
 * launch shape (0 = that field's default), subproblems and device time, in
 * the order they ran; *out_count = the trials written (at most capacity; the
 * search itself is not shortened).  NQ_EINVAL if trials or out_count is NULL.
 */
typedef struct nq_tune_trial {
    uint32_t depth, wg_size, waves_per_cu, refill_every, claim;
    uint32_t chunks;         /* 0 = a whole count; else one chunk of this many */
    double ms;
    uint64_t subproblems;    /* entries searched (0 for a chunk trial)         */
} nq_tune_trial;
int nq_autotune_trials(uint32_t n, uint32_t depth_lo, uint32_t depth_hi, double budget_ms,
                       nq_tuned* out, nq_tune_trial* trials, uint32_t capacity,
                       uint32_t* out_count);

/*
 * nq_tuned_lookup -- the tuning nq_autotune remembered for n on the current
 * device in this process (what nq_count's automatic depth and launch shape
 * use).  NQ_ENOENT when n has not been tuned; n in [1, 28].
 */
int nq_tuned_lookup(uint32_t n, nq_tuned* out);

/*
 * nq_set_loop_form -- choose the DFS inner-loop form of the launches planned
 * from now on, to measure the forms against each other; all give the same
 * counts.  form: -1 = the default (NQ_DFS_LOOP from the environment, else
 * the library's default form), 0 = compiler-scheduled C++ step, 1 = hand-placed
 * exec masks, 2 = form 1 with the untried set negated, 3 = a step without
 * selects (the frame being expanded is pushed while it has untried columns,
 * the child is computed into a second register frame, and a child that is not
 * searched is replaced by a pop), 4 = the frame being expanded read from the
 * LDS stack at every step with its untried set written back (Algorithm 2 as
 * printed in Section 2, with the last-row step of Algorithm 3, Section
 * 3.2.3), 5 = form 0 without the last-row step (Algorithm 2 alone), 6 = form 3
 * with a push that needs no exec mask (every lane writes the free slot above
 * its stack), 7 = form 6 without the sentinel frame below each lane's stack
 * (a lane whose search ends is parked in registers; the library's default).
 * Forms 3 to 7 keep one LDS frame more per lane than forms 0 to 2; form 7 has
 * no sentinel frame, one less than the others.  *previous (nullable) receives the
 * form in use.  NQ_EINVAL for any other form.
 * Process-wide; a launch keeps the form it was planned with (a server's epochs
 * or a batch plan made before the call keep theirs), so set it while no other
 * thread plans launches.  Touches no device.
 */
int nq_set_loop_form(int form, int* previous);

/*
 * Reusable batch plan: nq_count_batch split into set-up and replay.
 *
 * nq_batch_create builds and uploads the concatenated frontiers of ninst >= 1
 * instances (as nq_count_batch; depths[i] in [1, ns[i]] or NULL for
 * opts->depth, else max(5, ns[i] - 11) -- at most 9 stack frames per lane --
 * capped at ns[i] - 2 and at least 1; deep frontiers are built by device
 * expansion), allocates every device and
 * pinned host buffer the launch needs, and captures one HIP graph: zero the
 * totals, zero the work head, the persistent DFS kernel, copy the totals to
 * the host.  The plan owns a private stream.  nq_batch_run replays the graph,
 * waits for it and writes the ninst totals; kernel_ms (nullable) receives the
 * device time of the replay.  nq_batch_entries gives the number of concatenated
 * subproblems.  nq_batch_destroy waits for the plan's stream and frees
 * everything.  A plan may be replayed any number of times; replays of one plan
 * must not overlap (calls on one plan are not thread-safe).
 */
typedef struct nq_batch nq_batch;
int nq_batch_create(uint32_t ninst, const uint32_t* ns, const uint32_t* depths,
                    const nq_opts* opts, nq_batch** out);
int nq_batch_run(nq_batch* batch, uint64_t* out_totals, double* kernel_ms);
uint64_t nq_batch_entries(const nq_batch* batch);
int nq_batch_destroy(nq_batch* batch);

/*
 * Serving: continuous batching of count requests on one GPU.
 *
 * Not in the paper (its runs are single counts); the unit of work is still the
 * pre-placed subproblem of Section 1, searched by the DFS of Algorithm 2 /
 * Algorithm 3.  Requests:
 *   NQ_REQ_COUNT  Q(n); depth = pre-placement depth (0 = the server picks the
 *                 shallowest depth with >= 2^18 subproblems and at least
 *                 n - 11, at most n - 4).
 *   NQ_REQ_SLICE  sum(weight * count) over entries [start, start + len) of the
 *                 (n, depth) frontier in nq_frontier order.
 * Every (n, depth) frontier is built once and kept in device memory; requests
 * are copied out of it on the device.  For slices of a frontier of >= 2^16
 * entries (depth >= 2) the kept frontier is expanded by three rows (two when
 * n < depth + 13, one when n < depth + 10), as far as the budget allows (half
 * of it holds kept frontiers): a slice's subtrees are then
 * searched as their children, a contiguous range of the expanded frontier with
 * the same weights, so the result is unchanged and the work spreads wider.
 * A scheduler thread owned by the server admits requests in arrival order while
 * request slots (4096), work-ring space and the LDS stack of the epoch kernel
 * allow, and launches bounded persistent "epochs" over the newly admitted
 * subproblems on one of four streams, so new work overlaps the tail of
 * older work.  An epoch starts only on a stream with no epoch in flight; the
 * last stream takes only epochs of quick requests (COUNTs of boards up to
 * 16), which may start before older requests of other kinds.  With
 * NQ_FLAG_SERVE_RESERVE the other epochs run one at a time and leave a wave
 * slot per CU to quick ones (lower latency for quick requests, less
 * throughput).  A request's result is published to pinned host memory by the
 * GPU lane that retires its last subproblem (retirements are added to the
 * request's total and remaining count once per wave and request).
 *
 * nq_serve_create: opts may set flags (NQ_FLAG_SERVE_RESERVE; NQ_FLAG_KINGS
 * and NQ_FLAG_WIDE_TOTAL are NQ_EINVAL), depth (= the LDS stack frames per lane of the
 * epoch kernel, default 14, at most 26 (NQ_EINVAL beyond): a request whose
 * subproblems need more stack than that is refused with NQ_EINVAL at submit;
 * each epoch's LDS stack is sized for the deepest request in it), wg_size,
 * waves_per_cu and
 * refill_every; hbm_budget_bytes (0 = 8 GiB) is split between the work ring
 * (17 B per subproblem) and the resident slice frontiers.
 * nq_serve_submit: non-blocking; NQ_EINVAL for a malformed request, NQ_EFULL
 * when 65536 requests are already waiting.  A request larger than the ring, or
 * a slice past the end of its frontier, completes with that status in
 * nq_result.status.
 * nq_serve_poll: NQ_OK (result written, ticket released), NQ_EAGAIN (not done),
 * NQ_ENOENT (unknown or already collected ticket).  nq_serve_wait: the same,
 * blocking up to timeout_ns.  Timestamps are CLOCK_MONOTONIC nanoseconds:
 * submit, admission (subproblems enqueued), completion seen by the scheduler.
 * After a failure in the server (an epoch that cannot be enqueued or that
 * ends in a device error: NQ_EDEVICE; a host allocation of its thread:
 * NQ_ENOMEM) every unfinished request reports that status instead of
 * NQ_EAGAIN, and submit returns it too; the server's own thread met the
 * error, and nq_last_hip_error() on the thread that gets the status returns
 * its hipError_t.
 * nq_serve_destroy: drops requests not yet admitted, waits for admitted ones
 * (not after such a failure), frees everything, and returns the failure's
 * status or NQ_OK.  All calls on one server are thread-safe.
 */
enum nq_request_kind { NQ_REQ_COUNT = 1, NQ_REQ_SLICE = 2 };
typedef struct nq_request {
    uint32_t kind;           /* enum nq_request_kind                              */
    uint32_t n;              /* board size, 1..28                                  */
    uint32_t depth;          /* pre-placement depth (see above)                    */
    uint32_t reserved;       /* must be 0                                          */
    uint64_t start;          /* NQ_REQ_SLICE: first entry                          */
    uint64_t len;            /* NQ_REQ_SLICE: number of entries                    */
} nq_request;
typedef struct nq_result {
    int32_t status;          /* NQ_OK or why the request failed                    */
    uint32_t reserved;
    uint64_t count;          /* Q(n), or the slice's weighted sum                  */
    uint64_t entries;        /* subproblems searched for this request (after the
                                expansion of slices described above)              */
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;
} nq_result;
typedef struct nq_server nq_server;
int nq_serve_create(const nq_opts* opts, uint64_t hbm_budget_bytes, nq_server** out);
int nq_serve_submit(nq_server* server, const nq_request* req, uint64_t* out_ticket);
int nq_serve_poll(nq_server* server, uint64_t ticket, nq_result* out);
int nq_serve_wait(nq_server* server, uint64_t ticket, nq_result* out, uint64_t timeout_ns);
int nq_serve_destroy(nq_server* server);

/*
 * The third search on the same engine: the permanent of an n x n 0/1 matrix,
 * the number of permutations s with a[r][s(r)] = 1 for every row r, counted
 * by a depth-first search over the rows (the paper's conclusion, Section 5,
 * names combinatorial permutation problems among the searches its method
 * carries over to).  It uses a two-word frame (used columns, untried columns
 * of the row being filled) in the lane-interleaved LDS stack with 8-byte
 * slots, and its own leaf rule: the last two rows are never entered, their
 * completions are counted in closed form.  A node is one placement in rows
 * depth..n-3.
 *
 * rows (host, n words): rows[r] = the columns row r allows (bit c = a[r][c]);
 * bits at or above n are NQ_EINVAL.  n in [1, NQ_PERM_MAX_N] (20: the
 * permanent is at most n!, below 2^64).
 *
 * nq_perm_frontier: every assignment of rows 0..depth-1 to distinct allowed
 * columns, in lexicographic order of the columns, written as the set of used
 * columns (cols[i]); depth in [0, n].  The size query and partial fill follow
 * nq_frontier (NQ_ERANGE when capacity < F).  Host memory; thread-safe.
 *
 * nq_perm_count_subproblems: counts below `len` device-resident entries
 * d_cols (used-column sets with exactly `depth` rows assigned; the launch's
 * stack is sized for the n - 3 - depth frames such an entry needs (one more
 * with the hand-scheduled steps, whose frame of row n - 3 is written before
 * its leaves are counted), and an entry that needs more is
 * reported as UINT64_MAX in d_counts and left out of the total).  d_counts
 * (nullable, uint64[len]) receives each entry's count, *d_total (nullable) is
 * increased by their sum; opts: mode, wg_size, waves_per_cu, refill_every,
 * claim, stream, kernel_ms_out, d_nodes (uint64[len]: nodes per entry);
 * flags must be 0.  Asynchronous on opts->stream unless kernel_ms_out is set.
 *
 * nq_perm_count: the permanent.  Builds the frontier on the host at
 * opts->depth (0 = the shallowest depth with at least 2^20 entries, at most
 * n - 2 and 2^26 entries), copies it to the device and counts it;
 * synchronous.  opts->flags, counts_out and d_nodes must be 0.
 *
 * nq_perm_set_step: the inner step of the permanent launches from now on, to
 * measure the steps against each other; all give the same counts.  step: -1
 * = the default (NQ_PERM_STEP=0 or 1 from the environment, else 2), 0 = the
 * step in plain C++, 1 = hand-scheduled (two register frames, a push without
 * exec mask, the next row's allowed columns read before the child is known,
 * the last two rows counted under an exec mask), 2 = step 1 with the
 * children's row kept in the high bits of the used columns (the library's
 * default: two VALU instructions fewer per step).  *previous (nullable)
 * receives the step in use; NQ_EINVAL for any other step.  Process-wide, read
 * when a launch is made; touches no device.
 */
#define NQ_PERM_MAX_N 20
int nq_perm_frontier(uint32_t n, const uint32_t* rows, uint32_t depth, uint32_t* cols,
                     uint64_t capacity, uint64_t* out_len);
int nq_perm_count_subproblems(uint32_t n, const uint32_t* rows, const uint32_t* d_cols,
                              uint64_t len, uint32_t depth, uint64_t* d_counts,
                              unsigned long long* d_total, const nq_opts* opts);
int nq_perm_count(uint32_t n, const uint32_t* rows, const nq_opts* opts, uint64_t* out_total);
int nq_perm_set_step(int step, int* previous);

#ifdef __cplusplus
}
#endif

#endif /* NQ_H_ */
