// Host frontier generator: the pre-placed subproblems of Section 1 and the
// subproblem generation of Section 2 (Algorithm 1 stopped after `depth` rows).
//
// The enumeration is split into "roots" (placements of the first one or two
// rows under the symmetry rule).  Each root's entries form one contiguous run
// of the canonical order, so a large frontier is filled in parallel: every root
// is first sized, then written into its own slice by a pool of threads.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "nq_internal.h"

namespace nqi {

namespace {

struct Sink {
    uint32_t* cols;
    uint32_t* ld;
    uint32_t* rd;
    uint8_t* weight;
    uint64_t pos;
    uint32_t last;
    uint8_t w;
    bool kings;
};

// The triple below (c, l, r) after placing p: queens carry both diagonals down
// (Somers' recurrence); a king attacks only the next row's neighbours of p.
inline void child(bool kings, uint32_t c, uint32_t l, uint32_t r, uint32_t p, uint32_t& nc,
                  uint32_t& nl, uint32_t& nr) {
    nc = c | p;
    nl = kings ? (p << 1) : ((l | p) << 1);
    nr = kings ? (p >> 1) : ((r | p) >> 1);
}

// Placements of `rows_left` more rows below (c, l, r), lowest column first.
void expand_fill(Sink& s, int rows_left, uint32_t c, uint32_t l, uint32_t r) {
    if (rows_left == 0) {
        s.cols[s.pos] = c;
        s.ld[s.pos] = l & s.last;
        s.rd[s.pos] = r;
        if (s.weight) s.weight[s.pos] = s.w;
        ++s.pos;
        return;
    }
    uint32_t v = s.last & ~(c | l | r);
    while (v) {
        uint32_t p = v & (0u - v), nc, nl, nr;
        v ^= p;
        child(s.kings, c, l, r, p, nc, nl, nr);
        expand_fill(s, rows_left - 1, nc, nl, nr);
    }
}

uint64_t expand_count(uint32_t last, bool kings, int rows_left, uint32_t c, uint32_t l,
                      uint32_t r) {
    if (rows_left == 0) return 1;
    uint32_t v = last & ~(c | l | r);
    if (rows_left == 1) return (uint64_t)__builtin_popcount(v);
    uint64_t total = 0;
    while (v) {
        uint32_t p = v & (0u - v), nc, nl, nr;
        v ^= p;
        child(kings, c, l, r, p, nc, nl, nr);
        total += expand_count(last, kings, rows_left - 1, nc, nl, nr);
    }
    return total;
}

}  // namespace

// Roots in canonical order.  Every root sits at row `row` with `rows_left`
// rows still to place before the frontier depth.
std::vector<Root> frontier_roots(uint32_t n, uint32_t depth, bool kings) {
    std::vector<Root> roots;
    const uint32_t last = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
    if (depth == 0) {
        roots.push_back({0, 0, 0, 0, 0, 1, 0, kings});
        return roots;
    }
    const uint32_t half = n / 2;
    // Row 0 in the first half of the board, weight 2; expand one more row when
    // the frontier is deep enough, so that large frontiers split finely.
    for (uint32_t c0 = 0; c0 < half; ++c0) {
        uint32_t p = 1u << c0;
        uint32_t c = p, l = p << 1, r = p >> 1;
        if (depth >= 3) {
            uint32_t v = last & ~(c | l | r);
            while (v) {
                uint32_t q = v & (0u - v), nc, nl, nr;
                v ^= q;
                child(kings, c, l, r, q, nc, nl, nr);
                roots.push_back({nc, nl, nr, 2, (int)depth - 2, 2, c0, kings});
            }
        } else {
            roots.push_back({c, l, r, 1, (int)depth - 1, 2, c0, kings});
        }
    }
    if (n % 2 == 1) {
        const uint32_t m = half;
        uint32_t p = 1u << m;
        uint32_t c = p, l = p << 1, r = p >> 1;
        if (depth == 1) {
            roots.push_back({c, l, r, 1, 0, 1, m, kings});
        } else {
            // Row 1 restricted to columns 0..m-2: the mirror images of the
            // columns right of the centre (Section 1 and its footnote).
            uint32_t v = last & ~(c | l | r) & ((m >= 2) ? ((1u << (m - 1)) - 1u) : 0u);
            while (v) {
                uint32_t q = v & (0u - v), nc, nl, nr;
                v ^= q;
                child(kings, c, l, r, q, nc, nl, nr);
                roots.push_back({nc, nl, nr, 2, (int)depth - 2, 2, m, kings});
            }
        }
    }
    return roots;
}

uint64_t root_size(uint32_t n, const Root& rt) {
    const uint32_t last = (1u << n) - 1u;
    return expand_count(last, rt.kings, rt.rows_left, rt.cols, rt.ld, rt.rd);
}

void root_fill(uint32_t n, const Root& rt, uint32_t* cols, uint32_t* ld, uint32_t* rd,
               uint8_t* weight) {
    Sink s{cols, ld, rd, weight, 0, (1u << n) - 1u, rt.weight, rt.kings};
    expand_fill(s, rt.rows_left, rt.cols, rt.ld, rt.rd);
}

static unsigned pool_threads(uint64_t work) {
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    if (work < (1u << 16)) return 1;
    return std::min(hw, 32u);
}

template <class F>
static void parallel_for(size_t count, unsigned threads, F&& fn) {
    if (threads <= 1 || count <= 1) {
        for (size_t i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<size_t> next{0};
    auto work = [&] {
        for (size_t i; (i = next.fetch_add(1)) < count;) fn(i);
    };
    std::vector<std::thread> pool;
    try {
        for (unsigned t = 1; t < threads; ++t) pool.emplace_back(work);
    } catch (...) {
        // A thread that cannot be started leaves its share to the others.
    }
    work();                                       // the calling thread is one worker
    for (auto& th : pool) th.join();
}

std::vector<uint64_t> root_offsets(uint32_t n, const std::vector<Root>& roots) {
    std::vector<uint64_t> sizes(roots.size());
    parallel_for(roots.size(), roots.size() > 8 ? pool_threads(1u << 20) : 1,
                 [&](size_t i) { sizes[i] = root_size(n, roots[i]); });
    std::vector<uint64_t> off(roots.size() + 1, 0);
    for (size_t i = 0; i < roots.size(); ++i) off[i + 1] = off[i] + sizes[i];
    return off;
}

int frontier_fill(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld, uint32_t* rd,
                  uint8_t* weight, uint64_t capacity, uint64_t* out_len,
                  std::vector<uint64_t>* first_row_offsets, bool kings) {
    if (n < 1 || n > NQ_MAX_N_WIDE || depth > n || !out_len) return NQ_EINVAL;
    std::vector<Root> roots = frontier_roots(n, depth, kings);
    std::vector<uint64_t> off = root_offsets(n, roots);
    const uint64_t total = off.back();
    *out_len = total;
    if (first_row_offsets) {
        // Start offset of each first-row column's run, plus the end.
        first_row_offsets->clear();
        for (size_t i = 0; i < roots.size(); ++i)
            if (i == 0 || roots[i].first_col != roots[i - 1].first_col)
                first_row_offsets->push_back(off[i]);
        first_row_offsets->push_back(total);
    }
    if (!cols || !ld || !rd || capacity == 0) return NQ_OK;
    const bool partial = capacity < total;
    if (!partial) {
        parallel_for(roots.size(), pool_threads(total), [&](size_t i) {
            root_fill(n, roots[i], cols + off[i], ld + off[i], rd + off[i],
                      weight ? weight + off[i] : nullptr);
        });
        return NQ_OK;
    }
    // Partial fill: whole roots that fit, then the head of the next one.
    for (size_t i = 0; i < roots.size() && off[i] < capacity; ++i) {
        uint64_t sz = off[i + 1] - off[i];
        if (off[i] + sz <= capacity) {
            root_fill(n, roots[i], cols + off[i], ld + off[i], rd + off[i],
                      weight ? weight + off[i] : nullptr);
        } else {
            std::vector<uint32_t> c(sz), l(sz), r(sz);
            std::vector<uint8_t> w(sz);
            root_fill(n, roots[i], c.data(), l.data(), r.data(), w.data());
            uint64_t take = capacity - off[i];
            std::memcpy(cols + off[i], c.data(), take * 4);
            std::memcpy(ld + off[i], l.data(), take * 4);
            std::memcpy(rd + off[i], r.data(), take * 4);
            if (weight) std::memcpy(weight + off[i], w.data(), take);
        }
    }
    return NQ_ERANGE;
}

}  // namespace nqi

extern "C" int nq_frontier_runs(uint32_t n, uint32_t depth, uint64_t* offsets, uint32_t capacity,
                                uint32_t* out_runs) {
    if (n < 1 || n > NQ_MAX_N_WIDE || depth < 1 || depth > n || !out_runs) return NQ_EINVAL;
    try {
        std::vector<uint64_t> runs;
        uint64_t total = 0;
        int rc = nqi::frontier_fill(n, depth, nullptr, nullptr, nullptr, nullptr, 0, &total, &runs);
        if (rc != NQ_OK) return rc;
        const uint32_t count = (uint32_t)runs.size() - 1;
        *out_runs = count;
        if (!offsets) return NQ_OK;
        if (capacity < count + 1) return NQ_ERANGE;
        for (uint32_t i = 0; i <= count; ++i) offsets[i] = runs[i];
        return NQ_OK;
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_frontier(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld,
                           uint32_t* rd, uint8_t* weight, uint64_t capacity,
                           uint64_t* out_len) {
    try {
        return nqi::frontier_fill(n, depth, cols, ld, rd, weight, capacity, out_len, nullptr);
    } catch (...) {
        return NQ_ENOMEM;
    }
}

extern "C" int nq_kings_frontier(uint32_t n, uint32_t depth, uint32_t* cols, uint32_t* ld,
                                 uint32_t* rd, uint8_t* weight, uint64_t capacity,
                                 uint64_t* out_len) {
    try {
        return nqi::frontier_fill(n, depth, cols, ld, rd, weight, capacity, out_len, nullptr,
                                  true);
    } catch (...) {
        return NQ_ENOMEM;
    }
}
