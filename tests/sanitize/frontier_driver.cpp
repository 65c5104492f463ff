// Host-only driver for the sanitizer builds of the frontier enumeration
// (nq_frontier.cpp): fills frontiers of several shapes, whole and in part,
// and prints "tag n depth F cap digest" lines that the test compares with the
// library's own results.  digest = sum over the first cap entries of
// (i + 1) * (cols + 3 ld + 5 rd + 7 weight), modulo 2^64.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "nq.h"

static uint64_t digest(const std::vector<uint32_t>& c, const std::vector<uint32_t>& l,
                       const std::vector<uint32_t>& r, const std::vector<uint8_t>& w,
                       uint64_t m) {
    uint64_t h = 0;
    for (uint64_t i = 0; i < m; ++i)
        h += (i + 1) * ((uint64_t)c[i] + 3ull * l[i] + 5ull * r[i] + 7ull * w[i]);
    return h;
}

static int run(const char* tag, bool kings, uint32_t n, uint32_t depth, uint64_t cap_cut) {
    uint64_t F = 0;
    int rc = kings ? nq_kings_frontier(n, depth, nullptr, nullptr, nullptr, nullptr, 0, &F)
                   : nq_frontier(n, depth, nullptr, nullptr, nullptr, nullptr, 0, &F);
    if (rc != NQ_OK) return rc;
    const uint64_t cap = (cap_cut && cap_cut < F) ? cap_cut : F;
    std::vector<uint32_t> c(cap + 1), l(cap + 1), r(cap + 1);
    std::vector<uint8_t> w(cap + 1);
    uint64_t got = 0;
    rc = kings ? nq_kings_frontier(n, depth, c.data(), l.data(), r.data(), w.data(), cap, &got)
               : nq_frontier(n, depth, c.data(), l.data(), r.data(), w.data(), cap, &got);
    if (rc != (cap < F ? NQ_ERANGE : NQ_OK) || got != F) return -100;
    const uint64_t h = digest(c, l, r, w, cap);
    std::printf("%s %u %u %llu %llu %016llx\n", tag, n, depth, (unsigned long long)F,
                (unsigned long long)cap, (unsigned long long)h);
    return NQ_OK;
}

int main() {
    struct Case { const char* tag; bool kings; uint32_t n, depth; uint64_t cut; };
    const Case cases[] = {
        {"queens", false, 1, 1, 0},   {"queens", false, 3, 2, 0},  {"queens", false, 5, 2, 0},
        {"queens", false, 13, 4, 0},  {"queens", false, 17, 5, 0}, {"queens", false, 20, 6, 0},
        {"queens", false, 20, 6, 1000003}, {"queens", false, 15, 15, 0},
        {"kings", true, 2, 1, 0},     {"kings", true, 9, 3, 0},    {"kings", true, 16, 6, 0},
        {"kings", true, 16, 6, 77777},
    };
    for (const Case& k : cases) {
        int rc = run(k.tag, k.kings, k.n, k.depth, k.cut);
        if (rc != NQ_OK) {
            std::fprintf(stderr, "%s %u %u failed: %d\n", k.tag, k.n, k.depth, rc);
            return 1;
        }
    }
    uint64_t off[64];
    uint32_t runs = 0;
    if (nq_frontier_runs(20, 6, off, 64, &runs) != NQ_OK) return 1;
    std::printf("runs 20 6 %u %llu\n", runs, (unsigned long long)off[runs]);
    return 0;
}
