/* Driver for the sanitizer builds of the oracle (oracle/oracle.c): counts,
 * frontiers and threaded prefix counts of both searches, printed as
 * "tag values..." lines that the test compares with the oracle library. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oq_queens(int n, uint64_t* count, uint64_t* nodes);
int oq_frontier(int n, int k, int* prefixes, uint8_t* weights, uint64_t cap, uint64_t* out_len);
int oq_count_prefixes(int n, int k, const int* prefixes, uint64_t m, int threads,
                      uint64_t* counts, uint64_t* nodes);
int oq_brute_count(int n, int k, const int* prefix, uint64_t* count);
int oqk_frontier(int n, int k, int* prefixes, uint8_t* weights, uint64_t cap, uint64_t* out_len);
int oqk_count_prefixes(int n, int k, const int* prefixes, uint64_t m, int threads,
                       uint64_t* counts, uint64_t* nodes);

static int weighted(int kings, int n, int k, int threads, uint64_t* total, uint64_t* nodes) {
    uint64_t F = 0;
    if ((kings ? oqk_frontier : oq_frontier)(n, k, NULL, NULL, 0, &F)) return 1;
    int* pre = malloc(sizeof(int) * (F * k + 1));
    uint8_t* w = malloc(F + 1);
    uint64_t* c = malloc(8 * (F + 1));
    uint64_t* nd = malloc(8 * (F + 1));
    uint64_t got = 0;
    int rc = (kings ? oqk_frontier : oq_frontier)(n, k, pre, w, F, &got);
    if (!rc) rc = (kings ? oqk_count_prefixes : oq_count_prefixes)(n, k, pre, F, threads, c, nd);
    *total = 0;
    *nodes = 0;
    for (uint64_t i = 0; !rc && i < F; ++i) {
        *total += w[i] * c[i];
        *nodes += nd[i];
    }
    free(pre); free(w); free(c); free(nd);
    return rc;
}

int main(void) {
    uint64_t t = 0, nd = 0;
    for (int n = 1; n <= 11; ++n) {
        if (oq_queens(n, &t, &nd)) return 1;
        printf("queens %d %llu %llu\n", n, (unsigned long long)t, (unsigned long long)nd);
    }
    if (oq_brute_count(9, 0, NULL, &t)) return 1;
    printf("brute 9 %llu\n", (unsigned long long)t);
    if (weighted(0, 14, 3, 4, &t, &nd)) return 1;
    printf("frontier 14 3 %llu %llu\n", (unsigned long long)t, (unsigned long long)nd);
    if (weighted(1, 11, 3, 4, &t, &nd)) return 1;
    printf("kings 11 3 %llu %llu\n", (unsigned long long)t, (unsigned long long)nd);
    return 0;
}
