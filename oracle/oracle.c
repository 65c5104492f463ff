/*
 * N-Queens counting oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load or run this file.  It shares no code, header, table or helper with the
 * GPU library: no bitmasks, no shifts, no Somers state.  Every board is held as
 * three arrays of occupancy flags, exactly as the problem is defined.
 *
 * Three searches: the queens (below), the n kings of the second search and the
 * permanents of 0/1 matrices of the third (at the end of the file).
 *
 * What is computed (paper, Section 1 and Section 2):
 *   Q(N) = number of ways to put N queens on an N x N board, one per row, with
 *   no two on a common column or diagonal.  A prefix pi = (c_0..c_{k-1}) fixes
 *   the queen of row i in column c_i; Q_pi(N) counts the completions of pi.  The
 *   method pre-places k rows (Section 1, which splits the search into
 *   independent subtrees this way; Section 2, subproblem generation), keeps
 *   only the first half of row 0 by mirror symmetry, and for odd N adds the
 *   centre column of row 0 with the row-1 queen restricted to the first
 *   N/2 - 1 columns (Section 1 and its footnote).  Every kept prefix stands
 *   for itself and its mirror image (weight 2); the total is
 *   sum(w_pi * Q_pi(N)) = Q(N).
 *
 * Readings where the paper is silent (each one is pinned by the tests):
 *   - k = 1 with odd N: the centre prefix has no mirror partner and gets w = 1.
 *   - Frontier order: lexicographic in (c_0, ..., c_{k-1}).
 *   - A prefix whose row k has no free square is kept (count 0).
 *   - A "node" is one queen placement in rows k..N-2 below a prefix (the unit of
 *     one step of the iterative DFS of Algorithm 2 with the last-row step of
 *     Algorithm 3); placements in row N-1 are solutions, not nodes.
 *
 * Pins (tests/): brute-force permutation enumeration (N <= 10), published counts,
 * the 5-Queens worked example, the 27-Queens frontier size printed in the paper's
 * run log (Section 4.5), refinement and mirror invariants.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* Boards up to 31 columns: the widest whose attack masks (oq_prefix_masks)
 * fit in 32 bits.  Whole-board counts stop at 28, the last size whose count
 * fits in 64 bits (Section 4.5). */
#define OQ_MAXN 31
#define OQ_MAXN_COUNT 28

enum { OQ_OK = 0, OQ_EINVAL = -1, OQ_ERANGE = -2, OQ_ENOMEM = -3 };

/* ---------------------------------------------------------------- boards -- */

typedef struct {
    int n;
    unsigned char col[OQ_MAXN];          /* column j occupied                      */
    unsigned char dsum[2 * OQ_MAXN];     /* diagonal r + c occupied                */
    unsigned char ddif[2 * OQ_MAXN];     /* anti-diagonal r - c + n - 1 occupied   */
} board_t;

static void board_init(board_t* b, int n) {
    memset(b, 0, sizeof(*b));
    b->n = n;
}

static int board_free(const board_t* b, int r, int c) {
    return !(b->col[c] | b->dsum[r + c] | b->ddif[r - c + b->n - 1]);
}

static void board_set(board_t* b, int r, int c, unsigned char v) {
    b->col[c] = v;
    b->dsum[r + c] = v;
    b->ddif[r - c + b->n - 1] = v;
}

/* Place the prefix on an empty board.  Returns 0 if two prefix queens attack. */
static int board_place_prefix(board_t* b, int k, const int* prefix) {
    for (int r = 0; r < k; ++r) {
        int c = prefix[r];
        if (c < 0 || c >= b->n || !board_free(b, r, c)) return 0;
        board_set(b, r, c, 1);
    }
    return 1;
}

/* Count the completions of rows row..n-1; placements in rows <= n-2 are nodes. */
static uint64_t board_complete(board_t* b, int row, uint64_t* nodes) {
    if (row == b->n) return 1;
    uint64_t total = 0;
    for (int c = 0; c < b->n; ++c) {
        if (!board_free(b, row, c)) continue;
        if (row <= b->n - 2) ++*nodes;
        board_set(b, row, c, 1);
        total += board_complete(b, row + 1, nodes);
        board_set(b, row, c, 0);
    }
    return total;
}

static int valid_nk(int n, int k) { return n >= 1 && n <= OQ_MAXN && k >= 0 && k <= n; }

/* ------------------------------------------------------------ full count -- */

/* Q(n) with no symmetry at all: every column of every row (the definition). */
int oq_queens(int n, uint64_t* count, uint64_t* nodes) {
    if (!valid_nk(n, 0) || n > OQ_MAXN_COUNT || !count) return OQ_EINVAL;
    board_t b;
    board_init(&b, n);
    uint64_t nd = 0;
    *count = board_complete(&b, 0, &nd);
    if (nodes) *nodes = nd;
    return OQ_OK;
}

/* Completions of one prefix (rows 0..k-1 fixed).  An attacking prefix has 0. */
int oq_count_prefix(int n, int k, const int* prefix, uint64_t* count, uint64_t* nodes) {
    if (!valid_nk(n, k) || !count || (k > 0 && !prefix)) return OQ_EINVAL;
    board_t b;
    board_init(&b, n);
    uint64_t nd = 0;
    *count = board_place_prefix(&b, k, prefix) ? board_complete(&b, k, &nd) : 0;
    if (nodes) *nodes = nd;
    return OQ_OK;
}

/* ------------------------------------------------------------ brute force -- */

/* Next permutation in lexicographic order; returns 0 after the last one. */
static int next_perm(int* a, int m) {
    int i = m - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = m - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int lo = i + 1, hi = m - 1; lo < hi; ++lo, --hi) { t = a[lo]; a[lo] = a[hi]; a[hi] = t; }
    return 1;
}

static int perm_is_solution(const int* s, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int dc = s[i] - s[j];
            if (dc < 0) dc = -dc;
            if (dc == 0 || dc == j - i) return 0;
        }
    return 1;
}

/*
 * Brute force over permutations: rows 0..k-1 take the prefix, rows k..n-1 run
 * over every ordering of the remaining columns; each full assignment is checked
 * pairwise against the definition.  For n <= 11 only.
 */
int oq_brute_count(int n, int k, const int* prefix, uint64_t* count) {
    if (!valid_nk(n, k) || n > 11 || !count || (k > 0 && !prefix)) return OQ_EINVAL;
    int s[OQ_MAXN], used[OQ_MAXN] = {0};
    for (int r = 0; r < k; ++r) {
        if (prefix[r] < 0 || prefix[r] >= n || used[prefix[r]]) { *count = 0; return OQ_OK; }
        used[prefix[r]] = 1;
        s[r] = prefix[r];
    }
    int m = 0, rest[OQ_MAXN];
    for (int c = 0; c < n; ++c)
        if (!used[c]) rest[m++] = c;         /* ascending: the first permutation */
    uint64_t total = 0;
    do {
        for (int i = 0; i < m; ++i) s[k + i] = rest[i];
        total += (uint64_t)perm_is_solution(s, n);
    } while (next_perm(rest, m));
    *count = total;
    return OQ_OK;
}

/* --------------------------------------------------------------- frontier -- */

typedef struct {
    int n, k;
    int* prefixes;        /* out: len * k ints, or NULL                   */
    uint8_t* weights;     /* out: len bytes, or NULL                      */
    uint64_t cap, len;    /* capacity in prefixes; prefixes emitted       */
    int cur[OQ_MAXN];
} frontier_ctx;

static void emit(frontier_ctx* f, int w) {
    if (f->len < f->cap) {
        if (f->prefixes) memcpy(f->prefixes + f->len * (uint64_t)f->k, f->cur, sizeof(int) * f->k);
        if (f->weights) f->weights[f->len] = (uint8_t)w;
    }
    f->len++;
}

/* Rows row..k-1 unrestricted, columns ascending; emit at depth k. */
static void extend(frontier_ctx* f, board_t* b, int row, int w) {
    if (row == f->k) { emit(f, w); return; }
    for (int c = 0; c < f->n; ++c) {
        if (!board_free(b, row, c)) continue;
        f->cur[row] = c;
        board_set(b, row, c, 1);
        extend(f, b, row + 1, w);
        board_set(b, row, c, 0);
    }
}

/*
 * Symmetry-reduced prefixes of length k in lexicographic order (Section 1 and
 * its footnote): row 0 in columns [0, n/2) with weight 2; for odd n the centre
 * column n/2, then (k >= 2) row 1 in columns [0, n/2 - 2] with weight 2, or
 * (k == 1) the centre prefix alone with weight 1.  k == 0 is the empty prefix
 * with weight 1.  With prefixes == NULL or cap == 0 only the size is returned.
 */
int oq_frontier(int n, int k, int* prefixes, uint8_t* weights, uint64_t cap, uint64_t* out_len) {
    if (!valid_nk(n, k) || !out_len) return OQ_EINVAL;
    frontier_ctx f;
    memset(&f, 0, sizeof(f));
    f.n = n; f.k = k; f.prefixes = prefixes; f.weights = weights;
    f.cap = (prefixes || weights) ? cap : 0;
    board_t b;
    board_init(&b, n);
    if (k == 0) {
        emit(&f, 1);
    } else {
        int half = n / 2;
        for (int c0 = 0; c0 < half; ++c0) {
            f.cur[0] = c0;
            board_set(&b, 0, c0, 1);
            extend(&f, &b, 1, 2);
            board_set(&b, 0, c0, 0);
        }
        if (n % 2 == 1) {
            int m = half;
            f.cur[0] = m;
            board_set(&b, 0, m, 1);
            if (k == 1) {
                emit(&f, 1);
            } else {
                for (int c1 = 0; c1 <= m - 2; ++c1) {
                    if (!board_free(&b, 1, c1)) continue;
                    f.cur[1] = c1;
                    board_set(&b, 1, c1, 1);
                    extend(&f, &b, 2, 2);
                    board_set(&b, 1, c1, 0);
                }
            }
            board_set(&b, 0, m, 0);
        }
    }
    *out_len = f.len;
    if ((prefixes || weights) && f.len > cap) return OQ_ERANGE;
    return OQ_OK;
}

/*
 * The (cols, ld, rd) attack masks that a prefix casts on row k, by definition:
 * the queen at (i, c_i) attacks (k, c_i) down its column, (k, c_i + (k - i))
 * along one diagonal and (k, c_i - (k - i)) along the other; squares off the
 * board are dropped.  Bit j stands for column j.
 */
int oq_prefix_masks(int n, int k, const int* prefix, uint32_t* cols, uint32_t* ld, uint32_t* rd) {
    if (!valid_nk(n, k) || !cols || !ld || !rd || (k > 0 && !prefix)) return OQ_EINVAL;
    uint32_t C = 0, L = 0, R = 0;
    for (int i = 0; i < k; ++i) {
        int c = prefix[i], d = k - i;
        if (c < 0 || c >= n) return OQ_EINVAL;
        C |= (uint32_t)1 << c;
        if (c + d < n) L |= (uint32_t)1 << (c + d);
        if (c - d >= 0) R |= (uint32_t)1 << (c - d);
    }
    *cols = C; *ld = L; *rd = R;
    return OQ_OK;
}

/* Attack masks of m prefixes of length k (oq_prefix_masks applied to each). */
int oq_prefixes_masks(int n, int k, const int* prefixes, uint64_t m, uint32_t* cols,
                      uint32_t* ld, uint32_t* rd) {
    if (!valid_nk(n, k) || !cols || !ld || !rd || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    for (uint64_t i = 0; i < m; ++i) {
        int rc = oq_prefix_masks(n, k, prefixes + i * (uint64_t)k, cols + i, ld + i, rd + i);
        if (rc != OQ_OK) return rc;
    }
    return OQ_OK;
}

/* ------------------------------------------------- many prefixes, threaded -- */

typedef struct {
    int n, k;
    const int* prefixes;
    uint64_t m;
    uint64_t* counts;
    uint64_t* nodes;
    uint64_t next;           /* shared work index (atomic)        */
} pool_ctx;

static void* pool_worker(void* arg) {
    pool_ctx* p = (pool_ctx*)arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
        if (i >= p->m) break;
        uint64_t c = 0, nd = 0;
        oq_count_prefix(p->n, p->k, p->prefixes + i * (uint64_t)p->k, &c, &nd);
        p->counts[i] = c;
        if (p->nodes) p->nodes[i] = nd;
    }
    return NULL;
}

/*
 * Completions (and nodes) of m prefixes of length k.  Threads only spread the
 * prefixes; each prefix is counted single-threaded, so the results do not
 * depend on the thread count.
 */
int oq_count_prefixes(int n, int k, const int* prefixes, uint64_t m, int threads,
                      uint64_t* counts, uint64_t* nodes) {
    if (!valid_nk(n, k) || !counts || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    pool_ctx p = { n, k, prefixes, m, counts, nodes, 0 };
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (threads == 1 || m < 2) {
        pool_worker(&p);
        return OQ_OK;
    }
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, pool_worker, &p) == 0) ++started;
    if (started == 0) pool_worker(&p);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    return OQ_OK;
}

/* ============================================ second search: n kings ====== */
/*
 * Hertzsprung's problem: the number of ways to put n kings on an n x n board,
 * one per row and one per column, no two attacking, i.e. the permutations s
 * of 0..n-1 with |s(i) - s(i+1)| != 1 for every i.  It is the second depth-
 * first search run on the same lane-stack machinery (the paper's conclusion:
 * any DFS with many subproblems, an iterative stack form and frames of more
 * than one word).  A king attacks only the adjacent row, so a board is the
 * set of used columns plus the column of the last placed king.  Prefixes,
 * weights, order and the node unit follow the queens oracle: row 0 in
 * [0, n/2) with weight 2 (mirror symmetry s -> n-1-s); for odd n the centre
 * column with row 1 in [0, n/2 - 2] (the centre and its neighbours are
 * excluded by the rules) with weight 2, or alone with weight 1 when k = 1.
 *
 * Pins (tests/): permutation brute force (n <= 10), the recurrence that the
 * counts obey (a(n) = (n+1)a(n-1) - (n-2)a(n-2) - (n-5)a(n-3) + (n-3)a(n-4)),
 * and the weighted frontier totals against the unreduced counts.
 */

typedef struct {
    int n;
    unsigned char col[OQ_MAXN];    /* column j used                             */
    int last;                      /* column of the king in the row above, or -1 */
} kboard_t;

static int kboard_free(const kboard_t* b, int c) {
    if (b->col[c]) return 0;
    if (b->last >= 0 && (c == b->last - 1 || c == b->last + 1)) return 0;
    return 1;
}

/* Completions of rows row..n-1; placements in rows <= n-2 are nodes. */
static uint64_t kboard_complete(kboard_t* b, int row, uint64_t* nodes) {
    if (row == b->n) return 1;
    uint64_t total = 0;
    const int above = b->last;
    for (int c = 0; c < b->n; ++c) {
        if (!kboard_free(b, c)) continue;
        if (row <= b->n - 2) ++*nodes;
        b->col[c] = 1;
        b->last = c;
        total += kboard_complete(b, row + 1, nodes);
        b->last = above;
        b->col[c] = 0;
    }
    return total;
}

/* Place a prefix on an empty board; 0 if it breaks a rule. */
static int kboard_place_prefix(kboard_t* b, int k, const int* prefix) {
    for (int r = 0; r < k; ++r) {
        int c = prefix[r];
        if (c < 0 || c >= b->n || !kboard_free(b, c)) return 0;
        b->col[c] = 1;
        b->last = c;
    }
    return 1;
}

static void kboard_init(kboard_t* b, int n) {
    memset(b, 0, sizeof(*b));
    b->n = n;
    b->last = -1;
}

int oqk_count_prefix(int n, int k, const int* prefix, uint64_t* count, uint64_t* nodes) {
    if (!valid_nk(n, k) || !count || (k > 0 && !prefix)) return OQ_EINVAL;
    kboard_t b;
    kboard_init(&b, n);
    uint64_t nd = 0;
    *count = kboard_place_prefix(&b, k, prefix) ? kboard_complete(&b, k, &nd) : 0;
    if (nodes) *nodes = nd;
    return OQ_OK;
}

/* Every ordering of the free columns after the prefix, checked pairwise. */
int oqk_brute_count(int n, int k, const int* prefix, uint64_t* count) {
    if (!valid_nk(n, k) || n > 11 || !count || (k > 0 && !prefix)) return OQ_EINVAL;
    int s[OQ_MAXN], used[OQ_MAXN] = {0};
    for (int r = 0; r < k; ++r) {
        if (prefix[r] < 0 || prefix[r] >= n || used[prefix[r]]) { *count = 0; return OQ_OK; }
        used[prefix[r]] = 1;
        s[r] = prefix[r];
    }
    int m = 0, rest[OQ_MAXN];
    for (int c = 0; c < n; ++c)
        if (!used[c]) rest[m++] = c;
    uint64_t total = 0;
    do {
        for (int i = 0; i < m; ++i) s[k + i] = rest[i];
        int ok = 1;
        for (int i = 0; i + 1 < n && ok; ++i) {
            int d = s[i] - s[i + 1];
            if (d == 1 || d == -1) ok = 0;
        }
        total += (uint64_t)ok;
    } while (next_perm(rest, m));
    *count = total;
    return OQ_OK;
}

typedef struct {
    frontier_ctx f;
    kboard_t b;
} kfrontier_ctx;

static void kextend(kfrontier_ctx* x, int row, int w) {
    if (row == x->f.k) { emit(&x->f, w); return; }
    const int above = x->b.last;
    for (int c = 0; c < x->f.n; ++c) {
        if (!kboard_free(&x->b, c)) continue;
        x->f.cur[row] = c;
        x->b.col[c] = 1;
        x->b.last = c;
        kextend(x, row + 1, w);
        x->b.last = above;
        x->b.col[c] = 0;
    }
}

/* Symmetry-reduced king prefixes of length k, lexicographic (as oq_frontier). */
int oqk_frontier(int n, int k, int* prefixes, uint8_t* weights, uint64_t cap, uint64_t* out_len) {
    if (!valid_nk(n, k) || !out_len) return OQ_EINVAL;
    kfrontier_ctx x;
    memset(&x, 0, sizeof(x));
    x.f.n = n; x.f.k = k; x.f.prefixes = prefixes; x.f.weights = weights;
    x.f.cap = (prefixes || weights) ? cap : 0;
    kboard_init(&x.b, n);
    if (k == 0) {
        emit(&x.f, 1);
    } else {
        const int half = n / 2;
        for (int c0 = 0; c0 < half; ++c0) {
            x.f.cur[0] = c0;
            x.b.col[c0] = 1;
            x.b.last = c0;
            kextend(&x, 1, 2);
            x.b.last = -1;
            x.b.col[c0] = 0;
        }
        if (n % 2 == 1) {
            const int m = half;
            x.f.cur[0] = m;
            x.b.col[m] = 1;
            x.b.last = m;
            if (k == 1) {
                emit(&x.f, 1);
            } else {
                for (int c1 = 0; c1 <= m - 2; ++c1) {
                    if (!kboard_free(&x.b, c1)) continue;
                    x.f.cur[1] = c1;
                    x.b.col[c1] = 1;
                    x.b.last = c1;
                    kextend(&x, 2, 2);
                    x.b.last = m;
                    x.b.col[c1] = 0;
                }
            }
        }
    }
    *out_len = x.f.len;
    if ((prefixes || weights) && x.f.len > cap) return OQ_ERANGE;
    return OQ_OK;
}

/*
 * The masks a king prefix casts on row k, by definition: every placed king
 * blocks its column; the king of row k-1 also blocks (k, c+1) (in `ld`) and
 * (k, c-1) (in `rd`), squares off the board dropped.  Bit j is column j.
 */
int oqk_prefixes_masks(int n, int k, const int* prefixes, uint64_t m, uint32_t* cols,
                       uint32_t* ld, uint32_t* rd) {
    if (!valid_nk(n, k) || !cols || !ld || !rd || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    for (uint64_t i = 0; i < m; ++i) {
        const int* p = prefixes + i * (uint64_t)k;
        uint32_t C = 0, L = 0, R = 0;
        for (int r = 0; r < k; ++r) {
            if (p[r] < 0 || p[r] >= n) return OQ_EINVAL;
            C |= (uint32_t)1 << p[r];
        }
        if (k > 0) {
            const int c = p[k - 1];
            if (c + 1 < n) L = (uint32_t)1 << (c + 1);
            if (c - 1 >= 0) R = (uint32_t)1 << (c - 1);
        }
        cols[i] = C; ld[i] = L; rd[i] = R;
    }
    return OQ_OK;
}

typedef struct {
    int n, k;
    const int* prefixes;
    uint64_t m;
    uint64_t* counts;
    uint64_t* nodes;
    uint64_t next;
} kpool_ctx;

static void* kpool_worker(void* arg) {
    kpool_ctx* p = (kpool_ctx*)arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
        if (i >= p->m) break;
        uint64_t c = 0, nd = 0;
        oqk_count_prefix(p->n, p->k, p->prefixes + i * (uint64_t)p->k, &c, &nd);
        p->counts[i] = c;
        if (p->nodes) p->nodes[i] = nd;
    }
    return NULL;
}

/* Completions (and nodes) of m king prefixes; threads only spread prefixes. */
int oqk_count_prefixes(int n, int k, const int* prefixes, uint64_t m, int threads,
                       uint64_t* counts, uint64_t* nodes) {
    if (!valid_nk(n, k) || !counts || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    kpool_ctx p = { n, k, prefixes, m, counts, nodes, 0 };
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (threads == 1 || m < 2) {
        kpool_worker(&p);
        return OQ_OK;
    }
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, kpool_worker, &p) == 0) ++started;
    if (started == 0) kpool_worker(&p);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    return OQ_OK;
}

/* ================================= third search: permanents of 0/1 matrices */
/*
 * The number of permutations s of 0..n-1 with a[r][s(r)] = 1 for every row r:
 * the permanent of the 0/1 matrix a, a combinatorial permutation count of the
 * kind the paper's conclusion names as a target of the same method.  It is
 * run on the GPU with a frame of two words (the used columns and the untried
 * columns of the row being filled) and a different leaf rule: the last two
 * rows are never entered; their completions are counted in closed form.
 * Here a board is the
 * array of used columns and the matrix itself, n x n bytes in row-major order
 * (a[r * n + c] != 0: row r may take column c); prefixes fix the column of
 * rows 0..k-1 (no symmetry reduction: every weight is 1), in lexicographic
 * order.  A node is one placement in rows k..n-3 (the rows the search enters;
 * placements in the last two rows belong to the leaf count).
 *
 * Pins (tests/): permutation brute force, Ryser's inclusion-exclusion formula,
 * the all-ones matrix (n!), permutation matrices (1), the tridiagonal band
 * (Fibonacci numbers), and the frontier totals against the whole count.
 */

typedef struct {
    int n;
    const uint8_t* a;              /* the matrix, row-major                     */
    unsigned char used[OQ_MAXN];   /* column c taken by an earlier row          */
} pboard_t;

static int pboard_allows(const pboard_t* b, int r, int c) {
    return b->a[r * b->n + c] != 0 && !b->used[c];
}

/* Completions of rows row..n-1; placements in rows <= n-3 are nodes. */
static uint64_t pboard_complete(pboard_t* b, int row, uint64_t* nodes) {
    if (row == b->n) return 1;
    uint64_t total = 0;
    for (int c = 0; c < b->n; ++c) {
        if (!pboard_allows(b, row, c)) continue;
        if (row <= b->n - 3) ++*nodes;
        b->used[c] = 1;
        total += pboard_complete(b, row + 1, nodes);
        b->used[c] = 0;
    }
    return total;
}

static int pboard_init(pboard_t* b, int n, const uint8_t* a) {
    memset(b, 0, sizeof(*b));
    b->n = n;
    b->a = a;
    return a != NULL;
}

/* Place a prefix on an empty board; 0 if a row does not allow its column or a
 * column repeats. */
static int pboard_place_prefix(pboard_t* b, int k, const int* prefix) {
    for (int r = 0; r < k; ++r) {
        const int c = prefix[r];
        if (c < 0 || c >= b->n || !pboard_allows(b, r, c)) return 0;
        b->used[c] = 1;
    }
    return 1;
}

int oqp_count_prefix(int n, const uint8_t* a, int k, const int* prefix, uint64_t* count,
                     uint64_t* nodes) {
    if (!valid_nk(n, k) || !count || (k > 0 && !prefix)) return OQ_EINVAL;
    pboard_t b;
    if (!pboard_init(&b, n, a)) return OQ_EINVAL;
    uint64_t nd = 0;
    *count = pboard_place_prefix(&b, k, prefix) ? pboard_complete(&b, k, &nd) : 0;
    if (nodes) *nodes = nd;
    return OQ_OK;
}

typedef struct {
    frontier_ctx f;
    pboard_t b;
} pfrontier_ctx;

static void pextend(pfrontier_ctx* x, int row) {
    if (row == x->f.k) { emit(&x->f, 1); return; }
    for (int c = 0; c < x->f.n; ++c) {
        if (!pboard_allows(&x->b, row, c)) continue;
        x->f.cur[row] = c;
        x->b.used[c] = 1;
        pextend(x, row + 1);
        x->b.used[c] = 0;
    }
}

/* Every prefix of length k (rows 0..k-1 in allowed, distinct columns),
 * lexicographic; weights, when asked for, are all 1. */
int oqp_frontier(int n, const uint8_t* a, int k, int* prefixes, uint8_t* weights,
                 uint64_t cap, uint64_t* out_len) {
    if (!valid_nk(n, k) || !out_len) return OQ_EINVAL;
    pfrontier_ctx x;
    memset(&x, 0, sizeof(x));
    x.f.n = n; x.f.k = k; x.f.prefixes = prefixes; x.f.weights = weights;
    x.f.cap = (prefixes || weights) ? cap : 0;
    if (!pboard_init(&x.b, n, a)) return OQ_EINVAL;
    pextend(&x, 0);
    *out_len = x.f.len;
    if ((prefixes || weights) && x.f.len > cap) return OQ_ERANGE;
    return OQ_OK;
}

/* The used-column set of each prefix (bit c = some row of the prefix took
 * column c). */
int oqp_prefixes_cols(int n, int k, const int* prefixes, uint64_t m, uint32_t* cols) {
    if (!valid_nk(n, k) || !cols || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    for (uint64_t i = 0; i < m; ++i) {
        const int* p = prefixes + i * (uint64_t)k;
        uint32_t C = 0;
        for (int r = 0; r < k; ++r) {
            if (p[r] < 0 || p[r] >= n) return OQ_EINVAL;
            C |= (uint32_t)1 << p[r];
        }
        cols[i] = C;
    }
    return OQ_OK;
}

typedef struct {
    int n, k;
    const uint8_t* a;
    const int* prefixes;
    uint64_t m;
    uint64_t* counts;
    uint64_t* nodes;
    uint64_t next;
} ppool_ctx;

static void* ppool_worker(void* arg) {
    ppool_ctx* p = (ppool_ctx*)arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
        if (i >= p->m) break;
        uint64_t c = 0, nd = 0;
        oqp_count_prefix(p->n, p->a, p->k, p->prefixes + i * (uint64_t)p->k, &c, &nd);
        p->counts[i] = c;
        if (p->nodes) p->nodes[i] = nd;
    }
    return NULL;
}

/* Completions (and nodes) of m prefixes; threads only spread prefixes. */
int oqp_count_prefixes(int n, const uint8_t* a, int k, const int* prefixes, uint64_t m,
                       int threads, uint64_t* counts, uint64_t* nodes) {
    if (!valid_nk(n, k) || !a || !counts || (m > 0 && k > 0 && !prefixes)) return OQ_EINVAL;
    ppool_ctx p = { n, k, a, prefixes, m, counts, nodes, 0 };
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (threads == 1 || m < 2) {
        ppool_worker(&p);
        return OQ_OK;
    }
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, ppool_worker, &p) == 0) ++started;
    if (started == 0) ppool_worker(&p);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    return OQ_OK;
}

/*
 * The permanent by Ryser's inclusion-exclusion formula (H. J. Ryser,
 * Combinatorial Mathematics, 1963), a second and independent way to the same
 * number: perm(a) = (-1)^n sum over column sets S of (-1)^|S| prod_r
 * (number of columns of S that row r allows).  Every term is below
 * n^n <= 20^20 < 2^87, so 128-bit signed sums are exact for n <= 20.
 */
int oqp_ryser(int n, const uint8_t* a, uint64_t* count) {
    if (n < 1 || n > 20 || !a || !count) return OQ_EINVAL;
    __int128 total = 0;
    for (uint32_t s = 0; s < (1u << n); ++s) {
        __int128 prod = 1;
        int size = 0;
        for (int c = 0; c < n; ++c) size += (s >> c) & 1u;
        for (int r = 0; r < n && prod != 0; ++r) {
            int in_s = 0;
            for (int c = 0; c < n; ++c)
                if (((s >> c) & 1u) && a[r * n + c]) ++in_s;
            prod *= in_s;
        }
        total += ((n - size) % 2 == 0) ? prod : -prod;
    }
    if (total < 0) return OQ_ERANGE;          /* impossible for a 0/1 matrix */
    *count = (uint64_t)total;
    return OQ_OK;
}
