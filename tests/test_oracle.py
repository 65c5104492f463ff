"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: permutation
brute force, published counts, the 5-Queens decomposition of Figure 1, the
27-Queens frontier size of the run log in Section 4.5, the Somers recurrence of
Section 2, and invariants (refinement over k, mirror symmetry, node identity).
"""
import itertools

import numpy as np
import pytest

import oracle
from conftest import read_table


# ----------------------------------------------------------------- brute force

@pytest.mark.parametrize("n", range(1, 11))
def test_brute_force_matches_published_counts(n, known_counts):
    assert oracle.brute_count(n) == known_counts[n]


@pytest.mark.parametrize("n", range(1, 11))
def test_backtracker_matches_brute_force(n):
    assert oracle.queens(n)[0] == oracle.brute_count(n)


def test_backtracker_published_counts_up_to_14(known_counts):
    for n in range(1, 15):
        assert oracle.queens(n)[0] == known_counts[n], n


@pytest.mark.parametrize("n,k", [(15, 3), (16, 4)])
def test_symmetric_frontier_totals_15_16(n, k, known_counts):
    pre, w = oracle.frontier(n, k)
    counts, _ = oracle.count_prefixes(n, pre, threads=8)
    assert int(np.sum(counts * w.astype(np.uint64))) == known_counts[n]


def _python_brute(n, prefix):
    """Tiny brute force in Python: all orderings of the free columns."""
    k = len(prefix)
    rest = [c for c in range(n) if c not in prefix]
    total = 0
    for perm in itertools.permutations(rest):
        s = list(prefix) + list(perm)
        ok = all(abs(s[i] - s[j]) != j - i for i in range(n) for j in range(i + 1, n))
        total += ok and len(set(s)) == n
    return total


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_prefix_counts_vs_python_brute(n):
    for k in range(0, n + 1):
        pre, _ = oracle.frontier(n, k)
        for p in pre:
            assert oracle.count_prefix(n, p)[0] == _python_brute(n, list(p)), (n, k, p)


def test_prefix_counts_vs_c_brute_random():
    rng = np.random.default_rng(20251112)
    for _ in range(300):
        n = int(rng.integers(4, 10))
        k = int(rng.integers(0, n + 1))
        p = [int(x) for x in rng.integers(0, n, size=k)]   # may attack: count must be 0
        assert oracle.count_prefix(n, p)[0] == oracle.brute_count(n, p), (n, p)


# ---------------------------------------------------------- 5-Queens example

def test_queens5_worked_example():
    sols = [tuple(int(x) for x in r) for r in read_table("queens5_solutions.txt")]
    assert len(sols) == 10 and len(set(sols)) == 10
    for s in sols:                                   # each fixture line is a solution
        assert oracle.count_prefix(5, s)[0] == 1
    # k = 2: five half-board prefixes then the centre prefix (2, 0), all weight 2
    pre, w = oracle.frontier(5, 2)
    assert [tuple(p) for p in pre] == [(0, 2), (0, 3), (0, 4), (1, 3), (1, 4), (2, 0)]
    assert list(w) == [2] * 6
    for p in pre:
        expect = sum(1 for s in sols if s[:2] == tuple(p))
        assert oracle.count_prefix(5, p)[0] == expect
    counts, _ = oracle.count_prefixes(5, pre)
    assert int(np.sum(counts * w.astype(np.uint64))) == 10
    # k = 1: columns 0, 1 (weight 2) and the centre column 2 (weight 1)
    pre1, w1 = oracle.frontier(5, 1)
    assert [tuple(p) for p in pre1] == [(0,), (1,), (2,)] and list(w1) == [2, 2, 1]
    c1, _ = oracle.count_prefixes(5, pre1)
    assert list(c1) == [sum(1 for s in sols if s[0] == c) for c in (0, 1, 2)]
    assert int(np.sum(c1 * w1.astype(np.uint64))) == 10


# ------------------------------------------------------------ frontier rules

def test_frontier_27_7_size_matches_run_log():
    for n, k, f in read_table("frontier_sizes.txt"):
        assert oracle.frontier_size(int(n), int(k)) == int(f)


@pytest.mark.parametrize("n", range(1, 12))
def test_refinement_every_depth(n, known_counts):
    """sum(w * Q_pi) is Q(n) at every pre-placement depth, 0 <= k <= n."""
    for k in range(0, n + 1):
        pre, w = oracle.frontier(n, k)
        assert len(pre) == oracle.frontier_size(n, k)
        counts, _ = oracle.count_prefixes(n, pre) if len(pre) else (np.zeros(0, np.uint64), None)
        assert int(np.sum(counts * w.astype(np.uint64))) == known_counts[n], (n, k)


def test_frontier_is_lexicographic_and_symmetric():
    for n in range(2, 13):
        for k in range(1, min(n, 6) + 1):
            pre, w = oracle.frontier(n, k)
            tup = [tuple(p) for p in pre]
            assert tup == sorted(tup)
            half, odd = n // 2, n % 2
            for p, wt in zip(tup, w):
                assert p[0] < half or (odd and p[0] == half)
                if odd and p[0] == half and k >= 2:
                    assert p[1] <= half - 2
                assert wt == (1 if (odd and p[0] == half and k == 1) else 2)


def test_frontier_keeps_dead_entries():
    """A prefix whose row k has no free square stays in the frontier (count 0)."""
    found = 0
    for n in range(5, 11):
        for k in range(2, n - 1):
            pre, _ = oracle.frontier(n, k)
            for p in pre:
                free = [j for j in range(n)
                        if all(p[i] != j and abs(p[i] - j) != k - i for i in range(k))]
                if not free:
                    found += 1
                    assert oracle.count_prefix(n, p) == (0, 0)
    assert found > 0


def test_edge_sizes():
    assert oracle.frontier(1, 1)[1].tolist() == [1]
    assert oracle.count_prefix(1, [0])[0] == 1
    for k in range(0, 3):
        pre, w = oracle.frontier(2, k)
        c, _ = oracle.count_prefixes(2, pre) if len(pre) else (np.zeros(0, np.uint64), 0)
        assert int(np.sum(c * w.astype(np.uint64))) == 0
    assert oracle.frontier_size(2, 2) == 0
    assert oracle.frontier_size(3, 3) == 0
    assert oracle.frontier_size(4, 0) == 1
    with pytest.raises(oracle.OracleError):
        oracle.frontier_size(32, 3)
    with pytest.raises(oracle.OracleError):
        oracle.queens(29)                     # Q(29) does not fit in 64 bits
    with pytest.raises(oracle.OracleError):
        oracle.frontier_size(8, 9)
    with pytest.raises(oracle.OracleError):
        oracle.queens(0)


@pytest.mark.parametrize("n", [4, 5, 12, 13, 28, 29, 30, 31])
def test_frontier_sizes_closed_form_at_depth_one_and_two(n):
    """Depths 1 and 2 counted by hand from the symmetry rule (Section 1 and its
    footnote), also for the boards of 29..31 that only the 128-bit totals
    reach: row 0 takes the first n//2 columns, plus the centre for odd n; a
    row-0 queen in column c attacks c-1, c, c+1 of row 1 (two of them at the
    edge), and the centre's row-1 queen takes columns 0..n//2-2, none of which
    it attacks."""
    h = n // 2
    odd = n % 2
    assert oracle.frontier_size(n, 1) == h + odd
    row1 = sum(n - (2 if c == 0 else 3) for c in range(h))
    assert oracle.frontier_size(n, 2) == row1 + odd * (h - 1)


# ------------------------------------------------------------ mask definition

def test_prefix_masks_follow_somers_recurrence():
    """The masks obey the update of Section 2 (column OR, left shift, right shift)."""
    for n in range(2, 12):
        last = (1 << n) - 1
        for k in range(0, min(n, 5)):
            pre, _ = oracle.frontier(n, k) if k else (np.zeros((1, 0), np.int32), None)
            for p in pre:
                c, l, r = oracle.prefix_masks(n, p)
                for j in range(n):
                    bit = 1 << j
                    if (c | l | r) & bit:
                        continue
                    c2, l2, r2 = oracle.prefix_masks(n, list(p) + [j])
                    assert c2 == c | bit
                    assert l2 == ((l | bit) << 1) & last
                    assert r2 == (r | bit) >> 1


def test_prefix_masks_free_squares():
    """~(cols|ld|rd) on row k is exactly the set of non-attacked squares."""
    rng = np.random.default_rng(7)
    for _ in range(500):
        n = int(rng.integers(1, 20))
        k = int(rng.integers(0, n))
        p = []
        for row in range(k):
            opts = [j for j in range(n)
                    if all(p[i] != j and abs(p[i] - j) != row - i for i in range(row))]
            if not opts:
                break
            p.append(int(rng.choice(opts)))
        k = len(p)
        c, l, r = oracle.prefix_masks(n, p)
        free = ~(c | l | r) & ((1 << n) - 1)
        for j in range(n):
            attacked = any(p[i] == j or abs(p[i] - j) == k - i for i in range(k))
            assert bool(free >> j & 1) == (not attacked)


# ---------------------------------------------------------------- invariants

def test_mirror_invariance():
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = int(rng.integers(4, 12))
        k = int(rng.integers(1, 5))
        pre, _ = oracle.frontier(n, k)
        if len(pre) == 0:
            continue
        p = pre[int(rng.integers(0, len(pre)))]
        m = [n - 1 - int(x) for x in p]
        assert oracle.count_prefix(n, p) == oracle.count_prefix(n, m)


def _python_nodes(n, prefix):
    """Legal extensions of the prefix that end in rows k..n-2 (tiny n only)."""
    k = len(prefix)
    total = 0
    for depth in range(k + 1, n):                      # last placed row = depth-1 <= n-2
        rest = [c for c in range(n) if c not in prefix]
        for ext in itertools.permutations(rest, depth - k):
            s = list(prefix) + list(ext)
            if all(abs(s[i] - s[j]) != j - i for i in range(depth) for j in range(i + 1, depth)):
                total += 1
    return total


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_node_count_brute_force(n):
    for k in range(0, n):
        pre, _ = oracle.frontier(n, k)
        for p in pre:
            assert oracle.count_prefix(n, p)[1] == _python_nodes(n, list(p)), (n, p)


@pytest.mark.parametrize("n", [8, 10, 12, 13, 14])
def test_node_identity_over_depth(n):
    """nodes(base) = nodes(k) + sum_{j=base+1..k} F(j); base 1 (even n) or 2 (odd n)."""
    base = 1 if n % 2 == 0 else 2

    def nodes(k):
        pre, _ = oracle.frontier(n, k)
        _, nd = oracle.count_prefixes(n, pre, threads=8)
        return int(nd.sum())

    ref = nodes(base)
    for k in range(base + 1, min(n - 1, 6)):
        assert ref == nodes(k) + sum(oracle.frontier_size(n, j) for j in range(base + 1, k + 1))


def test_stored_oracle_runs_cover_the_ragged_batch():
    """Every board size of the 256-instance ragged batch above 14 has a stored
    oracle run (tests/golden/oracle_runs.txt), so the GPU batch tests check
    every instance against the oracle (live for n <= 14); every stored run's
    weighted total equals the published count of its board."""
    import seeded_inputs
    stored = {int(r[0]): int(r[3]) for r in read_table("oracle_runs.txt")}
    for n in set(seeded_inputs.ragged_batch_ns()):
        assert n <= 14 or n in stored, n
    published = {int(r[0]): int(r[1]) for r in read_table("known_counts.txt")}
    for n, t in stored.items():
        assert published[n] == t, n
