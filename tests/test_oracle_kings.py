"""The kings oracle (the second search run on the lane-stack engine) against
what pins it: permutation brute force, the recurrence its counts obey, the
weighted frontier identity and the definition of the masks."""
import itertools

import numpy as np
import pytest

import oracle


def _rec(a, n):
    """a(n) from a(n-1..n-4) by the recurrence of the king-placement counts
    (Hertzsprung's problem): (n+1)a(n-1) - (n-2)a(n-2) - (n-5)a(n-3) + (n-3)a(n-4)."""
    return (n + 1) * a[n - 1] - (n - 2) * a[n - 2] - (n - 5) * a[n - 3] + (n - 3) * a[n - 4]


def _weighted_total(n, k, threads=8):
    pre, w = oracle.kings_frontier(n, k)
    counts, _ = oracle.kings_count_prefixes(n, pre, threads=threads)
    return int((counts * w.astype(np.uint64)).sum())


@pytest.mark.parametrize("n", range(1, 10))
def test_brute_force_equals_backtracking(n):
    assert oracle.kings(n)[0] == oracle.kings_brute_count(n)


def test_brute_force_by_python_permutations():
    for n in range(1, 8):
        want = sum(all(abs(p[i] - p[i + 1]) != 1 for i in range(n - 1))
                   for p in itertools.permutations(range(n)))
        assert oracle.kings(n)[0] == want, n


def test_counts_follow_the_recurrence():
    a = {0: 1}
    for n in range(1, 13):
        a[n] = _weighted_total(n, min(n, 3))
    assert [a[n] for n in range(1, 5)] == [1, 0, 0, 2]
    for n in range(4, 13):
        assert a[n] == _rec(a, n), n


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9, 10, 11])
def test_weighted_frontier_equals_unreduced_count(n):
    full = oracle.kings(n)[0]
    for k in range(1, min(n, 5) + 1):
        assert _weighted_total(n, k) == full, (n, k)


def test_prefix_counts_vs_brute_random():
    rng = np.random.default_rng(7)
    for n in (6, 8, 9, 10):
        for k in (1, 2, 3, 5):
            pre, _ = oracle.kings_frontier(n, k)
            for i in rng.choice(len(pre), min(20, len(pre)), replace=False):
                c, _ = oracle.kings_count_prefixes(n, pre[i:i + 1])
                assert int(c[0]) == oracle.kings_brute_count(n, list(pre[i])), (n, list(pre[i]))


def test_frontier_order_and_symmetry():
    for n in (6, 7, 9):
        for k in (1, 2, 3):
            pre, w = oracle.kings_frontier(n, k)
            rows = [tuple(p) for p in pre]
            assert rows == sorted(rows)
            half = n // 2
            for p, wt in zip(rows, w):
                assert p[0] <= half
                if p[0] < half:
                    assert wt == 2
                else:                                   # odd n, centre column
                    assert n % 2 == 1
                    assert (k == 1 and wt == 1) or (p[1] <= half - 2 and wt == 2)
                for i in range(k - 1):                  # every prefix obeys the rule
                    assert abs(p[i] - p[i + 1]) > 1
                assert len(set(p)) == k


def test_masks_by_definition():
    rng = np.random.default_rng(11)
    for n in (5, 8, 12, 17):
        for k in (1, 2, 4):
            pre, _ = oracle.kings_frontier(n, k)
            sel = pre[rng.choice(len(pre), min(50, len(pre)), replace=False)]
            cols, ld, rd = oracle.kings_prefixes_masks(n, sel)
            for p, c, l, r in zip(sel, cols, ld, rd):
                free = {j for j in range(n) if j not in p and abs(j - p[-1]) != 1}
                blocked = int(c) | int(l) | int(r)
                assert {j for j in range(n) if not (blocked >> j) & 1} == free


def test_nodes_count_placements_above_the_last_row():
    # n = 4: the two solutions 1302 and 2031; every placement in rows 0..2 below
    # the empty prefix that the rules allow is a node
    total, nodes = oracle.kings(4)
    manual = 0
    for k in range(1, 4):
        manual += sum(1 for p in itertools.permutations(range(4), k)
                      if all(abs(p[i] - p[i + 1]) != 1 for i in range(k - 1)))
    assert (total, nodes) == (2, manual)
