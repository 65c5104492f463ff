"""The permanent oracle (third search) pinned to what mathematics fixes: the
definition by enumeration of permutations, Ryser's inclusion-exclusion
formula (H. J. Ryser, Combinatorial Mathematics, 1963), the all-ones matrix
(n!), permutation matrices (1), the tridiagonal band (Fibonacci numbers), and
the frontier totals and node identity.  The oracle's own Ryser routine (used
for boards too large for its search) is pinned the same way.  No GPU."""
import itertools
import math

import numpy as np
import pytest

import oracle
import seeded_inputs


def _brute(a, prefix=()):
    """Completions of `prefix` by enumerating every permutation."""
    n = a.shape[0]
    k = len(prefix)
    total = 0
    for s in itertools.permutations(range(n)):
        if tuple(s[:k]) != tuple(prefix):
            continue
        total += all(a[r, s[r]] for r in range(n))
    return total


def _ryser(a):
    """Ryser: perm(A) = (-1)^n sum over column subsets S of (-1)^|S| prod_r
    sum_{c in S} a[r, c]."""
    n = a.shape[0]
    total = 0
    for mask in range(1 << n):
        cols = [c for c in range(n) if mask >> c & 1]
        prod = 1
        for r in range(n):
            prod *= sum(int(a[r, c]) for c in cols)
            if prod == 0:
                break
        total += (-1) ** len(cols) * prod
    return (-1) ** n * total


def _matrix(n, density, seed):
    return np.array(seeded_inputs.matrix01(n, density, seeded_inputs.MATRIX_SEED + seed),
                    dtype=np.uint8)


@pytest.mark.parametrize("n", range(1, 8))
def test_permanent_matches_enumeration(n):
    for seed, dens in ((0, 0.5), (1, 0.7), (2, 0.3), (3, 0.9)):
        a = _matrix(n, dens, seed)
        assert oracle.permanent(a)[0] == _brute(a), (n, seed)


@pytest.mark.parametrize("n", [8, 10, 12])
def test_permanent_matches_ryser(n):
    for seed, dens in ((4, 0.5), (5, 0.75)):
        a = _matrix(n, dens, seed)
        assert oracle.permanent(a)[0] == _ryser(a), (n, seed)


def test_special_matrices():
    for n in range(1, 10):
        total, nodes = oracle.permanent(np.ones((n, n), np.uint8))
        assert total == math.factorial(n)
        # row j of the all-ones matrix is reached by n! / (n - j - 1)! placements;
        # rows 0..n-3 are nodes
        assert nodes == sum(math.perm(n, j + 1) for j in range(n - 2))
        assert oracle.permanent(np.eye(n, dtype=np.uint8))[0] == 1
        perm = np.eye(n, dtype=np.uint8)[np.roll(np.arange(n), 3 % n)]
        assert oracle.permanent(perm)[0] == 1
        z = np.ones((n, n), np.uint8)
        z[n // 2, :] = 0
        assert oracle.permanent(z)[0] == 0
    # the tridiagonal band |r - c| <= 1: its permutations are products of
    # fixed points and adjacent swaps, counted by Fibonacci numbers
    fib = [1, 1]
    for _ in range(30):
        fib.append(fib[-1] + fib[-2])
    for n in range(1, 20):
        band = np.array([[1 if abs(r - c) <= 1 else 0 for c in range(n)] for r in range(n)],
                        np.uint8)
        assert oracle.permanent(band)[0] == fib[n]


def test_frontier_is_every_prefix_in_lexicographic_order():
    for n, seed in ((5, 6), (6, 7)):
        a = _matrix(n, 0.6, seed)
        for k in range(0, n + 1):
            want = sorted({s[:k] for s in itertools.permutations(range(n))
                           if all(a[r, s[r]] for r in range(k))})
            got = [tuple(int(x) for x in p) for p in oracle.perm_frontier(a, k)]
            assert got == want, (n, k)
            assert oracle.perm_frontier_size(a, k) == len(want)


def test_prefix_counts_match_enumeration_and_rows_are_not_columns():
    """Per-prefix counts against brute force on a matrix that is not symmetric:
    reading a prefix as columns instead of rows would give other counts."""
    a = _matrix(7, 0.6, 8)
    assert not np.array_equal(a, a.T)
    for k in (1, 2, 3):
        pre = oracle.perm_frontier(a, k)
        counts, _ = oracle.perm_count_prefixes(a, pre, threads=4)
        for p, c in zip(pre, counts):
            assert int(c) == _brute(a, tuple(int(x) for x in p))
        # the same prefixes on the transposed matrix count differently, so a
        # transposed operand would fail the enumeration check above
        counts_t, _ = oracle.perm_count_prefixes(np.ascontiguousarray(a.T), pre, threads=4)
        assert counts.tolist() != counts_t.tolist()


@pytest.mark.parametrize("n", [9, 11])
def test_frontier_totals_and_node_identity(n):
    a = _matrix(n, 0.6, 9)
    total, nodes0 = oracle.permanent(a)
    sizes = [oracle.perm_frontier_size(a, j) for j in range(n + 1)]
    for k in range(0, n + 1):
        pre = oracle.perm_frontier(a, k)
        counts, nodes = oracle.perm_count_prefixes(a, pre, threads=4)
        assert int(counts.sum()) == total, k
        # nodes from row 0 = placements in rows 0..k-1 (that are nodes, i.e.
        # rows <= n-3) + nodes below every prefix
        above = sum(sizes[j + 1] for j in range(min(k, n - 2)))
        assert above + int(nodes.sum()) == nodes0, k
        assert len(pre) == sizes[k]


def test_prefix_columns_and_bad_arguments():
    cols = oracle.perm_prefixes_cols(6, np.array([[0, 2, 5], [1, 3, 4]], np.int32))
    assert cols.tolist() == [0b100101, 0b011010]
    with pytest.raises(oracle.OracleError):
        oracle.permanent(np.ones((3, 4), np.uint8))
    # a prefix with a column off the board, a repeated column or a forbidden
    # entry has no completion
    bad = np.array([[0, 9], [1, 1], [0, 1]], np.int32)
    a = np.ones((4, 4), np.uint8)
    a[1, 1] = 0
    assert oracle.perm_count_prefixes(a, bad)[0].tolist() == [0, 0, 0]


def test_oracle_ryser_routine():
    """oracle.permanent_ryser against the search, the formula retyped here in
    Python, and the closed forms up to n = 20."""
    for n in range(1, 13):
        for seed, dens in ((300 + n, 0.5), (400 + n, 0.8)):
            a = _matrix(n, dens, seed)
            assert oracle.permanent_ryser(a) == oracle.permanent(a)[0], (n, seed)
            if n <= 9:
                assert oracle.permanent_ryser(a) == _ryser(a)
    fib = [1, 1]
    for _ in range(30):
        fib.append(fib[-1] + fib[-2])
    for n in (1, 5, 13, 17, 20):
        assert oracle.permanent_ryser(np.ones((n, n), np.uint8)) == math.factorial(n)
        assert oracle.permanent_ryser(np.eye(n, dtype=np.uint8)) == 1
        band = np.array([[1 if abs(r - c) <= 1 else 0 for c in range(n)] for r in range(n)],
                        np.uint8)
        assert oracle.permanent_ryser(band) == fib[n]
    with pytest.raises(oracle.OracleError):
        oracle.permanent_ryser(np.ones((21, 21), np.uint8))


def test_stored_permanents_are_the_oracles():
    """tests/golden/perm_totals.txt (written by make_golden.py --perm): recomputed
    by the Ryser routine up to n = 18, and by the search up to n = 15."""
    from conftest import read_table
    rows = read_table("perm_totals.txt")
    assert {(int(r[0]), float(r[1])) for r in rows} >= {(20, 0.5), (20, 0.3)}
    for n, dens, seed, value in ((int(r[0]), float(r[1]), int(r[2]), int(r[3])) for r in rows):
        if n > 18:
            continue
        a = _matrix(n, dens, seed)
        assert oracle.permanent_ryser(a) == value
        if n <= 15:
            assert oracle.permanent(a)[0] == value
