"""GPU parity of the third search (permanents of 0/1 matrices, two-word frames,
two-row leaf rule): totals, per-entry counts and node counts against the
oracle, in plain and persistent launches, with the edge cases of the entry
format."""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

INVALID = (1 << 64) - 1


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-perm]", *a, flush=True)


def _matrix(n, density, seed):
    return np.array(seeded_inputs.matrix01(n, density, seeded_inputs.MATRIX_SEED + seed),
                    dtype=np.uint8)


def _dev(cols):
    return torch.from_numpy(np.ascontiguousarray(cols).view(np.int32)).cuda()


def test_totals_match_the_oracle():
    nq = _nq()
    for n in range(1, 15):
        cases = [(n, 0.5), (200 + n, 0.25)] + ([(100 + n, 0.8)] if n <= 10 else [])
        for seed, dens in cases:
            a = _matrix(n, dens, seed)
            ref = oracle.permanent(a)[0]
            for mode in ("persistent", "plain"):
                _say("total", n, dens, mode)
                assert nq.perm_count(a, mode=mode) == ref, (n, seed, mode)
                for k in sorted({1, n // 2, n - 2, n - 1, n} - {0}):
                    if k < 1:
                        continue
                    assert nq.perm_count(a, depth=k, mode=mode) == ref, (n, seed, k, mode)


def test_special_matrices():
    nq = _nq()
    fib = [1, 1]
    for _ in range(30):
        fib.append(fib[-1] + fib[-2])
    for n in (1, 2, 3, 5, 8, 11, 12):
        _say("special", n)
        assert nq.perm_count(np.ones((n, n), np.uint8)) == math.factorial(n)
        assert nq.perm_count(np.eye(n, dtype=np.uint8)) == 1
        z = np.ones((n, n), np.uint8)
        z[:, n // 2] = 0
        assert nq.perm_count(z) == 0
    for n in (4, 10, 20):
        band = np.array([[1 if abs(r - c) <= 1 else 0 for c in range(n)] for r in range(n)],
                        np.uint8)
        assert nq.perm_count(band) == fib[n], n


@pytest.mark.parametrize("n,dens,seed", [(13, 0.6, 7), (14, 0.5, 8)])
def test_per_entry_counts_and_nodes(n, dens, seed):
    nq = _nq()
    a = _matrix(n, dens, seed)
    for k in (2, 4, 6):
        pre = oracle.perm_frontier(a, k)
        ref, ref_nodes = oracle.perm_count_prefixes(a, pre, threads=8)
        cols = nq.perm_frontier(a, k)
        np.testing.assert_array_equal(cols, oracle.perm_prefixes_cols(n, pre))
        d = _dev(cols)
        nodes = torch.empty(len(cols), dtype=torch.int64, device="cuda")
        for mode, claim in (("persistent", 0), ("persistent", 1), ("persistent", 4096),
                            ("plain", 0)):
            _say("entries", n, k, mode, claim)
            counts, total = nq.perm_count_subproblems(a, d, k, nodes=nodes, mode=mode,
                                                      claim=claim)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
            np.testing.assert_array_equal(nodes.cpu().numpy().view(np.uint64), ref_nodes)
            assert int(total.item()) == int(ref.sum())


def test_edges():
    nq = _nq()
    a = _matrix(12, 0.6, 9)
    ref = oracle.permanent(a)[0]
    # an empty input, and depths that leave the last two rows, the last row or
    # nothing to the device (every entry settled without a search)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    counts, total = nq.perm_count_subproblems(a, e, 3)
    torch.cuda.synchronize()
    assert counts.numel() == 0 and int(total.item()) == 0
    for k in (10, 11, 12):
        _say("edge depth", k)
        cols = nq.perm_frontier(a, k)
        pre = oracle.perm_frontier(a, k)
        counts, total = nq.perm_count_subproblems(a, _dev(cols), k)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64),
                                      oracle.perm_count_prefixes(a, pre)[0])
        assert int(total.item()) == ref
    # entries with fewer rows assigned than the launch was promised do not fit
    # its stack: reported as UINT64_MAX and left out of the total
    shallow = nq.perm_frontier(a, 1)
    counts, total = nq.perm_count_subproblems(a, _dev(shallow), 8)
    torch.cuda.synchronize()
    assert set(counts.cpu().numpy().view(np.uint64).tolist()) <= {INVALID, 0}
    assert int(total.item()) == 0
    # a ragged input: entries of several depths in one launch, sized for the
    # shallowest
    mixed = np.concatenate([nq.perm_frontier(a, 3), nq.perm_frontier(a, 5)[::7],
                            nq.perm_frontier(a, 9)[::3]])
    pre_counts = []
    for k, step in ((3, 1), (5, 7), (9, 3)):
        pre_counts.append(oracle.perm_count_prefixes(a, oracle.perm_frontier(a, k)[::step])[0])
    counts, _ = nq.perm_count_subproblems(a, _dev(mixed), 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64),
                                  np.concatenate(pre_counts))


def test_stored_permanents_up_to_the_largest_board():
    """Every stored permanent (n = 15..20, the oracle's Ryser routine) from
    nq_perm_count at its automatic depth and at two others (6 and 8 for the
    boards of 19 and 20, whose depth-5 subtrees are too few to balance)."""
    from conftest import read_table
    nq = _nq()
    for r in read_table("perm_totals.txt"):
        n, dens, seed, value = int(r[0]), float(r[1]), int(r[2]), int(r[3])
        a = _matrix(n, dens, seed)
        _say("stored", n, dens, seed)
        assert nq.perm_count(a) == value, (n, dens, seed)
        for k in ((6, 8) if n >= 19 else (5, 8)):
            assert nq.perm_count(a, depth=k) == value, (n, dens, seed, k)


def test_largest_board_sampled_entries():
    """n = 20 (the largest board), density 1/2, the benchmark's matrix: seeded
    entries of the depth-7 frontier counted in one persistent launch over the
    whole frontier, compared with the oracle one by one."""
    nq = _nq()
    n, k = 20, 7
    a = np.array(seeded_inputs.matrix01(n, 0.5), np.uint8)
    cols = nq.perm_frontier(a, k)
    pre = oracle.perm_frontier(a, k)
    np.testing.assert_array_equal(cols, oracle.perm_prefixes_cols(n, pre))
    _say("n=20 whole frontier", len(cols))
    counts, total = nq.perm_count_subproblems(a, _dev(cols), k)
    torch.cuda.synchronize()
    got = counts.cpu().numpy().view(np.uint64)
    idx = sorted({seeded_inputs.splitmix64(0x9E20 + i) % len(cols) for i in range(24)})
    ref, _ = oracle.perm_count_prefixes(a, pre[idx], threads=8)
    np.testing.assert_array_equal(got[idx], ref)
    assert int(total.item()) == int(got.sum())
    from conftest import read_table
    stored = {(int(r[0]), float(r[1]), int(r[2])): int(r[3]) for r in read_table("perm_totals.txt")}
    assert int(total.item()) == stored[(20, 0.5, 0)]


@pytest.mark.parametrize("step", [0, 1, 2])
def test_every_inner_step_matches_the_oracle(step):
    """The three inner steps (nq_perm_set_step: plain C++, hand-scheduled, and
    the default with the children's row in the used-column word) give the
    oracle's per-entry counts, node counts and totals, persistent and plain,
    including full matrices (n!) and boards whose rows run out early."""
    nq = _nq()
    prev = nq.perm_set_step(step)
    try:
        a = _matrix(13, 0.6, 7)
        for k in (3, 5):
            pre = oracle.perm_frontier(a, k)
            ref, ref_nodes = oracle.perm_count_prefixes(a, pre, threads=8)
            d = _dev(nq.perm_frontier(a, k))
            nodes = torch.empty(len(pre), dtype=torch.int64, device="cuda")
            for mode in ("persistent", "plain"):
                _say("step", step, "entries", k, mode)
                counts, total = nq.perm_count_subproblems(a, d, k, nodes=nodes, mode=mode)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
                np.testing.assert_array_equal(nodes.cpu().numpy().view(np.uint64), ref_nodes)
                assert int(total.item()) == int(ref.sum())
        for n in (1, 2, 3, 4, 9, 12):
            assert nq.perm_count(np.ones((n, n), dtype=np.uint8)) == math.factorial(n), n
        for n, dens, seed in ((8, 0.2, 5), (14, 0.5, 3), (18, 0.4, 11), (20, 0.3, 1)):
            m = _matrix(n, dens, seed)
            _say("step", step, "total", n, dens)
            assert nq.perm_count(m) == oracle.permanent_ryser(m), (n, dens)
    finally:
        nq.perm_set_step(prev)
