"""GPU parity: the HIP DFS kernels against the CPU oracle, bit for bit.

Every expected value comes from the oracle (live, or stored by
tests/golden/make_golden.py, which calls only the oracle) or from the published
counts in tests/golden/known_counts.txt.  All calls go through the C-ABI.
"""
import hashlib

import numpy as np
import pytest

import oracle
from conftest import read_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-parity]", *a, flush=True)


def _golden_runs():
    return {(int(r[0]), int(r[1])): r for r in read_table("oracle_runs.txt")}


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _triples_from_prefixes(n, prefixes):
    c, l, r = oracle.prefixes_masks(n, prefixes)
    return _dev(c), _dev(l), _dev(r)


@pytest.mark.parametrize("mode", ["plain", "persistent"])
def test_small_boards_every_depth(mode, known_counts):
    nq = _nq()
    for n in range(1, 13):
        for k in range(1, n + 1):
            _say("count", n, k, mode)
            assert nq.count(n, depth=k, mode=mode) == known_counts[n], (n, k, mode)


def test_automatic_depth(known_counts):
    """depth 0: the library picks the pre-placement (deep ones by device expansion)."""
    nq = _nq()
    for n in range(1, 17):
        _say("auto depth", n)
        assert nq.count(n) == known_counts[n], n


@pytest.mark.parametrize("mode", ["plain", "persistent"])
def test_n14_depth3_per_subproblem(mode):
    nq = _nq()
    _say("n14 k3", mode)
    total, counts = nq.count(14, depth=3, mode=mode, counts=True)
    pre, w = oracle.frontier(14, 3)
    ref, _ = oracle.count_prefixes(14, pre, threads=8)
    assert total == 365596
    np.testing.assert_array_equal(counts, ref)


def test_n17_depth5_persistent_per_subproblem():
    nq = _nq()
    n, k = 17, 5
    _say("n17 k5 persistent")
    total, counts = nq.count(n, depth=k, mode="persistent", counts=True)
    g = _golden_runs()[(n, k)]
    assert len(counts) == int(g[2])
    assert total == int(g[3]) == 95815104
    assert _digest(counts) == g[5]
    # a seeded sample re-counted live by the oracle, element by element
    pre, _ = oracle.frontier(n, k)
    idx = np.random.default_rng(17).choice(len(pre), 200, replace=False)
    ref, _ = oracle.count_prefixes(n, pre[idx], threads=8)
    np.testing.assert_array_equal(counts[idx], ref)


@pytest.mark.parametrize("claim", [1, 5, 63, 64, 100, 1000, 1 << 20])
def test_block_claims_per_subproblem(claim):
    """Persistent refills from per-wave claimed blocks of any size (smaller and
    larger than a wave, and than the frontier), both claim orders."""
    nq = _nq()
    pre, _ = oracle.frontier(14, 3)
    ref, _ = oracle.count_prefixes(14, pre, threads=8)
    for forward in (False, True):
        _say("n14 k3 claim", claim, "forward" if forward else "reverse")
        total, counts = nq.count(14, depth=3, counts=True, claim=claim, forward=forward)
        assert total == 365596
        np.testing.assert_array_equal(counts, ref)
    _say("n17 k5 claim", claim)
    assert nq.count(17, depth=5, claim=claim) == 95815104


def test_count_subproblems_random_prefixes():
    """Random legal prefixes of every depth, including dead ones and k = n-1, n."""
    nq = _nq()
    rng = np.random.default_rng(2511)
    for n in [4, 5, 8, 11, 13, 15, 16]:
        for k in sorted({1, 2, n // 2, max(1, n - 3), n - 1, n}):
            pre_all, _ = oracle.frontier(n, k)
            if len(pre_all) == 0:
                continue
            take = rng.choice(len(pre_all), min(300, len(pre_all)), replace=False)
            pre = pre_all[np.sort(take)]
            c, l, r = _triples_from_prefixes(n, pre)
            ref, _ = oracle.count_prefixes(n, pre, threads=8)
            for mode in ("plain", "persistent"):
                _say("subproblems", n, k, mode, len(pre))
                counts, total = nq.count_subproblems(n, c, l, r, depth=k, mode=mode)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
                assert int(total.item()) == int(ref.sum())


def test_weights_and_accumulating_total():
    nq = _nq()
    n, k = 12, 4
    pre, w = oracle.frontier(n, k)
    c, l, r = _triples_from_prefixes(n, pre)
    tw = torch.from_numpy(w).cuda()
    total = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    _say("weights", n, k)
    nq.count_subproblems(n, c, l, r, weight=tw, total=total, depth=k)
    torch.cuda.synchronize()
    assert int(total.item()) == 5 + 14200


@pytest.mark.parametrize("mode", ["persistent", "plain"])
def test_totals_without_per_entry_counts(mode):
    """Totals when no per-entry result is written: uniform weights (counted per
    wave), mixed weights and no weights (counted per lane), against the oracle."""
    nq = _nq()
    n, k = 14, 3
    pre, _ = oracle.frontier(n, k)
    ref, _ = oracle.count_prefixes(n, pre, threads=8)
    ref = ref.astype(np.uint64)
    c, l, r = _triples_from_prefixes(n, pre)
    rng = np.random.default_rng(1403)
    cases = {"uniform 3": np.full(len(pre), 3, np.uint8),
             "uniform 0": np.zeros(len(pre), np.uint8),
             "mixed": rng.integers(0, 256, len(pre)).astype(np.uint8),
             "none": None}
    for name, w in cases.items():
        _say("totals", mode, name)
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        tw = None if w is None else torch.from_numpy(w).cuda()
        nq.count_subproblems(n, c, l, r, weight=tw, counts=False, total=total, depth=k,
                             mode=mode)
        torch.cuda.synchronize()
        expect = int((ref * (np.ones(len(pre), np.uint64) if w is None
                             else w.astype(np.uint64))).sum())
        assert int(total.item()) == expect, name


def test_large_boards_deep_prefixes():
    """n = 24..28 with deep prefixes: the popcount leaf test and the widest masks."""
    nq = _nq()
    rng = np.random.default_rng(28)
    for n in [24, 26, 27, 28]:
        k = n - 7
        pre = []
        while len(pre) < 64:
            p = []
            for row in range(k):
                opts = [j for j in range(n)
                        if all(p[i] != j and abs(p[i] - j) != row - i for i in range(row))]
                if not opts:
                    break
                p.append(int(rng.choice(opts)))
            if len(p) == k:
                pre.append(p)
        pre = np.array(pre, dtype=np.int32)
        c, l, r = _triples_from_prefixes(n, pre)
        ref, _ = oracle.count_prefixes(n, pre, threads=8)
        for depth in (k, 0):               # depth 0: no promise, deepest stack
            _say("large", n, k, "depth", depth)
            counts, total = nq.count_subproblems(n, c, l, r, depth=depth)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)


def test_mirror_images_count_the_same():
    nq = _nq()
    n, k = 16, 5
    pre, _ = oracle.frontier(n, k)
    mir = (n - 1 - pre).astype(np.int32)
    c, l, r = _triples_from_prefixes(n, pre)
    mc, ml, mr = _triples_from_prefixes(n, mir)
    _say("mirror", n, k)
    a, _ = nq.count_subproblems(n, c, l, r, depth=k)
    b, _ = nq.count_subproblems(n, mc, ml, mr, depth=k)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_entries_deeper_than_the_promise_are_rejected():
    nq = _nq()
    n = 12
    pre_deep, _ = oracle.frontier(n, 6)
    pre_shallow, _ = oracle.frontier(n, 2)
    c1, l1, r1 = _triples_from_prefixes(n, pre_deep[:50])
    c2, l2, r2 = _triples_from_prefixes(n, pre_shallow[:5])
    c, l, r = torch.cat([c1, c2]), torch.cat([l1, l2]), torch.cat([r1, r2])
    ref, _ = oracle.count_prefixes(n, pre_deep[:50])
    _say("promise", n)
    counts, total = nq.count_subproblems(n, c, l, r, depth=6)
    torch.cuda.synchronize()
    got = counts.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got[:50], ref)
    assert (got[50:] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    assert int(total.item()) == int(ref.sum())


def test_empty_inputs():
    nq = _nq()
    z = torch.zeros(0, dtype=torch.int32, device="cuda")
    counts, total = nq.count_subproblems(10, z, z, z)
    torch.cuda.synchronize()
    assert counts.numel() == 0 and int(total.item()) == 0
    assert nq.count(2, depth=2) == 0 and nq.count(3, depth=3) == 0


def test_n20_bench_shape():
    """The N=20 counts at depth 6 in both modes, plus a live per-entry sample."""
    nq = _nq()
    n, k = 20, 6
    for mode in ("persistent", "plain"):
        _say("n20 k6", mode)
        total, counts = nq.count(n, depth=k, mode=mode, counts=True)
        assert total == 39029188884, mode
        g = _golden_runs().get((n, k))
        if g is not None:
            assert _digest(counts) == g[5]
        pre, _ = oracle.frontier(n, k)
        idx = np.random.default_rng(20).choice(len(pre), 48, replace=False)
        ref, _ = oracle.count_prefixes(n, pre[idx], threads=16)
        np.testing.assert_array_equal(counts[idx], ref)


@pytest.mark.parametrize("n,k", [(14, 3), (17, 5), (16, 4), (12, 2), (20, 6)])
def test_node_counts_per_subproblem(n, k):
    """DFS steps of the node-counting kernel equal the oracle's nodes entry by entry
    (N=20: the node total behind the benchmark's nodes/s)."""
    nq = _nq()
    g = _golden_runs()[(n, k)]
    cols, ld, rd, w = nq.frontier(n, k)
    t = [_dev(x) for x in (cols, ld, rd)]
    nodes = torch.empty(len(cols), dtype=torch.int64, device="cuda")
    for mode in ("persistent", "plain"):
        _say("nodes", n, k, mode)
        counts, _ = nq.count_subproblems(n, *t, depth=k, mode=mode, nodes=nodes)
        torch.cuda.synchronize()
        got_nodes = nodes.cpu().numpy().view(np.uint64)
        assert int(got_nodes.sum()) == int(g[4])
        assert _digest(got_nodes) == g[6]
        assert _digest(counts.cpu().numpy().view(np.uint64)) == g[5]


@pytest.mark.parametrize("n,k,rows", [(12, 2, 1), (13, 3, 2), (16, 4, 3), (11, 2, 3), (12, 1, 3),
                                      (20, 5, 2)])
def test_device_expansion_matches_oracle_frontier(n, k, rows):
    """nq_expand of the depth-k frontier is the oracle's depth k+rows frontier
    (k >= 2, or even n: see the next test for odd n from depth 1)."""
    nq = _nq()
    cols, ld, rd, w = nq.frontier(n, k)
    t = [_dev(x) for x in (cols, ld, rd)]
    _say("expand", n, k, rows)
    oc, ol, orr, ow = nq.expand(n, rows, *t, weight=torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    rc, rl, rr, rw = oracle.frontier_masks(n, k + rows)
    np.testing.assert_array_equal(oc.cpu().numpy().view(np.uint32), rc)
    np.testing.assert_array_equal(ol.cpu().numpy().view(np.uint32), rl)
    np.testing.assert_array_equal(orr.cpu().numpy().view(np.uint32), rr)
    np.testing.assert_array_equal(ow.cpu().numpy(), rw)


def test_count_with_device_expansion(known_counts):
    """nq_count at depth >= 7 builds a shallow frontier and deepens it on the device."""
    nq = _nq()
    for n, k in [(12, 7), (14, 8), (16, 7)]:
        for mode in ("persistent", "plain"):
            _say("count via expansion", n, k, mode)
            total, counts = nq.count(n, depth=k, mode=mode, counts=True)
            assert total == known_counts[n]
            pre, _ = oracle.frontier(n, k)
            ref, _ = oracle.count_prefixes(n, pre, threads=8)
            np.testing.assert_array_equal(counts, ref)


@pytest.mark.parametrize("n,k", [(19, 6), (20, 7), (20, 8), (20, 10), (21, 7)])
def test_large_counts_at_tuned_depths(n, k, known_counts):
    """Full counts at the depths the autotuner chooses from (published totals);
    depth >= 7 goes through the device expansion."""
    nq = _nq()
    _say("large count", n, k)
    assert nq.count(n, depth=k, mode="persistent") == known_counts[n]


def test_benchmark_configuration():
    """The benchmark's workload, N=20 at depth 9 (812 M subproblems resident,
    built on the device, persistent launch): the total without per-entry output
    (wave-level leaf count) and, with per-entry output, the node total of the
    node-counting kernel against the oracle's (the numerator of the reported
    nodes/s); then seeded depth-9 subproblems (random legal extensions of
    oracle depth-7 prefixes) counted per entry against the oracle."""
    nq = _nq()
    n, k = 20, 9
    _say("bench config: total")
    assert nq.count(n, depth=k) == 39029188884
    nodes_ref = {(int(r[0]), int(r[1])): int(r[2]) for r in read_table("oracle_nodes.txt")}
    _say("bench config: nodes")
    cols, ld, rd, w = nq.frontier(n, 7)
    dev = [_dev(x) for x in (cols, ld, rd)]
    c, l, r, tw = nq.expand(n, 2, *dev, weight=torch.from_numpy(w).cuda())
    del dev
    torch.cuda.synchronize()
    assert c.numel() == 811572426
    nodes = torch.empty(c.numel(), dtype=torch.int64, device="cuda")
    _, total = nq.count_subproblems(n, c, l, r, weight=tw, depth=k, nodes=nodes)
    torch.cuda.synchronize()
    assert int(total.item()) == 39029188884
    assert int(nodes.sum().item()) == nodes_ref[(n, k)]
    del c, l, r, tw, nodes
    _say("bench config: sampled subproblems")
    pre7, _ = oracle.frontier(n, 7)
    rng = np.random.default_rng(209)
    sample = []
    while len(sample) < 256:
        p = [int(x) for x in pre7[rng.integers(len(pre7))]]
        for _row in range(2):
            free = [col for col in range(n) if _free(p, col)]
            if not free:
                break
            p.append(free[rng.integers(len(free))])
        if len(p) == 9:
            sample.append(p)
    pre9 = np.asarray(sample, dtype=np.int32)
    ref, _ = oracle.count_prefixes(n, pre9, threads=8)
    tc, tl, tr = _triples_from_prefixes(n, pre9)
    counts, _ = nq.count_subproblems(n, tc, tl, tr, depth=k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)


def _free(prefix, col):
    """True when a queen in the next row at `col` attacks none of `prefix`."""
    row = len(prefix)
    return all(c != col and abs(c - col) != row - i for i, c in enumerate(prefix))


def test_expansion_of_odd_board_from_depth_one(known_counts):
    """For odd n the depth-1 centre entry has weight 1 and an unrestricted row 1,
    so its expansion differs from the deeper frontier (which restricts row 1 and
    doubles the weight) but the weighted count is the same."""
    nq = _nq()
    n = 11
    cols, ld, rd, w = nq.frontier(n, 1)
    t = [_dev(x) for x in (cols, ld, rd)]
    oc, ol, orr, ow = nq.expand(n, 3, *t, weight=torch.from_numpy(w).cuda())
    assert oc.numel() != oracle.frontier_size(n, 4)
    counts, total = nq.count_subproblems(n, oc, ol, orr, weight=ow, depth=4)
    torch.cuda.synchronize()
    assert int(total.item()) == known_counts[n]
