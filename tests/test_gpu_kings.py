"""GPU parity of the second search on the lane-stack engine: n non-attacking
kings, one per row and column (NQ_FLAG_KINGS).  Totals against the counts'
recurrence (pinned against the oracle in test_oracle_kings.py), per-subproblem
counts and node counts against the kings oracle, element by element."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-kings]", *a, flush=True)


def _kings_counts(upto):
    """a(n) by the recurrence of the king-placement counts from a(0..3) = 1, 1, 0, 0."""
    a = {0: 1, 1: 1, 2: 0, 3: 0}
    for n in range(4, upto + 1):
        a[n] = (n + 1) * a[n - 1] - (n - 2) * a[n - 2] - (n - 5) * a[n - 3] + (n - 3) * a[n - 4]
    return a


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def test_small_boards_every_depth():
    nq = _nq()
    a = _kings_counts(12)
    for mode in ("plain", "persistent"):
        _say("small boards", mode)
        for n in range(1, 11):
            for k in range(1, n + 1):
                assert nq.count(n, depth=k, mode=mode, kings=True) == a[n], (n, k, mode)


def test_automatic_depth_up_to_16():
    nq = _nq()
    a = _kings_counts(16)
    for n in range(1, 17):
        _say("auto depth", n)
        assert nq.count(n, kings=True) == a[n], n


@pytest.mark.parametrize("n,k", [(12, 4), (13, 5), (14, 6)])
def test_per_subproblem_counts(n, k):
    nq = _nq()
    pre, w = oracle.kings_frontier(n, k)
    idx = np.sort(np.random.default_rng(n * 100 + k).choice(len(pre), min(300, len(pre)),
                                                            replace=False))
    ref, _ = oracle.kings_count_prefixes(n, pre[idx], threads=8)
    for mode in ("persistent", "plain"):
        _say("per subproblem", n, k, mode)
        total, counts = nq.count(n, depth=k, mode=mode, counts=True, kings=True)
        assert total == _kings_counts(n)[n]
        np.testing.assert_array_equal(counts[idx], ref)


def test_node_counts_and_dead_entries():
    nq = _nq()
    n, k = 11, 3
    pre, w = oracle.kings_frontier(n, k)
    ref, ref_nodes = oracle.kings_count_prefixes(n, pre, threads=8)
    c, l, r = (_dev(x) for x in oracle.kings_prefixes_masks(n, pre))
    nodes = torch.empty(len(pre), dtype=torch.int64, device="cuda")
    for mode in ("persistent", "plain"):
        _say("nodes", n, k, mode)
        counts, _ = nq.count_subproblems(n, c, l, r, depth=k, mode=mode, nodes=nodes, kings=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
        np.testing.assert_array_equal(nodes.cpu().numpy().view(np.uint64), ref_nodes)
    # prefixes of every depth up to n, many of them dead ends
    rng = np.random.default_rng(5)
    for n in (6, 9, 12):
        for k in (2, n // 2, n - 2, n - 1, n):
            pre, _ = oracle.kings_frontier(n, k)
            if len(pre) == 0:
                continue
            pre = pre[np.sort(rng.choice(len(pre), min(200, len(pre)), replace=False))]
            ref, _ = oracle.kings_count_prefixes(n, pre, threads=8)
            c, l, r = (_dev(x) for x in oracle.kings_prefixes_masks(n, pre))
            _say("prefixes", n, k)
            counts, _ = nq.count_subproblems(n, c, l, r, depth=k, kings=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)


def test_kings_forms_under_every_selected_form():
    """The kings search runs form 1's step while the queens run form 1 and
    form 7's step (the popcount leaf test) under every other form, the
    default included.  Totals stay exact under each selection; under form 1
    the per-subproblem and node counts also equal the oracle's (the other
    tests above run form 7)."""
    nq = _nq()
    want = _kings_counts(10)[10]
    for form in (0, 1, 2, 3, 4, 5, 6, 7):
        prev = nq.set_loop_form(form)
        try:
            _say("kings under form", form)
            for mode in ("persistent", "plain"):
                assert nq.count(10, depth=3, mode=mode, kings=True) == want, (form, mode)
        finally:
            nq.set_loop_form(-1)
        assert prev in range(8)
    n, k = 11, 3
    pre, _ = oracle.kings_frontier(n, k)
    ref, ref_nodes = oracle.kings_count_prefixes(n, pre, threads=8)
    c, l, r = (_dev(x) for x in oracle.kings_prefixes_masks(n, pre))
    nodes = torch.empty(len(pre), dtype=torch.int64, device="cuda")
    nq.set_loop_form(1)
    try:
        for mode in ("persistent", "plain"):
            _say("form 1 nodes", n, k, mode)
            counts, _ = nq.count_subproblems(n, c, l, r, depth=k, mode=mode, nodes=nodes,
                                             kings=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
            np.testing.assert_array_equal(nodes.cpu().numpy().view(np.uint64), ref_nodes)
        _say("form 1 auto depth 14")
        assert nq.count(14, kings=True) == _kings_counts(14)[14]
    finally:
        nq.set_loop_form(-1)
