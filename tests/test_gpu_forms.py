"""GPU parity of every inner-loop form of the DFS kernel (nq_set_loop_form):
the compiler-scheduled step (0), the hand-placed exec masks (1), the
negated-untried-set form (2), the step without selects (3), the paper's loop
with the frame read from the LDS stack at every step (4), the step without
the last-row shortcut (5), form 3 with a push that needs no exec mask (6) and
form 6 without the sentinel frame below each lane's stack (7, the default)
give the oracle's counts and node counts, in plain
and persistent launches, batches and the serving loop, with the row counter
(forms 3, 6 and 7: the rd marker) and with the popcount leaf test."""
import hashlib

import numpy as np
import pytest

import oracle
from conftest import read_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FORMS = [0, 1, 2, 3, 4, 5, 6, 7]


def _say(*a):
    print("[gpu-forms]", *a, flush=True)


@pytest.fixture(params=FORMS)
def nq_form(request):
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prev = nq.set_loop_form(request.param)
    try:
        yield nq, request.param
    finally:
        nq.set_loop_form(-1)
        assert prev in FORMS


def _golden_runs():
    return {(int(r[0]), int(r[1])): r for r in read_table("oracle_runs.txt")}


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def test_small_boards(nq_form, known_counts):
    nq, form = nq_form
    for mode in ("plain", "persistent"):
        _say("form", form, "small boards", mode)
        for n in range(1, 11):
            for k in sorted(k for k in {1, 2, n // 2, n - 1, n} if 1 <= k <= n):
                assert nq.count(n, depth=k, mode=mode) == known_counts[n], (form, n, k, mode)


def test_per_subproblem_and_nodes(nq_form):
    nq, form = nq_form
    g = _golden_runs()
    for n, k, modes in ((14, 3, ("persistent", "plain")), (17, 5, ("persistent",))):
        cols, ld, rd, _ = nq.frontier(n, k)
        t = [_dev(x) for x in (cols, ld, rd)]
        nodes = torch.empty(len(cols), dtype=torch.int64, device="cuda")
        for mode in modes:
            _say("form", form, "nodes", n, k, mode)
            counts, _ = nq.count_subproblems(n, *t, depth=k, mode=mode, nodes=nodes)
            torch.cuda.synchronize()
            assert _digest(counts.cpu().numpy().view(np.uint64)) == g[(n, k)][5], (form, n, k)
            assert _digest(nodes.cpu().numpy().view(np.uint64)) == g[(n, k)][6], (form, n, k)


def test_random_prefixes_with_dead_entries(nq_form):
    nq, form = nq_form
    rng = np.random.default_rng(2512)
    for n in (5, 11, 13):
        for k in sorted({1, 2, n // 2, n - 1, n}):
            pre_all, _ = oracle.frontier(n, k)
            if len(pre_all) == 0:
                continue
            pre = pre_all[np.sort(rng.choice(len(pre_all), min(200, len(pre_all)), replace=False))]
            c, l, r = (_dev(x) for x in oracle.prefixes_masks(n, pre))
            ref, _ = oracle.count_prefixes(n, pre, threads=8)
            for mode in ("plain", "persistent"):
                _say("form", form, "prefixes", n, k, mode)
                counts, total = nq.count_subproblems(n, c, l, r, depth=k, mode=mode)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)


def test_batch_and_serving(nq_form, known_counts):
    nq, form = nq_form
    ns = [8, 13, 5, 16, 1, 12, 15, 9]
    _say("form", form, "batch", ns)
    assert nq.count_batch(ns) == [known_counts[n] for n in ns]
    _say("form", form, "serving")
    with nq.Server() as srv:
        tickets = [srv.submit_count(n) for n in (10, 14, 16)]
        sl = srv.submit_slice(16, 5, 100, 300)
        for n, t in zip((10, 14, 16), tickets):
            r = srv.wait(t, timeout_s=60)
            assert r["status"] == 0 and r["count"] == known_counts[n], (form, n)
        r = srv.wait(sl, timeout_s=60)
        pre, w = oracle.frontier(16, 5)
        ref, _ = oracle.count_prefixes(16, pre[100:400], threads=8)
        assert r["count"] == int((ref * w[100:400].astype(np.uint64)).sum())


def test_shallow_promise_uses_popcount_leaf_test(nq_form):
    """Entries of the N=18 depth-6 frontier counted under a promise of only 2
    queens placed: the launch sizes its stack for 14 frames, and forms 3, 6 and
    7 cannot use their rd marker for such entries (n + frames > 30), so their
    popcount leaf test runs; counts and node counts equal the oracle's per entry."""
    nq, form = nq_form
    n, k = 18, 6
    pre_all, _ = oracle.frontier(n, k)
    rng = np.random.default_rng(1806)
    pre = pre_all[np.sort(rng.choice(len(pre_all), 400, replace=False))]
    c, l, r = (_dev(x) for x in oracle.prefixes_masks(n, pre))
    ref, ref_nodes = oracle.count_prefixes(n, pre, threads=8)
    nodes = torch.empty(len(pre), dtype=torch.int64, device="cuda")
    for mode in ("persistent", "plain"):
        _say("form", form, "shallow promise", n, mode)
        counts, _ = nq.count_subproblems(n, c, l, r, depth=2, mode=mode, nodes=nodes)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(counts.cpu().numpy().view(np.uint64), ref)
        np.testing.assert_array_equal(nodes.cpu().numpy().view(np.uint64), ref_nodes)
