"""GPU: the autotuner measures, agrees on the count, and feeds nq_count."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_autotune_small_board(known_counts):
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-tune] autotune n=14", flush=True)
    best = nq.autotune(14, 2, 5, budget_ms=5000, table=True)
    assert 2 <= best["depth"] <= 5
    assert best["count"] == known_counts[14]
    assert best["trials"] >= 4 and best["ms"] > 0
    table = best["table"]
    assert len(table) == best["trials"]
    assert {r["depth"] for r in table} >= {2, 3, 4, 5}
    # the workgroup-size axis was measured at the best depth
    assert {r["wg_size"] for r in table if r["depth"] == best["depth"]} >= {64, 128, 256}
    assert min(r["ms"] for r in table) == best["ms"]
    assert best["wg_size"] in (0, 64, 128, 256)
    # nq_count with automatic depth now uses the tuned choice, remembered here
    assert nq.tuned_lookup(14) == {k: v for k, v in best.items() if k != "table"}
    assert nq.count(14) == known_counts[14]


def test_tuned_workgroup_size_is_used_and_exact(known_counts):
    """A tuning whose best launch has a workgroup of several waves: nq_count
    with the automatic depth runs that shape (the remembered tuning says so)
    and stays exact."""
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for n in (15, 16):
        print(f"[gpu-tune] autotune n={n}", flush=True)
        best = nq.autotune(n, 4, 6, budget_ms=8000, table=True)
        assert best["count"] == known_counts[n]
        for wg in (128, 256):
            assert any(r["wg_size"] == wg for r in best["table"]), (n, wg)
        assert nq.tuned_lookup(n)["wg_size"] == best["wg_size"]
        assert nq.count(n) == known_counts[n]
        for wg in (64, 128, 256):
            assert nq.count(n, depth=best["depth"], wg_size=wg) == known_counts[n], (n, wg)


def test_autotune_rejects_bad_ranges():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with pytest.raises(nq.NQError):
        nq.autotune(3)
    with pytest.raises(nq.NQError):
        nq.autotune(12, 6, 4)


def test_chunked_board_is_tuned_on_one_chunk(known_counts):
    """N = 21 counts in 16 chunks of its depth-5 frontier: the tuner times the
    middle chunk at depths 9..11 (every depth must give that chunk the same
    count), and nq_count then runs the chunked count at the tuned depth,
    exactly.  The chunk's count is also taken by a launch over the same
    depth-5 entries without any expansion."""
    import numpy as np
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 21
    print("[gpu-tune] autotune n=21 (chunked)", flush=True)
    best = nq.autotune(n, table=True)
    assert best["chunks"] == 16 and 9 <= best["depth"] <= 11
    table = best["table"]
    assert [r["depth"] for r in table] == [9, 9, 10, 11]
    assert all(r["chunks"] == 16 and r["ms"] > 0 for r in table)
    assert min(r["ms"] for r in table) == best["ms"]
    assert nq.tuned_lookup(n) == {k: v for k, v in best.items() if k != "table"}
    cols, ld, rd, w = nq.frontier(n, 5)
    F = len(cols)
    lo, hi = F * 8 // 16, F * 9 // 16
    dev = [torch.from_numpy(np.ascontiguousarray(a[lo:hi]).view(np.int32)).cuda()
           for a in (cols, ld, rd)]
    wt = torch.from_numpy(np.ascontiguousarray(w[lo:hi])).cuda()
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("[gpu-tune] middle chunk at depth 5", flush=True)
    nq.count_subproblems(n, *dev, weight=wt, counts=False, total=total, depth=5)
    torch.cuda.synchronize()
    assert int(total.item()) == best["count"]
    print("[gpu-tune] count(21) with the tuned chunk plan", flush=True)
    assert nq.count(n) == known_counts[n]
