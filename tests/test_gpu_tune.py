"""GPU: the autotuner measures, agrees on the count, and feeds nq_count."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_autotune_small_board(known_counts):
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-tune] autotune n=14", flush=True)
    best = nq.autotune(14, 2, 5, budget_ms=5000)
    assert 2 <= best["depth"] <= 5
    assert best["count"] == known_counts[14]
    assert best["trials"] >= 4 and best["ms"] > 0
    # nq_count with automatic depth now uses the tuned choice
    assert nq.count(14) == known_counts[14]


def test_autotune_rejects_bad_ranges():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with pytest.raises(nq.NQError):
        nq.autotune(3)
    with pytest.raises(nq.NQError):
        nq.autotune(12, 6, 4)
