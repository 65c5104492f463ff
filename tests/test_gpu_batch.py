"""GPU parity of ragged batches: many board sizes in one persistent launch,
captured as a HIP graph and replayed."""
import numpy as np
import pytest

import oracle
import seeded_inputs
from conftest import read_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-batch]", *a, flush=True)


def _oracle_totals():
    """Weighted totals of the stored oracle runs (tests/golden/oracle_runs.txt,
    written by make_golden.py from the oracle alone), by board size."""
    return {int(r[0]): int(r[3]) for r in read_table("oracle_runs.txt")}


def _expected(ns, known_counts):
    """The oracle's counts: computed now for n <= 14, from its stored runs
    above that (every size the ragged batch draws, 15..19, has one), and the
    published count only for a size with neither."""
    stored = _oracle_totals()
    cache = {}
    for n in sorted(set(ns)):
        cache[n] = oracle.queens(n)[0] if n <= 14 else stored.get(n, known_counts[n])
    return [cache[n] for n in ns]


def test_count_batch_mixed_sizes_and_depths(known_counts):
    nq = _nq()
    ns = list(range(1, 15)) + [12, 5, 13, 1, 2, 3]
    exp = _expected(ns, known_counts)
    _say("count_batch default depths", len(ns))
    assert nq.count_batch(ns) == exp
    depths = [max(1, min(n, (i % 5) + 1)) for i, n in enumerate(ns)]
    _say("count_batch explicit depths", depths)
    assert nq.count_batch(ns, depths=depths) == exp
    full = [n for n in ns]                     # depth n: every entry is a complete board
    _say("count_batch depth = n")
    assert nq.count_batch(ns, depths=full) == exp


def test_batch_alternating_sizes_with_dead_entries(known_counts):
    """Consecutive entries of different board sizes, many of which need no search
    (dead entries, last-row entries): a lane that parks on such an entry after a
    task of another size must stay parked."""
    nq = _nq()
    ns = [8, 13, 9, 12, 10, 14, 8, 11] * 4
    depths = [n - 2 if i % 2 else n - 3 for i, n in enumerate(ns)]
    exp = _expected(ns, known_counts)
    for fwd in (False, True):
        _say("alternating sizes, forward", fwd)
        with nq.Batch(ns, depths=depths) as b:
            for rep in range(2):
                assert b.run() == exp, (fwd, rep)


def test_count_batch_edges():
    nq = _nq()
    assert nq.count_batch([]) == []
    with pytest.raises(nq.NQError):
        nq.count_batch([8, 29])
    with pytest.raises(nq.NQError):
        nq.count_batch([8, 9], depths=[3, 10])


def test_ragged_256_graph_replays(known_counts):
    """256 instances, N uniform in 8..19 (seeded): every replay of the captured
    graph, with eager GPU work in between, gives every instance's exact count."""
    nq = _nq()
    ns = seeded_inputs.ragged_batch_ns()
    exp = _expected(ns, known_counts)
    _say("ragged 256 create")
    with nq.Batch(ns) as b:
        assert b.entries > 0
        for rep in range(3):
            _say("ragged 256 replay", rep)
            got, ms = b.run(timing=True)
            assert got == exp, rep
            assert ms > 0
            x = torch.randn(1 << 20, device="cuda")       # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(x.sum())


def test_batch_matches_single_counts_per_depth(known_counts):
    nq = _nq()
    ns = [16, 17, 11, 16]
    for k in (2, 4, 6):
        _say("batch depth", k)
        with nq.Batch(ns, depth=k) as b:
            assert b.run() == [known_counts[n] for n in ns]
