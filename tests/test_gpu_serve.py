"""GPU: the serving loop.  Results are exact, identical alone and in a mix of
concurrent requests, and slices of the N=21 depth-6 frontier add up to Q(21)."""
import numpy as np
import pytest

import oracle
import seeded_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-serve]", *a, flush=True)


@pytest.mark.parametrize("reserve", [False, True])
def test_counts_alone_and_in_a_mix(known_counts, reserve):
    """Counts and slices give the same results alone and in a mix; with
    NQ_FLAG_SERVE_RESERVE (reserve=True) the quick COUNTs overtake the others
    and large epochs run one at a time, with the same results."""
    nq = _nq()
    ns = seeded_inputs.serve_count_ns(40)
    with nq.Server(reserve=reserve) as srv:
        alone = {}
        for n in sorted(set(ns)):
            _say("alone", n)
            r = srv.wait(srv.submit_count(n), timeout_s=60)
            assert r["status"] == 0 and r["count"] == known_counts[n], n
            alone[n] = r["count"]
        _say("mix of", len(ns))
        tickets = [srv.submit_count(n) for n in ns]
        slices = [srv.submit_slice(16, 5, s, 200) for s in range(0, 4000, 400)]
        for n, t in zip(ns, tickets):
            r = srv.wait(t, timeout_s=120)
            assert r["status"] == 0 and r["count"] == alone[n]
            assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
        pre, w = oracle.frontier(16, 5)
        # the server searches a slice as the slice's children two rows down
        # (the depth-5 frontier has >= 2^16 entries): count them in the depth-7
        # frontier by their 5-row prefixes
        pre7, _ = oracle.frontier(16, 7)
        code = lambda p: (p.astype(np.int64) * (16 ** np.arange(4, -1, -1))).sum(axis=1)  # noqa
        code7 = code(pre7[:, :5])
        for i, t in enumerate(slices):
            r = srv.wait(t, timeout_s=120)
            lo = i * 400
            ref, _ = oracle.count_prefixes(16, pre[lo:lo + 200], threads=8)
            assert r["count"] == int((ref * w[lo:lo + 200].astype(np.uint64)).sum())
            assert r["entries"] == int(np.isin(code7, code(pre[lo:lo + 200])).sum())


def test_small_boards_and_bad_requests(known_counts):
    nq = _nq()
    with nq.Server() as srv:
        for n in (1, 2, 3, 4, 5, 8):
            r = srv.wait(srv.submit_count(n), timeout_s=30)
            assert r["count"] == known_counts[n], n
        with pytest.raises(nq.NQError):
            srv.submit_count(29)
        with pytest.raises(nq.NQError):
            srv.submit_slice(21, 0, 0, 10)
        with pytest.raises(nq.NQError):
            srv.submit_count(24, depth=2)          # needs more stack than the server has
        t = srv.submit_slice(12, 3, 10 ** 6, 5)   # past the end of the frontier
        r = srv.wait(t, timeout_s=30)
        assert r["status"] != 0
        with pytest.raises(nq.NQError):
            srv.poll(t)                            # ticket already collected


def test_n21_slices_sum_to_q21(known_counts):
    """Every 4096-entry slice of the N=21 depth-6 frontier (the last one short),
    submitted at once; the weighted slice sums add up to Q(21)."""
    nq = _nq()
    F = nq.frontier_size(21, 6)
    starts = list(range(0, F, 4096))
    assert len(starts) == 1092
    with nq.Server(hbm_budget=2 << 30) as srv:
        _say("n21 slices", len(starts))
        tickets = [srv.submit_slice(21, 6, s, min(4096, F - s)) for s in starts]
        total = 0
        for i, t in enumerate(tickets):
            r = srv.wait(t, timeout_s=300)
            assert r["status"] == 0
            total += r["count"]
            if i % 200 == 0:
                _say("slices done", i)
        assert total == known_counts[21]


def test_many_tiny_slices_share_waves():
    """Hundreds of 1..7-entry slices of the N=13 depth-4 frontier submitted at
    once: one wave retires entries of many requests at the same visit, and each
    request's total and completion must still be its own (oracle per slice)."""
    nq = _nq()
    pre, w = oracle.frontier(13, 4)
    F = len(pre)
    assert nq.frontier_size(13, 4) == F and F < 2 ** 16       # kept unexpanded
    ref, _ = oracle.count_prefixes(13, pre, threads=8)
    wref = ref * w.astype(np.uint64)
    rng = np.random.default_rng(20251112)
    spans, s = [], 0
    while s < F:
        ln = int(rng.integers(1, 8))
        spans.append((s, min(ln, F - s)))
        s += ln
    with nq.Server() as srv:
        _say("tiny slices", len(spans))
        tickets = [srv.submit_slice(13, 4, a, ln) for a, ln in spans]
        for (a, ln), t in zip(spans, tickets):
            r = srv.wait(t, timeout_s=120)
            assert r["status"] == 0
            assert r["entries"] == ln
            assert r["count"] == int(wref[a:a + ln].sum()), (a, ln)


def test_requests_beyond_a_small_budget_fail_alone(known_counts):
    """A server with an 8 MiB budget: a request whose subproblems cannot fit its
    ring or resident space completes with NQ_ENOMEM in its result, while the
    small requests around it are still answered exactly."""
    nq = _nq()
    with nq.Server(hbm_budget=8 << 20) as srv:
        _say("small budget")
        small = [srv.submit_count(n) for n in (8, 10, 11)]
        big = srv.submit_count(18)
        more = [srv.submit_count(n) for n in (9, 12)]
        r = srv.wait(big, timeout_s=60)
        assert r["status"] == -3                     # NQ_ENOMEM
        for n, t in zip((8, 10, 11, 9, 12), small + more):
            r = srv.wait(t, timeout_s=60)
            assert r["status"] == 0 and r["count"] == known_counts[n], n


def test_n21_seeded_slices_match_the_oracle():
    """Seeded N=21 depth-6 slices (and the last, short one), against the
    oracle's stored counts of the same slices (tests/golden/oracle_slices.txt,
    make_golden.py --slices): each slice's weighted sum from the server, and
    every entry's count from one direct launch over the slices' entries
    (no expansion), element by element through the digest of the counts."""
    import hashlib
    from conftest import read_table
    nq = _nq()
    rows = [r for r in read_table("oracle_slices.txt") if r[:2] == ["21", "6"]]
    assert len(rows) >= 5
    cols, ld, rd, w = nq.frontier(21, 6)
    with nq.Server() as srv:
        tickets = [srv.submit_slice(21, 6, int(r[2]), int(r[3])) for r in rows]
        for r, t in zip(rows, tickets):
            _say("n21 slice at", r[2])
            res = srv.wait(t, timeout_s=300)
            assert res["status"] == 0
            assert res["count"] == int(r[4]), r[2]
    idx = np.concatenate([np.arange(int(r[2]), int(r[2]) + int(r[3])) for r in rows])
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(np.ascontiguousarray(x[idx]).view(np.int32)).to(dev)
         for x in (cols, ld, rd)]
    nodes = torch.empty(len(idx), dtype=torch.int64, device=dev)
    _say("n21 slices per entry", len(idx))
    counts, _ = nq.count_subproblems(21, *t, depth=6, nodes=nodes)
    counts = counts.cpu().numpy().view(np.uint64)
    nodes = nodes.cpu().numpy().view(np.uint64)
    pos = 0
    for r in rows:
        ln = int(r[3])
        c = counts[pos:pos + ln]
        assert hashlib.sha256(np.ascontiguousarray(c, dtype="<u8").tobytes()).hexdigest() == r[6]
        assert int(nodes[pos:pos + ln].sum()) == int(r[5])
        assert int((c.astype(object) * w[int(r[2]):int(r[2]) + ln].astype(object)).sum()) == \
            int(r[4])
        pos += ln
