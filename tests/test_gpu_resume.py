"""GPU: the resumable count.  A count cut into chunks stops after any number of
them and resumes from its progress file, in the same process or another; a
record rolled back to an earlier chunk redoes the later chunks with the same
result; partial totals equal the oracle's weighted count of the chunks done."""
import os
import shutil

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
    print("[gpu-resume]", *a, flush=True)


def _fields(path):
    with open(path) as f:
        line = f.read()
    assert line.endswith("\n") and line.count("\n") == 1
    return dict(x.split("=", 1) for x in line.split() if "=" in x)


def test_stop_resume_and_roll_back(tmp_path, known_counts):
    nq = _nq()
    n, depth, chunks = 16, 7, 8
    path = str(tmp_path / "n16.progress")
    pre, w = oracle.frontier(n, 5)                 # chunks are ranges of the depth-5 frontier
    ref, _ = oracle.count_prefixes(n, pre, threads=8)
    wref = ref * w.astype(np.uint64)
    F = len(pre)

    def partial(done):
        return int(wref[:F * done // chunks].sum())

    _say("n16 first 3 chunks")
    assert nq.count_resumable(n, path, chunks=chunks, max_chunks=3, depth=depth) == \
        (partial(3), 3, False)
    rec = _fields(path)
    assert (rec["n"], rec["depth"], rec["host_depth"], rec["chunks"], rec["done"]) == \
        ("16", "7", "5", "8", "3")
    assert int(rec["total"]) == partial(3)
    _say("n16 next 3 chunks")
    assert nq.count_resumable(n, path, chunks=chunks, max_chunks=3, depth=depth) == \
        (partial(6), 6, False)
    shutil.copy(path, path + ".at6")
    _say("n16 the rest")
    assert nq.count_resumable(n, path, chunks=chunks, depth=depth) == (known_counts[n], 8, True)
    assert not os.path.exists(path + ".tmp")
    # a finished record answers again without counting
    assert nq.count_resumable(n, path, chunks=chunks, depth=depth) == (known_counts[n], 8, True)
    # rolled back to 6 chunks: the last two are counted again, same result
    shutil.copy(path + ".at6", path)
    _say("n16 from a rolled-back record")
    assert nq.count_resumable(n, path, chunks=chunks, depth=depth) == (known_counts[n], 8, True)


def test_more_chunks_than_entries_and_plain_mode(tmp_path, known_counts):
    nq = _nq()
    # N=8 at depth 3: the depth-3 host frontier has fewer entries than chunks
    path = str(tmp_path / "n8")
    _say("n8 64 chunks")
    assert nq.count_resumable(8, path, chunks=64, depth=3) == (known_counts[8], 64, True)
    path = str(tmp_path / "n13")
    _say("n13 plain")
    assert nq.count_resumable(13, path, chunks=5, depth=6, mode="plain") == \
        (known_counts[13], 5, True)


def test_n20_in_four_chunks(tmp_path, known_counts):
    nq = _nq()
    path = str(tmp_path / "n20")
    _say("n20 two of four chunks")
    total, done, fin = nq.count_resumable(20, path, chunks=4, max_chunks=2, depth=9)
    assert (done, fin) == (2, False)
    _say("n20 the other two")
    assert nq.count_resumable(20, path, chunks=4, depth=9) == (known_counts[20], 4, True)


def test_wide_total_carries_into_the_high_word(known_counts):
    """NQ_FLAG_WIDE_TOTAL: the device total is 128 bits and is increased with
    carry.  Started just below 2^64, an N = 12 count (14,200) must carry into
    the high word, which keeps what it held."""
    nq = _nq()
    n, k = 12, 4
    cols, ld, rd, w = nq.frontier(n, k)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x.view(np.int32)).to(dev) for x in (cols, ld, rd)]
    tw = torch.from_numpy(w).to(dev)
    start_lo = 2**64 - 100
    total = torch.tensor([start_lo - 2**64, 7], dtype=torch.int64, device=dev)
    _say("wide total N=12 persistent")
    nq.count_subproblems(n, *t, weight=tw, counts=False, total=total, depth=k, wide=True)
    lo, hi = (int(x) & (2**64 - 1) for x in total.cpu())
    assert (hi << 64) + lo == (7 << 64) + start_lo + known_counts[n]
    total = torch.tensor([-1, 0], dtype=torch.int64, device=dev)            # 2^64 - 1
    _say("wide total N=12 plain")
    nq.count_subproblems(n, *t, weight=tw, counts=False, total=total, depth=k, wide=True,
                         mode="plain")
    lo, hi = (int(x) & (2**64 - 1) for x in total.cpu())
    assert (hi << 64) + lo == 2**64 - 1 + known_counts[n]


def test_wide_resumable_crosses_two_to_the_64(tmp_path, known_counts):
    """A record whose total is just below 2^64 with one chunk left: the last
    chunk takes the 128-bit total across 2^64 in the record and the result;
    the 64-bit entry point reports NQ_ERANGE for the same file.  A board of at
    most 16 through the wide entry gives the published count."""
    nq = _nq()
    n, depth, chunks = 13, 6, 4
    pre, w = oracle.frontier(n, 5)
    ref, _ = oracle.count_prefixes(n, pre, threads=8)
    wref = (ref * w.astype(np.uint64)).astype(object)
    F = len(pre)
    last = int(sum(wref[F * 3 // chunks:]))
    assert last > 0
    base = 2**64 - last // 2
    path = str(tmp_path / "carry")
    body = (f"nq-progress 1 n={n} depth={depth} host_depth=5 chunks={chunks} done=3 "
            f"total={base}")
    h = 0xcbf29ce484222325
    for ch in body.encode():
        h = ((h ^ ch) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    with open(path, "w") as f:
        f.write(f"{body} check={h:016x}\n")
    _say("wide resumable across 2^64")
    assert nq.count_resumable(n, path, chunks=chunks, depth=depth, wide=True) == \
        (base + last, chunks, True)
    assert int(_fields(path)["total"]) == base + last > 2**64
    with pytest.raises(nq.NQError) as e:
        nq.count_resumable(n, path, chunks=chunks, depth=depth)
    assert e.value.status == nq._native.NQ_ERANGE
    _say("wide resumable N=16")
    assert nq.count_resumable(16, str(tmp_path / "n16"), chunks=8, depth=8, wide=True) == \
        (known_counts[16], 8, True)


def test_automatic_depth_ignores_the_tuner(tmp_path, known_counts):
    """With depth 0 the resumable count picks its depth without this process's
    tuning results, and a record of the same count supplies its own depth, so
    a tuned process and a fresh one continue the same file."""
    nq = _nq()
    n = 15
    path = str(tmp_path / "n15")
    _say("n15 resumable, depth 0, first half")
    total, done, fin = nq.count_resumable(n, path, chunks=4, max_chunks=2)
    assert (done, fin) == (2, False)
    depth0 = int(_fields(path)["depth"])
    _say("n15 autotune over other depths")
    nq.autotune(n, depth0 + 1, depth0 + 2, budget_ms=2000)      # the tuner remembers another depth
    _say("n15 resumable, depth 0, after tuning")
    assert nq.count_resumable(n, path, chunks=4) == (known_counts[n], 4, True)
    assert int(_fields(path)["depth"]) == depth0
    fresh = str(tmp_path / "n15b")
    _say("n15 resumable, depth 0, new file after tuning")
    nq.count_resumable(n, fresh, chunks=4, max_chunks=1)
    assert int(_fields(fresh)["depth"]) == depth0
