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
