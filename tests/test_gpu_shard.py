"""GPU: one GPU's share of a count sharded over 8 GPUs.  The N=21 depth-6
frontier is dealt round-robin (entry i to share i mod 8); each share is
deepened three rows on the device and searched by one persistent launch, as one
GPU of eight would do.  The eight weighted share totals add up to Q(21), and
seeded entries of every share have the oracle's per-entry counts."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHARES, N, K, DEEPEN = 8, 21, 6, 3


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-shard]", *a, flush=True)


def _share(arr, r):
    return np.ascontiguousarray(arr[r::SHARES])


def test_strided_shares_of_n21(known_counts):
    nq = _nq()
    dev = torch.device("cuda:0")
    cols, ld, rd, w = nq.frontier(N, K)
    pre, pw = oracle.frontier(N, K)
    assert len(pre) == len(cols) and np.array_equal(pw, w)
    rng = np.random.default_rng(21_06)
    grand = 0
    for r in range(SHARES):
        _say("share", r, "of", SHARES)
        t = [torch.from_numpy(_share(x, r).view(np.int32)).to(dev) for x in (cols, ld, rd)]
        tw = torch.from_numpy(_share(w, r)).to(dev)
        # the share searched as a GPU would: deepened, one persistent launch
        c, l, rr, ww = nq.expand(N, DEEPEN, t[0], t[1], t[2], tw)
        tot = torch.zeros(1, dtype=torch.int64, device=dev)
        nq.count_subproblems(N, c, l, rr, weight=ww, counts=False, total=tot, depth=K + DEEPEN)
        torch.cuda.synchronize()
        grand += int(tot.item())
        del c, l, rr, ww
        # seeded entries of the share at their own depth against the oracle
        j = np.sort(rng.choice(t[0].numel(), 6, replace=False))
        sel = torch.from_numpy(j).to(dev)
        counts, _ = nq.count_subproblems(N, t[0][sel].contiguous(), t[1][sel].contiguous(),
                                         t[2][sel].contiguous(), depth=K)
        ref, _ = oracle.count_prefixes(N, pre[r + SHARES * j], threads=6)
        assert np.array_equal(counts.cpu().numpy().astype(np.uint64), ref), (r, j)
    assert grand == known_counts[N]
