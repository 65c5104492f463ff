"""GPU: nq_count_subproblems_noalloc (work head in the library's static
device array) gives the same per-entry counts, node counts and weighted
totals as nq_count_subproblems, called through the C-ABI: two calls in a row,
the second on a smaller input, in persistent and plain mode, and with a
128-bit total."""
import ctypes as ct

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nq():
    import paper_2511_12009_amd as nq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return nq


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def _resident(nq, n, k):
    cols, ld, rd, w = nq.frontier(n, k)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x.view(np.int32)).to(dev) for x in (cols, ld, rd)]
    return t, torch.from_numpy(w).to(dev)


def _call(nq, fn, n, t, w, k, mode, stream, flags=0, words=1):
    L = nq._native.lib()
    counts = torch.full((t[0].numel(),), -7, dtype=torch.int64, device="cuda")
    nodes = torch.full((t[0].numel(),), -7, dtype=torch.int64, device="cuda")
    total = torch.zeros(words, dtype=torch.int64, device="cuda")
    o = nq._native._opts(k, mode, 0, 0, 0, stream.cuda_stream, flags, 0)
    o.d_nodes = nodes.data_ptr()
    rc = getattr(L, fn)(n, t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), w.data_ptr(),
                        t[0].numel(), counts.data_ptr(), total.data_ptr(), ct.byref(o))
    nq._native._check(rc, fn)
    stream.synchronize()
    return counts.cpu().numpy(), nodes.cpu().numpy(), total.cpu().numpy()


def test_noalloc_matches_the_allocating_entry_point(known_counts):
    nq = _nq()
    stream = torch.cuda.Stream()
    for n, k in ((17, 5), (12, 3)):                   # the second call: a smaller input
        t, w = _resident(nq, n, k)
        for mode in ("persistent", "plain"):
            _say("noalloc", n, k, mode)
            a = _call(nq, "nq_count_subproblems_noalloc", n, t, w, k, mode, stream)
            b = _call(nq, "nq_count_subproblems", n, t, w, k, mode, stream)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
            assert int(a[2][0]) == int(b[2][0]) == known_counts[n]
    t, w = _resident(nq, 13, 4)
    _say("noalloc wide total")
    a = _call(nq, "nq_count_subproblems_noalloc", 13, t, w, 4, "persistent", stream,
              flags=nq._native.FLAG_WIDE_TOTAL, words=2)
    assert [int(x) for x in a[2]] == [known_counts[13], 0]


def test_noalloc_refuses_timing_before_any_launch():
    nq = _nq()
    L = nq._native.lib()
    o = nq._native._opts(3, "persistent", 0, 0, 0, None, 0, 0)
    ms = ct.c_double(0.0)
    o.kernel_ms_out = ct.pointer(ms)
    fake = ct.c_void_p(16)                            # never dereferenced: refused first
    assert L.nq_count_subproblems_noalloc(12, fake, fake, fake, None, 10, None, None,
                                          ct.byref(o)) == nq._native.NQ_EINVAL
