"""Property tests (hypothesis, CPU): random boards, depths and prefixes.

The library's host frontier equals the oracle's prefix masks entry by entry for
any (n, depth) of both searches; a random legal prefix's oracle count equals
permutation brute force; the weighted frontier total does not depend on the
depth; and a mirrored prefix has the same count."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import paper_2511_12009_amd as nq

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(n=st.integers(1, 12), data=st.data(), kings=st.booleans())
def test_library_frontier_equals_oracle_masks(n, data, kings):
    k = data.draw(st.integers(0 if not kings else 1, min(n, 6)))
    if k == 0:
        return
    c, l, r, w = nq.frontier(n, k, kings=kings)
    if kings:
        pre, pw = oracle.kings_frontier(n, k)
        masks = oracle.kings_prefixes_masks(n, pre) if len(pre) else None
    else:
        pre, pw = oracle.frontier(n, k)
        masks = oracle.prefixes_masks(n, pre) if len(pre) else None
    assert len(c) == len(pre)
    if masks is not None:
        for got, want in zip((c, l, r, w), masks + (pw,)):
            np.testing.assert_array_equal(got, want)


def _random_legal_prefix(draw, n, k, kings):
    p = []
    for row in range(k):
        if kings:
            opts = [j for j in range(n) if j not in p and (not p or abs(p[-1] - j) != 1)]
        else:
            opts = [j for j in range(n) if all(p[i] != j and abs(p[i] - j) != row - i
                                               for i in range(row))]
        if not opts:
            return None
        p.append(draw(st.sampled_from(opts)))
    return p


@SETTINGS
@given(n=st.integers(4, 9), data=st.data(), kings=st.booleans())
def test_prefix_count_equals_brute_force_and_mirror(n, data, kings):
    k = data.draw(st.integers(1, n))
    p = _random_legal_prefix(data.draw, n, k, kings)
    if p is None:
        return
    count = (oracle.kings_count_prefixes if kings else oracle.count_prefixes)(
        n, np.array([p], dtype=np.int32))[0][0]
    brute = (oracle.kings_brute_count if kings else oracle.brute_count)(n, p)
    assert int(count) == brute
    mirror = [n - 1 - x for x in p]
    mcount = (oracle.kings_count_prefixes if kings else oracle.count_prefixes)(
        n, np.array([mirror], dtype=np.int32))[0][0]
    assert int(mcount) == int(count)


@SETTINGS
@given(n=st.integers(4, 11), k1=st.integers(1, 4), k2=st.integers(1, 4), kings=st.booleans())
def test_weighted_total_independent_of_depth(n, k1, k2, kings):
    def total(k):
        if kings:
            pre, w = oracle.kings_frontier(n, min(k, n))
            c, _ = oracle.kings_count_prefixes(n, pre, threads=4)
        else:
            pre, w = oracle.frontier(n, min(k, n))
            c, _ = oracle.count_prefixes(n, pre, threads=4)
        return int((c * w.astype(np.uint64)).sum())
    assert total(k1) == total(k2)
