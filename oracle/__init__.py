"""N-Queens counting oracle -- test infrastructure, not part of the product.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
board arrays, built from ``oracle.c`` by ``oracle/build.py``) and shares no code
with the GPU library.  What each function computes, and the readings of the
paper it takes, are stated in ``oracle.c``.

Functions
---------
queens(n)                      -> (Q(n), nodes from row 0)
count_prefix(n, prefix)        -> (completions, nodes in rows k..n-2)
brute_count(n, prefix=())      -> completions by permutation enumeration (n <= 11)
frontier(n, k)                 -> (prefixes int32[F, k], weights uint8[F])
frontier_size(n, k)            -> F
prefix_masks(n, prefix)        -> (cols, ld, rd) attack masks on row len(prefix)
frontier_masks(n, k)           -> (cols, ld, rd uint32[F], weights uint8[F])
prefixes_masks(n, prefixes)    -> (cols, ld, rd uint32[m]) for many prefixes
count_prefixes(n, prefixes, threads) -> (counts uint64[F], nodes uint64[F])

The second search (n non-attacking kings, one per row and column; see the
kings section of ``oracle.c``), with the same shapes:
kings(n), kings_brute_count(n, prefix=()), kings_frontier(n, k),
kings_frontier_size(n, k), kings_prefixes_masks(n, prefixes),
kings_count_prefixes(n, prefixes, threads)

The third search (the permanent of a 0/1 matrix ``a``, uint8[n, n]: the
permutations s with a[r, s(r)] != 0 for every row r; see the permanents
section of ``oracle.c``); prefixes carry no weights:
permanent(a), perm_frontier(a, k), perm_frontier_size(a, k),
perm_prefixes_cols(n, prefixes), perm_count_prefixes(a, prefixes, threads),
permanent_ryser(a) (Ryser's formula, n <= 20)
"""
from __future__ import annotations

import ctypes as _ct
import os as _os

import numpy as _np

from . import build as _build

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_LIB = None

OQ_OK, OQ_EINVAL, OQ_ERANGE, OQ_ENOMEM = 0, -1, -2, -3


class OracleError(RuntimeError):
    pass


def _lib():
    global _LIB
    if _LIB is None:
        path = _os.path.join(_HERE, "liboracle.so")
        if not _os.path.exists(path):
            _build.build()
        lib = _ct.CDLL(path)
        u64p = _ct.POINTER(_ct.c_uint64)
        u32p = _ct.POINTER(_ct.c_uint32)
        i32p = _ct.POINTER(_ct.c_int)
        u8p = _ct.POINTER(_ct.c_uint8)
        lib.oq_queens.argtypes = [_ct.c_int, u64p, u64p]
        lib.oq_count_prefix.argtypes = [_ct.c_int, _ct.c_int, i32p, u64p, u64p]
        lib.oq_brute_count.argtypes = [_ct.c_int, _ct.c_int, i32p, u64p]
        lib.oq_frontier.argtypes = [_ct.c_int, _ct.c_int, i32p, u8p, _ct.c_uint64, u64p]
        lib.oq_prefix_masks.argtypes = [_ct.c_int, _ct.c_int, i32p, u32p, u32p, u32p]
        lib.oq_prefixes_masks.argtypes = [_ct.c_int, _ct.c_int, i32p, _ct.c_uint64, u32p, u32p,
                                          u32p]
        lib.oq_count_prefixes.argtypes = [_ct.c_int, _ct.c_int, i32p, _ct.c_uint64, _ct.c_int,
                                          u64p, u64p]
        lib.oqk_count_prefix.argtypes = [_ct.c_int, _ct.c_int, i32p, u64p, u64p]
        lib.oqk_brute_count.argtypes = [_ct.c_int, _ct.c_int, i32p, u64p]
        lib.oqk_frontier.argtypes = [_ct.c_int, _ct.c_int, i32p, u8p, _ct.c_uint64, u64p]
        lib.oqk_prefixes_masks.argtypes = [_ct.c_int, _ct.c_int, i32p, _ct.c_uint64, u32p, u32p,
                                           u32p]
        lib.oqk_count_prefixes.argtypes = [_ct.c_int, _ct.c_int, i32p, _ct.c_uint64, _ct.c_int,
                                           u64p, u64p]
        lib.oqp_count_prefix.argtypes = [_ct.c_int, u8p, _ct.c_int, i32p, u64p, u64p]
        lib.oqp_frontier.argtypes = [_ct.c_int, u8p, _ct.c_int, i32p, u8p, _ct.c_uint64, u64p]
        lib.oqp_prefixes_cols.argtypes = [_ct.c_int, _ct.c_int, i32p, _ct.c_uint64, u32p]
        lib.oqp_count_prefixes.argtypes = [_ct.c_int, u8p, _ct.c_int, i32p, _ct.c_uint64,
                                           _ct.c_int, u64p, u64p]
        lib.oqp_ryser.argtypes = [_ct.c_int, u8p, u64p]
        for f in (lib.oq_queens, lib.oq_count_prefix, lib.oq_brute_count, lib.oq_frontier,
                  lib.oq_prefix_masks, lib.oq_prefixes_masks, lib.oq_count_prefixes,
                  lib.oqk_count_prefix, lib.oqk_brute_count, lib.oqk_frontier,
                  lib.oqk_prefixes_masks, lib.oqk_count_prefixes, lib.oqp_count_prefix,
                  lib.oqp_frontier, lib.oqp_prefixes_cols, lib.oqp_count_prefixes,
                  lib.oqp_ryser):
            f.restype = _ct.c_int
        _LIB = lib
    return _LIB


def _check(rc, what):
    if rc != OQ_OK:
        raise OracleError(f"{what} failed with status {rc}")


def _iarr(seq):
    a = _np.ascontiguousarray(_np.asarray(seq, dtype=_np.int32))
    return a, a.ctypes.data_as(_ct.POINTER(_ct.c_int))


def queens(n: int):
    """Q(n) by plain backtracking over every column of every row."""
    c, nd = _ct.c_uint64(), _ct.c_uint64()
    _check(_lib().oq_queens(n, _ct.byref(c), _ct.byref(nd)), "oq_queens")
    return c.value, nd.value


def count_prefix(n: int, prefix):
    """Completions of rows len(prefix)..n-1 below ``prefix`` and the node count."""
    a, p = _iarr(prefix)
    c, nd = _ct.c_uint64(), _ct.c_uint64()
    _check(_lib().oq_count_prefix(n, len(a), p, _ct.byref(c), _ct.byref(nd)), "oq_count_prefix")
    return c.value, nd.value


def brute_count(n: int, prefix=()):
    """Completions of ``prefix`` by enumerating permutations (n <= 11)."""
    a, p = _iarr(list(prefix) if len(prefix) else [0])
    c = _ct.c_uint64()
    _check(_lib().oq_brute_count(n, len(prefix), p, _ct.byref(c)), "oq_brute_count")
    return c.value


def frontier_size(n: int, k: int) -> int:
    ln = _ct.c_uint64()
    _check(_lib().oq_frontier(n, k, None, None, 0, _ct.byref(ln)), "oq_frontier(size)")
    return ln.value


def frontier(n: int, k: int):
    """Symmetry-reduced prefixes (int32[F, k]) and weights (uint8[F]) in canonical order."""
    size = frontier_size(n, k)
    pre = _np.zeros((max(size, 1), max(k, 1)), dtype=_np.int32)
    w = _np.zeros(max(size, 1), dtype=_np.uint8)
    ln = _ct.c_uint64()
    _check(_lib().oq_frontier(n, k, pre.ctypes.data_as(_ct.POINTER(_ct.c_int)),
                              w.ctypes.data_as(_ct.POINTER(_ct.c_uint8)), size, _ct.byref(ln)),
           "oq_frontier")
    return pre[:size, :k], w[:size]


def prefix_masks(n: int, prefix):
    a, p = _iarr(list(prefix) if len(prefix) else [0])
    c, l, r = _ct.c_uint32(), _ct.c_uint32(), _ct.c_uint32()
    _check(_lib().oq_prefix_masks(n, len(prefix), p, _ct.byref(c), _ct.byref(l), _ct.byref(r)),
           "oq_prefix_masks")
    return c.value, l.value, r.value


def frontier_masks(n: int, k: int):
    """(cols, ld, rd) uint32[F] for every frontier prefix, plus weights uint8[F]."""
    pre, w = frontier(n, k)
    return prefixes_masks(n, pre) + (w,)


def prefixes_masks(n: int, prefixes):
    """(cols, ld, rd) uint32[m] for each row of ``prefixes`` (int[m, k])."""
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    m, k = pre.shape
    cols = _np.zeros(max(m, 1), dtype=_np.uint32)
    ld = _np.zeros(max(m, 1), dtype=_np.uint32)
    rd = _np.zeros(max(m, 1), dtype=_np.uint32)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    u32 = lambda a: a.ctypes.data_as(_ct.POINTER(_ct.c_uint32))  # noqa: E731
    _check(_lib().oq_prefixes_masks(n, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), m,
                                    u32(cols), u32(ld), u32(rd)), "oq_prefixes_masks")
    return cols[:m], ld[:m], rd[:m]


def count_prefixes(n: int, prefixes, threads: int = 1):
    """Completions and nodes of each row of ``prefixes`` (int[F, k])."""
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    if pre.ndim == 1:
        pre = pre.reshape(-1, 0) if pre.size == 0 else pre.reshape(1, -1)
    m, k = pre.shape
    counts = _np.zeros(max(m, 1), dtype=_np.uint64)
    nodes = _np.zeros(max(m, 1), dtype=_np.uint64)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    _check(_lib().oq_count_prefixes(n, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), m, threads,
                                    counts.ctypes.data_as(_ct.POINTER(_ct.c_uint64)),
                                    nodes.ctypes.data_as(_ct.POINTER(_ct.c_uint64))),
           "oq_count_prefixes")
    return counts[:m], nodes[:m]


# ---- the second search: n non-attacking kings, one per row and column ----

def kings(n: int):
    """The number of king placements (permutations with no two adjacent rows in
    adjacent columns) by plain backtracking, and its nodes from row 0."""
    c, nd = _ct.c_uint64(), _ct.c_uint64()
    _check(_lib().oqk_count_prefix(n, 0, None, _ct.byref(c), _ct.byref(nd)), "oqk_count_prefix")
    return c.value, nd.value


def kings_brute_count(n: int, prefix=()):
    """Completions of a king prefix by enumerating permutations (n <= 11)."""
    a, p = _iarr(list(prefix) if len(prefix) else [0])
    c = _ct.c_uint64()
    _check(_lib().oqk_brute_count(n, len(prefix), p, _ct.byref(c)), "oqk_brute_count")
    return c.value


def kings_frontier_size(n: int, k: int) -> int:
    ln = _ct.c_uint64()
    _check(_lib().oqk_frontier(n, k, None, None, 0, _ct.byref(ln)), "oqk_frontier(size)")
    return ln.value


def kings_frontier(n: int, k: int):
    """Symmetry-reduced king prefixes (int32[F, k]) and weights (uint8[F])."""
    size = kings_frontier_size(n, k)
    pre = _np.zeros((max(size, 1), max(k, 1)), dtype=_np.int32)
    w = _np.zeros(max(size, 1), dtype=_np.uint8)
    ln = _ct.c_uint64()
    _check(_lib().oqk_frontier(n, k, pre.ctypes.data_as(_ct.POINTER(_ct.c_int)),
                               w.ctypes.data_as(_ct.POINTER(_ct.c_uint8)), size, _ct.byref(ln)),
           "oqk_frontier")
    return pre[:size, :k], w[:size]


def kings_prefixes_masks(n: int, prefixes):
    """(cols, ld, rd) uint32[m] that each king prefix casts on its next row."""
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    m, k = pre.shape
    cols = _np.zeros(max(m, 1), dtype=_np.uint32)
    ld = _np.zeros(max(m, 1), dtype=_np.uint32)
    rd = _np.zeros(max(m, 1), dtype=_np.uint32)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    u32 = lambda a: a.ctypes.data_as(_ct.POINTER(_ct.c_uint32))  # noqa: E731
    _check(_lib().oqk_prefixes_masks(n, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), m,
                                     u32(cols), u32(ld), u32(rd)), "oqk_prefixes_masks")
    return cols[:m], ld[:m], rd[:m]


def kings_count_prefixes(n: int, prefixes, threads: int = 1):
    """Completions and nodes (rows k..n-2) of each king prefix."""
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    if pre.ndim == 1:
        pre = pre.reshape(-1, 0) if pre.size == 0 else pre.reshape(1, -1)
    m, k = pre.shape
    counts = _np.zeros(max(m, 1), dtype=_np.uint64)
    nodes = _np.zeros(max(m, 1), dtype=_np.uint64)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    _check(_lib().oqk_count_prefixes(n, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), m,
                                     threads, counts.ctypes.data_as(_ct.POINTER(_ct.c_uint64)),
                                     nodes.ctypes.data_as(_ct.POINTER(_ct.c_uint64))),
           "oqk_count_prefixes")
    return counts[:m], nodes[:m]


# ---- the third search: permanents of 0/1 matrices ----

def _matrix(a):
    m = _np.ascontiguousarray(_np.asarray(a, dtype=_np.uint8))
    if m.ndim != 2 or m.shape[0] != m.shape[1] or m.shape[0] < 1:
        raise OracleError("the matrix must be n x n with n >= 1")
    return m, m.shape[0], m.ctypes.data_as(_ct.POINTER(_ct.c_uint8))


def permanent(a):
    """The permanent of the 0/1 matrix ``a`` (uint8[n, n]) by plain backtracking
    over the rows, and its nodes (placements in rows 0..n-3)."""
    m, n, p = _matrix(a)
    c, nd = _ct.c_uint64(), _ct.c_uint64()
    _check(_lib().oqp_count_prefix(n, p, 0, None, _ct.byref(c), _ct.byref(nd)),
           "oqp_count_prefix")
    return c.value, nd.value


def perm_frontier_size(a, k: int) -> int:
    m, n, p = _matrix(a)
    ln = _ct.c_uint64()
    _check(_lib().oqp_frontier(n, p, k, None, None, 0, _ct.byref(ln)), "oqp_frontier(size)")
    return ln.value


def perm_frontier(a, k: int):
    """Every prefix of length k (int32[F, k]): rows 0..k-1 in allowed, distinct
    columns, lexicographic."""
    m, n, p = _matrix(a)
    size = perm_frontier_size(m, k)
    pre = _np.zeros((max(size, 1), max(k, 1)), dtype=_np.int32)
    ln = _ct.c_uint64()
    _check(_lib().oqp_frontier(n, p, k, pre.ctypes.data_as(_ct.POINTER(_ct.c_int)), None, size,
                               _ct.byref(ln)), "oqp_frontier")
    return pre[:size, :k]


def perm_prefixes_cols(n: int, prefixes):
    """The used-column set (uint32[m], bit c = column c) of each prefix."""
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    m, k = pre.shape
    cols = _np.zeros(max(m, 1), dtype=_np.uint32)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    _check(_lib().oqp_prefixes_cols(n, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), m,
                                    cols.ctypes.data_as(_ct.POINTER(_ct.c_uint32))),
           "oqp_prefixes_cols")
    return cols[:m]


def perm_count_prefixes(a, prefixes, threads: int = 1):
    """Completions and nodes (rows k..n-3) of each prefix of the permanent search."""
    m, n, p = _matrix(a)
    pre = _np.ascontiguousarray(_np.asarray(prefixes, dtype=_np.int32))
    if pre.ndim == 1:
        pre = pre.reshape(-1, 0) if pre.size == 0 else pre.reshape(1, -1)
    cnt, k = pre.shape
    counts = _np.zeros(max(cnt, 1), dtype=_np.uint64)
    nodes = _np.zeros(max(cnt, 1), dtype=_np.uint64)
    buf = pre if pre.size else _np.zeros(1, dtype=_np.int32)
    _check(_lib().oqp_count_prefixes(n, p, k, buf.ctypes.data_as(_ct.POINTER(_ct.c_int)), cnt,
                                     threads, counts.ctypes.data_as(_ct.POINTER(_ct.c_uint64)),
                                     nodes.ctypes.data_as(_ct.POINTER(_ct.c_uint64))),
           "oqp_count_prefixes")
    return counts[:cnt], nodes[:cnt]


def permanent_ryser(a):
    """The permanent of ``a`` by Ryser's inclusion-exclusion formula (exact in
    128-bit arithmetic, n <= 20): independent of the search above."""
    m, n, p = _matrix(a)
    c = _ct.c_uint64()
    _check(_lib().oqp_ryser(n, p, _ct.byref(c)), "oqp_ryser")
    return c.value
