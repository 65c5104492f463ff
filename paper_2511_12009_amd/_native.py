"""ctypes declarations of libnq.so and the Python-level wrappers."""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libnq.so")

NQ_OK, NQ_EINVAL, NQ_ERANGE, NQ_ENOMEM, NQ_EDEVICE, NQ_EAGAIN, NQ_EFULL, NQ_ENOENT = (
    0, -1, -2, -3, -4, -5, -6, -7)
MODES = {"auto": 0, "plain": 1, "persistent": 2}
COUNT_INVALID = 0xFFFFFFFFFFFFFFFF


class NQError(RuntimeError):
    """A libnq call returned a negative status."""

    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


class NqOpts(ct.Structure):
    _fields_ = [
        ("depth", ct.c_uint32),
        ("mode", ct.c_uint32),
        ("wg_size", ct.c_uint32),
        ("waves_per_cu", ct.c_uint32),
        ("refill_every", ct.c_uint32),
        ("flags", ct.c_uint32),
        ("stream", ct.c_void_p),
        ("counts_out", ct.POINTER(ct.c_uint64)),
        ("counts_capacity", ct.c_uint64),
        ("kernel_ms_out", ct.POINTER(ct.c_double)),
        ("d_nodes", ct.c_void_p),
        ("claim", ct.c_uint32),
    ]


class NqTuned(ct.Structure):
    _fields_ = [
        ("depth", ct.c_uint32),
        ("waves_per_cu", ct.c_uint32),
        ("refill_every", ct.c_uint32),
        ("trials", ct.c_uint32),
        ("ms", ct.c_double),
        ("count", ct.c_uint64),
        ("claim", ct.c_uint32),
        ("wg_size", ct.c_uint32),
        ("chunks", ct.c_uint32),
        ("reserved", ct.c_uint32),
    ]


class NqTuneTrial(ct.Structure):
    _fields_ = [
        ("depth", ct.c_uint32),
        ("wg_size", ct.c_uint32),
        ("waves_per_cu", ct.c_uint32),
        ("refill_every", ct.c_uint32),
        ("claim", ct.c_uint32),
        ("chunks", ct.c_uint32),
        ("ms", ct.c_double),
        ("subproblems", ct.c_uint64),
    ]


class NqRequest(ct.Structure):
    _fields_ = [
        ("kind", ct.c_uint32),
        ("n", ct.c_uint32),
        ("depth", ct.c_uint32),
        ("reserved", ct.c_uint32),
        ("start", ct.c_uint64),
        ("len", ct.c_uint64),
    ]


class NqResult(ct.Structure):
    _fields_ = [
        ("status", ct.c_int32),
        ("reserved", ct.c_uint32),
        ("count", ct.c_uint64),
        ("entries", ct.c_uint64),
        ("t_submit_ns", ct.c_uint64),
        ("t_admit_ns", ct.c_uint64),
        ("t_done_ns", ct.c_uint64),
    ]


REQ_COUNT, REQ_SLICE = 1, 2

_LIB = None


def lib():
    """The loaded libnq.so; raises NQError if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(library_path):
            raise NQError(NQ_EINVAL, "load",
                          f"{library_path} is missing; run python -m paper_2511_12009_amd.build")
        L = ct.CDLL(library_path)
        u32, u64, vp = ct.c_uint32, ct.c_uint64, ct.c_void_p
        pu32, pu64, pu8 = ct.POINTER(u32), ct.POINTER(u64), ct.POINTER(ct.c_uint8)
        L.nq_strerror.argtypes = [ct.c_int]
        L.nq_strerror.restype = ct.c_char_p
        L.nq_last_hip_error.argtypes = []
        L.nq_last_hip_error.restype = ct.c_int
        L.nq_frontier.argtypes = [u32, u32, pu32, pu32, pu32, pu8, u64, pu64]
        L.nq_frontier.restype = ct.c_int
        L.nq_kings_frontier.argtypes = [u32, u32, pu32, pu32, pu32, pu8, u64, pu64]
        L.nq_kings_frontier.restype = ct.c_int
        L.nq_frontier_runs.argtypes = [u32, u32, pu64, u32, pu32]
        L.nq_frontier_runs.restype = ct.c_int
        L.nq_expand.argtypes = [u32, u32, vp, vp, vp, vp, u64, vp, vp, vp, vp, u64, pu64, vp]
        L.nq_expand.restype = ct.c_int
        L.nq_count.argtypes = [u32, ct.POINTER(NqOpts), pu64]
        L.nq_count.restype = ct.c_int
        L.nq_count_subproblems.argtypes = [u32, vp, vp, vp, vp, u64, vp, vp, ct.POINTER(NqOpts)]
        L.nq_count_subproblems.restype = ct.c_int
        L.nq_count_subproblems_noalloc.argtypes = [u32, vp, vp, vp, vp, u64, vp, vp,
                                                   ct.POINTER(NqOpts)]
        L.nq_count_subproblems_noalloc.restype = ct.c_int
        L.nq_count_batch.argtypes = [u32, pu32, pu32, ct.POINTER(NqOpts), pu64]
        L.nq_count_batch.restype = ct.c_int
        L.nq_serve_create.argtypes = [ct.POINTER(NqOpts), u64, ct.POINTER(vp)]
        L.nq_serve_create.restype = ct.c_int
        L.nq_serve_submit.argtypes = [vp, ct.POINTER(NqRequest), pu64]
        L.nq_serve_submit.restype = ct.c_int
        L.nq_serve_poll.argtypes = [vp, u64, ct.POINTER(NqResult)]
        L.nq_serve_poll.restype = ct.c_int
        L.nq_serve_wait.argtypes = [vp, u64, ct.POINTER(NqResult), u64]
        L.nq_serve_wait.restype = ct.c_int
        L.nq_serve_destroy.argtypes = [vp]
        L.nq_serve_destroy.restype = ct.c_int
        L.nq_autotune.argtypes = [u32, u32, u32, ct.c_double, ct.POINTER(NqTuned)]
        L.nq_autotune.restype = ct.c_int
        L.nq_autotune_trials.argtypes = [u32, u32, u32, ct.c_double, ct.POINTER(NqTuned),
                                         ct.POINTER(NqTuneTrial), u32, pu32]
        L.nq_autotune_trials.restype = ct.c_int
        L.nq_tuned_lookup.argtypes = [u32, ct.POINTER(NqTuned)]
        L.nq_tuned_lookup.restype = ct.c_int
        L.nq_batch_create.argtypes = [u32, pu32, pu32, ct.POINTER(NqOpts), ct.POINTER(vp)]
        L.nq_batch_create.restype = ct.c_int
        L.nq_batch_run.argtypes = [vp, pu64, ct.POINTER(ct.c_double)]
        L.nq_batch_run.restype = ct.c_int
        L.nq_batch_entries.argtypes = [vp]
        L.nq_batch_entries.restype = u64
        L.nq_batch_destroy.argtypes = [vp]
        L.nq_batch_destroy.restype = ct.c_int
        L.nq_count_resumable.argtypes = [u32, ct.POINTER(NqOpts), ct.c_char_p, u32, u32, pu64, pu32]
        L.nq_count_resumable.restype = ct.c_int
        L.nq_count_resumable_wide.argtypes = [u32, ct.POINTER(NqOpts), ct.c_char_p, u32, u32, pu64,
                                              pu32]
        L.nq_count_resumable_wide.restype = ct.c_int
        L.nq_set_loop_form.argtypes = [ct.c_int, ct.POINTER(ct.c_int)]
        L.nq_set_loop_form.restype = ct.c_int
        pd = ct.POINTER(ct.c_double)
        L.nq_ubench_valu.argtypes = [u32, u32, u32, u64, pd, pd]
        L.nq_ubench_valu.restype = ct.c_int
        L.nq_ubench_lds.argtypes = [u32, u32, u32, u32, u32, u64, pd]
        L.nq_ubench_lds.restype = ct.c_int
        L.nq_perm_frontier.argtypes = [u32, pu32, u32, pu32, u64, pu64]
        L.nq_perm_frontier.restype = ct.c_int
        L.nq_perm_count_subproblems.argtypes = [u32, pu32, vp, u64, u32, vp, vp,
                                                ct.POINTER(NqOpts)]
        L.nq_perm_count_subproblems.restype = ct.c_int
        L.nq_perm_count.argtypes = [u32, pu32, ct.POINTER(NqOpts), pu64]
        L.nq_perm_count.restype = ct.c_int
        L.nq_perm_set_step.argtypes = [ct.c_int, ct.POINTER(ct.c_int)]
        L.nq_perm_set_step.restype = ct.c_int
        _LIB = L
    return _LIB


def _check(rc: int, what: str):
    if rc != NQ_OK:
        L = lib()
        msg = L.nq_strerror(rc).decode()
        if rc == NQ_EDEVICE:
            msg += f" (hipError {L.nq_last_hip_error()})"
        raise NQError(rc, what, msg)


FLAG_FORWARD_ORDER = 1
FLAG_KINGS = 2
FLAG_WIDE_TOTAL = 4
FLAG_SERVE_RESERVE = 8


def _opts(depth=0, mode="persistent", wg_size=0, waves_per_cu=0, refill_every=0, stream=None,
          flags=0, claim=0):
    o = NqOpts()
    o.claim = claim
    o.flags = flags
    o.depth = depth
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.wg_size = wg_size
    o.waves_per_cu = waves_per_cu
    o.refill_every = refill_every
    o.stream = stream
    return o


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def frontier_size(n: int, depth: int, kings: bool = False) -> int:
    """F of the (n, depth) frontier (kings=True: of the kings search)."""
    fn = lib().nq_kings_frontier if kings else lib().nq_frontier
    ln = ct.c_uint64()
    _check(fn(n, depth, None, None, None, None, 0, ct.byref(ln)), "frontier size")
    return ln.value


def frontier_runs(n: int, depth: int):
    """Start offset of each row-0 column's run of entries, followed by F."""
    cnt = ct.c_uint32()
    _check(lib().nq_frontier_runs(n, depth, None, 0, ct.byref(cnt)), "nq_frontier_runs")
    off = np.zeros(cnt.value + 1, np.uint64)
    _check(lib().nq_frontier_runs(n, depth, off.ctypes.data_as(ct.POINTER(ct.c_uint64)),
                                  len(off), ct.byref(cnt)), "nq_frontier_runs")
    return [int(x) for x in off]


def frontier(n: int, depth: int, kings: bool = False):
    """(cols, ld, rd) uint32[F] and weight uint8[F] in canonical order (host arrays);
    kings=True: the kings search's frontier (nq_kings_frontier)."""
    fn = lib().nq_kings_frontier if kings else lib().nq_frontier
    f = frontier_size(n, depth, kings)
    ln = ct.c_uint64()
    cols = np.zeros(max(f, 1), np.uint32)
    ld = np.zeros(max(f, 1), np.uint32)
    rd = np.zeros(max(f, 1), np.uint32)
    w = np.zeros(max(f, 1), np.uint8)
    p32 = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_uint32))  # noqa: E731
    _check(fn(n, depth, p32(cols), p32(ld), p32(rd), w.ctypes.data_as(ct.POINTER(ct.c_uint8)), f,
              ct.byref(ln)), "nq_kings_frontier" if kings else "nq_frontier")
    return cols[:f], ld[:f], rd[:f], w[:f]


def expand(n: int, rows: int, cols, ld, rd, weight=None, stream=None):
    """Children `rows` rows below device-resident triples (nq_expand): returns
    (cols, ld, rd, weight) int32/uint8 CUDA tensors in canonical order."""
    import torch
    length = cols.numel()
    st = _stream_handle(stream)
    cnt = ct.c_uint64()
    wp = None if weight is None else weight.data_ptr()
    _check(lib().nq_expand(n, rows, cols.data_ptr(), ld.data_ptr(), rd.data_ptr(), wp, length,
                           None, None, None, None, 0, ct.byref(cnt), st), "nq_expand")
    m = cnt.value
    oc = torch.empty(max(m, 1), dtype=torch.int32, device=cols.device)
    ol = torch.empty_like(oc)
    orr = torch.empty_like(oc)
    ow = torch.empty(max(m, 1), dtype=torch.uint8, device=cols.device)
    _check(lib().nq_expand(n, rows, cols.data_ptr(), ld.data_ptr(), rd.data_ptr(), wp, length,
                           oc.data_ptr(), ol.data_ptr(), orr.data_ptr(), ow.data_ptr(), m,
                           ct.byref(cnt), st), "nq_expand")
    return oc[:m], ol[:m], orr[:m], ow[:m]


def count(n: int, depth: int = 0, mode="persistent", wg_size: int = 0, waves_per_cu: int = 0,
          refill_every: int = 0, counts: bool = False, timing: bool = False, stream=None,
          forward: bool = False, claim: int = 0, kings: bool = False):
    """Q(n) (kings=True: the number of ways to place n non-attacking kings, one
    per row and column).  With counts=True also the per-subproblem counts (numpy
    uint64, frontier order); with timing=True also the DFS kernel time in ms.
    Synchronous."""
    o = _opts(depth, mode, wg_size, waves_per_cu, refill_every,
              stream if stream is None else _stream_handle(stream),
              (FLAG_FORWARD_ORDER if forward else 0) | (FLAG_KINGS if kings else 0), claim)
    buf = None
    if counts:
        if depth == 0:
            raise ValueError("counts=True needs an explicit depth")
        buf = np.zeros(max(frontier_size(n, depth, kings), 1), np.uint64)
        o.counts_out = buf.ctypes.data_as(ct.POINTER(ct.c_uint64))
        o.counts_capacity = len(buf)
    ms = ct.c_double(0.0)
    if timing:
        o.kernel_ms_out = ct.pointer(ms)
    total = ct.c_uint64()
    _check(lib().nq_count(n, ct.byref(o), ct.byref(total)), "nq_count")
    out = [total.value]
    if counts:
        out.append(buf[:frontier_size(n, depth, kings)])
    if timing:
        out.append(ms.value)
    return out[0] if len(out) == 1 else tuple(out)


def count_subproblems(n: int, cols, ld, rd, weight=None, counts=None, total=None,
                      depth: int = 0, mode="persistent", wg_size: int = 0,
                      waves_per_cu: int = 0, refill_every: int = 0, stream=None,
                      timing: bool = False, nodes=None, forward: bool = False, claim: int = 0,
                      kings: bool = False, wide: bool = False):
    """Counts every subtree of device-resident triples (torch int32 CUDA tensors).

    ``wide=True`` (NQ_FLAG_WIDE_TOTAL; needed for n > 28): ``total`` is int64[2],
    a 128-bit total (low word first) increased with carry.

    ``counts`` (int64[F]) and ``total`` (int64[1], accumulated) are torch tensors
    allocated here when not given; ``counts=False`` requests no per-entry counts.  ``depth`` promises that every triple has at
    least that many queens placed (sizes the LDS stack).  Asynchronous on
    ``stream`` (default: torch's current stream) unless timing=True.
    ``nodes`` (int64[F] CUDA tensor) receives the DFS nodes of every entry.
    Returns (counts, total) or (counts, total, kernel_ms).
    """
    import torch
    length = cols.numel()
    for t in (cols, ld, rd):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.numel() != length:
            raise ValueError("cols, ld, rd must be contiguous int32 CUDA tensors of one length")
    if weight is not None and (weight.dtype != torch.uint8 or weight.numel() != length):
        raise ValueError("weight must be a uint8 CUDA tensor of the same length")
    if counts is None:
        counts = torch.empty(length, dtype=torch.int64, device=cols.device)
    if total is None:
        total = torch.zeros(2 if wide else 1, dtype=torch.int64, device=cols.device)
    if total is not False and total.numel() < (2 if wide else 1):
        raise ValueError("total needs two int64 words with wide=True")
    o = _opts(depth, mode, wg_size, waves_per_cu, refill_every, _stream_handle(stream),
              (FLAG_FORWARD_ORDER if forward else 0) | (FLAG_KINGS if kings else 0) |
              (FLAG_WIDE_TOTAL if wide else 0), claim)
    if nodes is not None:
        if nodes.dtype != torch.int64 or nodes.numel() != length or not nodes.is_cuda:
            raise ValueError("nodes must be an int64 CUDA tensor of the same length")
        o.d_nodes = nodes.data_ptr()
    ms = ct.c_double(0.0)
    if timing:
        o.kernel_ms_out = ct.pointer(ms)
    _check(lib().nq_count_subproblems(
        n, cols.data_ptr(), ld.data_ptr(), rd.data_ptr(),
        None if weight is None else weight.data_ptr(), length,
        None if counts is False else counts.data_ptr(),
        None if total is False else total.data_ptr(), ct.byref(o)),
        "nq_count_subproblems")
    return (counts, total, ms.value) if timing else (counts, total)


def perm_rows(a):
    """The rows of a 0/1 matrix (n x n, anything numpy reads) as the library
    takes them: uint32[n], bit c of word r = a[r][c] != 0."""
    m = np.asarray(a)
    if m.ndim != 2 or m.shape[0] != m.shape[1] or not 1 <= m.shape[0] <= 32:
        raise ValueError("the matrix must be n x n with 1 <= n <= 32")
    bits = (m != 0).astype(np.uint64) << np.arange(m.shape[0], dtype=np.uint64)
    return np.ascontiguousarray(bits.sum(axis=1).astype(np.uint32))


def _rows_arg(a):
    rows = perm_rows(a)
    return rows, len(rows), rows.ctypes.data_as(ct.POINTER(ct.c_uint32))


def perm_frontier(a, depth: int):
    """Used-column sets (uint32[F], host) of every assignment of rows
    0..depth-1 of the 0/1 matrix `a` (nq_perm_frontier), lexicographic."""
    rows, n, rp = _rows_arg(a)
    ln = ct.c_uint64()
    _check(lib().nq_perm_frontier(n, rp, depth, None, 0, ct.byref(ln)), "nq_perm_frontier")
    f = ln.value
    cols = np.zeros(max(f, 1), np.uint32)
    _check(lib().nq_perm_frontier(n, rp, depth, cols.ctypes.data_as(ct.POINTER(ct.c_uint32)),
                                  f, ct.byref(ln)), "nq_perm_frontier")
    return cols[:f]


def perm_count(a, depth: int = 0, mode="persistent", wg_size: int = 0, waves_per_cu: int = 0,
               refill_every: int = 0, claim: int = 0, timing: bool = False, stream=None):
    """The permanent of the 0/1 matrix `a` (nq_perm_count); with timing=True
    also the DFS kernel time in ms.  Synchronous."""
    rows, n, rp = _rows_arg(a)
    o = _opts(depth, mode, wg_size, waves_per_cu, refill_every,
              stream if stream is None else _stream_handle(stream), 0, claim)
    ms = ct.c_double(0.0)
    if timing:
        o.kernel_ms_out = ct.pointer(ms)
    total = ct.c_uint64()
    _check(lib().nq_perm_count(n, rp, ct.byref(o), ct.byref(total)), "nq_perm_count")
    return (total.value, ms.value) if timing else total.value


def perm_count_subproblems(a, cols, depth: int, counts=None, total=None, nodes=None,
                           mode="persistent", wg_size: int = 0, waves_per_cu: int = 0,
                           refill_every: int = 0, claim: int = 0, stream=None,
                           timing: bool = False):
    """Counts below device-resident used-column sets `cols` (int32 CUDA tensor;
    every entry has `depth` rows assigned) of the matrix `a`
    (nq_perm_count_subproblems).  ``counts`` (int64[F]) and ``total``
    (int64[1], accumulated) are allocated when not given; ``counts=False``
    requests none; ``nodes`` (int64[F]) receives the nodes of every entry.
    Returns (counts, total) or (counts, total, kernel_ms)."""
    import torch
    rows, n, rp = _rows_arg(a)
    length = cols.numel()
    if not cols.is_cuda or cols.dtype != torch.int32 or not cols.is_contiguous():
        raise ValueError("cols must be a contiguous int32 CUDA tensor")
    if counts is None:
        counts = torch.empty(length, dtype=torch.int64, device=cols.device)
    if total is None:
        total = torch.zeros(1, dtype=torch.int64, device=cols.device)
    o = _opts(depth, mode, wg_size, waves_per_cu, refill_every, _stream_handle(stream), 0, claim)
    if nodes is not None:
        if nodes.dtype != torch.int64 or nodes.numel() != length or not nodes.is_cuda:
            raise ValueError("nodes must be an int64 CUDA tensor of the same length")
        o.d_nodes = nodes.data_ptr()
    ms = ct.c_double(0.0)
    if timing:
        o.kernel_ms_out = ct.pointer(ms)
    _check(lib().nq_perm_count_subproblems(
        n, rp, cols.data_ptr(), length, depth,
        None if counts is False else counts.data_ptr(),
        None if total is False else total.data_ptr(), ct.byref(o)),
        "nq_perm_count_subproblems")
    return (counts, total, ms.value) if timing else (counts, total)


def count_resumable(n: int, path: str, chunks: int = 0, max_chunks: int = 0, depth: int = 0,
                    mode="persistent", waves_per_cu: int = 0, refill_every: int = 0,
                    claim: int = 0, wide: bool = False):
    """nq_count_resumable: Q(n) in chunks whose progress is kept in the file
    `path`; returns (total, chunks_done, finished).  While not finished, total
    is the weighted count of the chunks done so far; call again to go on.
    wide=True calls nq_count_resumable_wide (boards up to 31, 128-bit total)."""
    o = _opts(depth, mode, 0, waves_per_cu, refill_every, None, 0, claim)
    words = (ct.c_uint64 * 2)()
    done = ct.c_uint32()
    fn = lib().nq_count_resumable_wide if wide else lib().nq_count_resumable
    rc = fn(n, ct.byref(o), os.fsencode(path), chunks, max_chunks, words, ct.byref(done))
    total = int(words[0]) | (int(words[1]) << 64)
    if rc == NQ_EAGAIN:
        return total, done.value, False
    _check(rc, "nq_count_resumable_wide" if wide else "nq_count_resumable")
    return total, done.value, True


def set_loop_form(form: int) -> int:
    """nq_set_loop_form: the DFS inner-loop form of launches planned from now on
    (-1 = default; 0 to 7); returns the form that was in use."""
    prev = ct.c_int(0)
    _check(lib().nq_set_loop_form(int(form), ct.byref(prev)), "nq_set_loop_form")
    return prev.value


def perm_set_step(step: int) -> int:
    """nq_perm_set_step: the permanent kernel's inner step of launches from now
    on (-1 = default; 0, 1 or 2); returns the step that was in use."""
    prev = ct.c_int(0)
    _check(lib().nq_perm_set_step(int(step), ct.byref(prev)), "nq_perm_set_step")
    return prev.value


def ubench_valu(op: int, chains: int, waves_per_simd: int, iters: int):
    """nq_ubench_valu: (kernel ms, mean shader-clock cycles of a wave's loop)."""
    ms, cyc = ct.c_double(), ct.c_double()
    _check(lib().nq_ubench_valu(op, chains, waves_per_simd, iters, ct.byref(ms), ct.byref(cyc)),
           "nq_ubench_valu")
    return ms.value, cyc.value


def ubench_lds(layout: int, active_lanes: int, waves_per_cu: int, frames: int, iters: int,
               op: int = 0):
    """nq_ubench_lds: kernel ms."""
    ms = ct.c_double()
    _check(lib().nq_ubench_lds(layout, op, active_lanes, waves_per_cu, frames, iters,
                               ct.byref(ms)), "nq_ubench_lds")
    return ms.value


def count_batch(ns, depths=None, mode="persistent", wg_size: int = 0, waves_per_cu: int = 0,
                refill_every: int = 0, stream=None, claim: int = 0):
    """[Q(n) for n in ns], all instances in one persistent launch."""
    ns_a = np.ascontiguousarray(np.asarray(ns, dtype=np.uint32))
    d_a = None if depths is None else np.ascontiguousarray(np.asarray(depths, dtype=np.uint32))
    out = np.zeros(max(len(ns_a), 1), np.uint64)
    o = _opts(0, mode, wg_size, waves_per_cu, refill_every,
              stream if stream is None else _stream_handle(stream), 0, claim)
    p32 = lambda a: None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_uint32))  # noqa: E731
    _check(lib().nq_count_batch(len(ns_a), p32(ns_a), p32(d_a), ct.byref(o),
                                out.ctypes.data_as(ct.POINTER(ct.c_uint64))), "nq_count_batch")
    return [int(x) for x in out[:len(ns_a)]]


class Batch:
    """A replayable batch plan (nq_batch_create / nq_batch_run / nq_batch_destroy)."""

    def __init__(self, ns, depths=None, depth: int = 0, wg_size: int = 0, waves_per_cu: int = 0,
                 refill_every: int = 0, forward: bool = False, claim: int = 0):
        self.ns = np.ascontiguousarray(np.asarray(ns, dtype=np.uint32))
        self._d = None if depths is None else np.ascontiguousarray(np.asarray(depths, np.uint32))
        o = _opts(depth, "persistent", wg_size, waves_per_cu, refill_every, None,
                  FLAG_FORWARD_ORDER if forward else 0, claim)
        h = ct.c_void_p()
        p32 = lambda a: None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_uint32))  # noqa
        _check(lib().nq_batch_create(len(self.ns), p32(self.ns), p32(self._d), ct.byref(o),
                                     ct.byref(h)), "nq_batch_create")
        self._h = h

    @property
    def entries(self) -> int:
        return int(lib().nq_batch_entries(self._h))

    def run(self, timing: bool = False):
        out = np.zeros(len(self.ns), np.uint64)
        ms = ct.c_double(0.0)
        _check(lib().nq_batch_run(self._h, out.ctypes.data_as(ct.POINTER(ct.c_uint64)),
                                  ct.byref(ms) if timing else None), "nq_batch_run")
        res = [int(x) for x in out]
        return (res, ms.value) if timing else res

    def close(self):
        if self._h:
            _check(lib().nq_batch_destroy(self._h), "nq_batch_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tuned(t) -> dict:
    return {"depth": t.depth, "wg_size": t.wg_size, "waves_per_cu": t.waves_per_cu,
            "refill_every": t.refill_every, "claim": t.claim, "trials": t.trials, "ms": t.ms,
            "count": t.count, "chunks": t.chunks}


def autotune(n: int, depth_lo: int = 0, depth_hi: int = 0, budget_ms: float = 0.0,
             table: bool = False) -> dict:
    """Measured best depth / workgroup size / waves per CU / visit interval /
    claim block for n (nq_autotune; for n = 21..23 the depth of the chunked
    count, "chunks" > 0); table=True adds every trial (nq_autotune_trials)
    under "table"."""
    t = NqTuned()
    if not table:
        _check(lib().nq_autotune(n, depth_lo, depth_hi, budget_ms, ct.byref(t)), "nq_autotune")
        return _tuned(t)
    cap = 256
    rows = (NqTuneTrial * cap)()
    cnt = ct.c_uint32()
    _check(lib().nq_autotune_trials(n, depth_lo, depth_hi, budget_ms, ct.byref(t), rows, cap,
                                    ct.byref(cnt)), "nq_autotune_trials")
    out = _tuned(t)
    out["table"] = [{"depth": r.depth, "wg_size": r.wg_size, "waves_per_cu": r.waves_per_cu,
                     "refill_every": r.refill_every, "claim": r.claim, "chunks": r.chunks,
                     "ms": r.ms, "subproblems": r.subproblems} for r in rows[:cnt.value]]
    return out


def tuned_lookup(n: int):
    """nq_tuned_lookup: the tuning remembered for n in this process, or None."""
    t = NqTuned()
    rc = lib().nq_tuned_lookup(n, ct.byref(t))
    if rc == NQ_ENOENT:
        return None
    _check(rc, "nq_tuned_lookup")
    return _tuned(t)


class Server:
    """Continuous-batching count server (nq_serve_*).

    reserve=True (NQ_FLAG_SERVE_RESERVE) favours the latency of quick requests
    (COUNTs of boards up to 16) over throughput.
    submit_count(n, depth=0) / submit_slice(n, depth, start, length) return a
    ticket; poll(ticket) returns None while the request runs, else a dict with
    status, count, entries and the submit/admit/done timestamps (ns).
    """

    def __init__(self, hbm_budget: int = 0, max_frames: int = 0, wg_size: int = 0,
                 waves_per_cu: int = 0, refill_every: int = 0, reserve: bool = False):
        o = _opts(max_frames, "persistent", wg_size, waves_per_cu, refill_every, None)
        if reserve:                      # NQ_FLAG_SERVE_RESERVE: latency of quick requests first
            o.flags |= FLAG_SERVE_RESERVE
        h = ct.c_void_p()
        _check(lib().nq_serve_create(ct.byref(o), hbm_budget, ct.byref(h)), "nq_serve_create")
        self._h = h

    def _submit(self, kind, n, depth, start, length):
        rq = NqRequest(kind, n, depth, 0, start, length)
        t = ct.c_uint64()
        _check(lib().nq_serve_submit(self._h, ct.byref(rq), ct.byref(t)), "nq_serve_submit")
        return t.value

    def submit_count(self, n: int, depth: int = 0) -> int:
        return self._submit(REQ_COUNT, n, depth, 0, 0)

    def submit_slice(self, n: int, depth: int, start: int, length: int) -> int:
        return self._submit(REQ_SLICE, n, depth, start, length)

    @staticmethod
    def _res(r):
        return {"status": r.status, "count": r.count, "entries": r.entries,
                "t_submit_ns": r.t_submit_ns, "t_admit_ns": r.t_admit_ns,
                "t_done_ns": r.t_done_ns}

    def poll(self, ticket: int):
        r = NqResult()
        rc = lib().nq_serve_poll(self._h, ticket, ct.byref(r))
        if rc == NQ_EAGAIN:
            return None
        _check(rc, "nq_serve_poll")
        return self._res(r)

    def wait(self, ticket: int, timeout_s: float = 60.0):
        r = NqResult()
        rc = lib().nq_serve_wait(self._h, ticket, ct.byref(r), int(timeout_s * 1e9))
        if rc == NQ_EAGAIN:
            raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
        _check(rc, "nq_serve_wait")
        return self._res(r)

    def close(self):
        if self._h:
            h, self._h = self._h, None
            _check(lib().nq_serve_destroy(h), "nq_serve_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
