"""Exact N-Queens counting on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libnq.so`` (see ``include/nq.h``): argument
marshalling only, every step of the counting runs in the library's host code
and HIP kernels.  PyTorch is used for device buffers and streams.  The library
must have been built (``python -m paper_2511_12009_amd.build``); importing the
binding without it raises ``NQError``.

Functions (same names as the C entry points, without the ``nq_`` prefix):
  frontier(n, depth)                         -> (cols, ld, rd, weight) numpy arrays
  frontier_size(n, depth)                    -> F
  frontier_runs(n, depth)                    -> start of each row-0 column's entries, then F
  expand(n, rows, cols, ld, rd, weight=None)  -> the frontier rows deeper, on the device
  count(n, depth=0, mode="persistent", ...)  -> Q(n)   (and counts / kernel ms)
  count_subproblems(n, cols, ld, rd, ...)    -> per-entry counts and weighted total
  count_batch(ns, depths=None, ...)          -> [Q(n) for n in ns]
  Batch(ns, depths=None).run()               -> replayable batch plan (HIP graph)
  autotune(n, depth_lo=0, depth_hi=0, table=False) -> measured best depth and launch shape
  tuned_lookup(n)                            -> the tuning nq_count uses for n, or None
  Server(...).submit_count / submit_slice / poll / wait -> continuous-batching serving
  count_resumable(n, path, ..., wide=False)  -> a count in chunks with a progress file
  ubench_valu / ubench_lds                   -> the microbenchmarks behind the roofline
  perm_count / perm_frontier / perm_count_subproblems -> the third search: permanents of
                                               0/1 matrices on the same engine
  perm_set_step(step)                        -> the permanent kernel's inner step (measurement)
"""
from ._native import (  # noqa: F401
    Batch,
    NQError,
    MODES,
    Server,
    autotune,
    count,
    count_batch,
    count_resumable,
    count_subproblems,
    expand,
    frontier,
    frontier_runs,
    frontier_size,
    set_loop_form,
    tuned_lookup,
    lib,
    library_path,
    perm_count,
    perm_count_subproblems,
    perm_frontier,
    perm_rows,
    perm_set_step,
    ubench_lds,
    ubench_valu,
)
