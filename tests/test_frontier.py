"""Host side of the library (no GPU needed): the C-ABI loads, exports every
declared symbol, and nq_frontier matches the oracle's frontier index by index."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import oracle
import paper_2511_12009_amd as nq
from conftest import ROOT, read_table


HEADERS = ("nq.h", "nq_ubench.h")


def _header_text(name):
    with open(os.path.join(ROOT, "include", name)) as f:
        return f.read()


def _declared_functions(name="nq.h"):
    text = _header_text(name)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(nq_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


@pytest.mark.parametrize("header", HEADERS)
def test_library_exports_every_declared_symbol(header):
    names = _declared_functions(header)
    assert len(names) >= 2
    if header == "nq.h":
        assert "nq_frontier" in names and "nq_count" in names and len(names) >= 6
    lib = ct.CDLL(nq.library_path)
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("header", HEADERS)
def test_every_declared_function_is_documented(header):
    """Each entry point of a C-ABI header carries its own documentation: its
    name appears in a comment, or a comment ends right above its declaration."""
    text = _header_text(header)
    comments = " ".join(re.findall(r"/\*.*?\*/", text, flags=re.S))
    for name in _declared_functions(header):
        if name in comments:
            continue
        decl = re.search(r"^[^\n]*\b" + name + r"\s*\(", text, flags=re.M)
        before = text[:decl.start()].rstrip()
        assert before.endswith("*/"), f"{name} has no documentation"


def test_strerror_covers_every_status():
    lib = nq.lib()
    for st in range(0, -8, -1):
        assert lib.nq_strerror(st).decode() not in ("", "unknown status")
    assert lib.nq_strerror(-99).decode() == "unknown status"


@pytest.mark.parametrize("n", range(1, 14))
def test_frontier_matches_oracle_every_depth(n):
    for k in range(0, n + 1):
        cols, ld, rd, w = nq.frontier(n, k)
        oc, ol, orr, ow = oracle.frontier_masks(n, k) if k else (None, None, None, None)
        if k == 0:
            assert list(cols) == [0] and list(w) == [1]
            continue
        assert len(cols) == len(oc) == oracle.frontier_size(n, k), (n, k)
        np.testing.assert_array_equal(cols, oc)
        np.testing.assert_array_equal(ld, ol)
        np.testing.assert_array_equal(rd, orr)
        np.testing.assert_array_equal(w, ow)


@pytest.mark.parametrize("n,k", [(14, 3), (17, 5), (16, 6), (19, 4)])
def test_frontier_matches_oracle_bench_shapes(n, k):
    cols, ld, rd, w = nq.frontier(n, k)
    oc, ol, orr, ow = oracle.frontier_masks(n, k)
    np.testing.assert_array_equal(cols, oc)
    np.testing.assert_array_equal(ld, ol)
    np.testing.assert_array_equal(rd, orr)
    np.testing.assert_array_equal(w, ow)


@pytest.mark.parametrize("n,k", [(29, 3), (30, 3), (31, 3), (31, 4)])
def test_frontier_beyond_64_bit_boards_matches_oracle(n, k):
    """Boards of 29..31 (beyond the 64-bit counts of Section 4.5, still 32-bit
    masks): the same prefixes, masks and weights as the oracle, index by index."""
    cols, ld, rd, w = nq.frontier(n, k)
    oc, ol, orr, ow = oracle.frontier_masks(n, k)
    np.testing.assert_array_equal(cols, oc)
    np.testing.assert_array_equal(ld, ol)
    np.testing.assert_array_equal(rd, orr)
    np.testing.assert_array_equal(w, ow)


def test_frontier_sizes_match_oracle():
    for n, k in [(20, 5), (20, 6), (21, 6), (18, 5), (19, 5)]:
        assert nq.frontier_size(n, k) == oracle.frontier_size(n, k)


def test_frontier_27_7_size_matches_run_log():
    for n, k, f in read_table("frontier_sizes.txt"):
        assert nq.frontier_size(int(n), int(k)) == int(f)


def test_frontier_partial_fill_reports_range():
    lib = nq.lib()
    n, k = 12, 4
    full = nq.frontier(n, k)
    cap = len(full[0]) // 3
    c = np.zeros(cap, np.uint32)
    l = np.zeros(cap, np.uint32)
    r = np.zeros(cap, np.uint32)
    w = np.zeros(cap, np.uint8)
    ln = ct.c_uint64()
    p = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_uint32))  # noqa: E731
    rc = lib.nq_frontier(n, k, p(c), p(l), p(r), w.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                         cap, ct.byref(ln))
    assert rc == -2 and ln.value == len(full[0])
    np.testing.assert_array_equal(c, full[0][:cap])
    np.testing.assert_array_equal(l, full[1][:cap])
    np.testing.assert_array_equal(r, full[2][:cap])
    np.testing.assert_array_equal(w, full[3][:cap])


def test_frontier_rejects_bad_arguments():
    lib = nq.lib()
    ln = ct.c_uint64()
    assert lib.nq_frontier(0, 0, None, None, None, None, 0, ct.byref(ln)) == -1
    assert lib.nq_frontier(32, 3, None, None, None, None, 0, ct.byref(ln)) == -1
    assert lib.nq_frontier(31, 3, None, None, None, None, 0, ct.byref(ln)) == 0
    assert lib.nq_frontier(8, 9, None, None, None, None, 0, ct.byref(ln)) == -1
    assert lib.nq_frontier(8, 3, None, None, None, None, 0, None) == -1


def test_count_entry_points_validate_before_touching_the_gpu():
    lib = nq.lib()
    out = ct.c_uint64()
    assert lib.nq_count(0, None, ct.byref(out)) == -1
    assert lib.nq_count(29, None, ct.byref(out)) == -1
    assert lib.nq_count(8, None, None) == -1
    assert lib.nq_count_subproblems(30, None, None, None, None, 5, None, None, None) == -1
    assert lib.nq_count_subproblems(8, None, None, None, None, 5, None, None, None) == -1
    # len == 0 is a valid empty call: nothing is launched
    assert lib.nq_count_subproblems(8, None, None, None, None, 0, None, None, None) == 0


def test_batch_serve_tune_entry_points_validate_before_touching_the_gpu():
    """Malformed calls of the batch, serving and autotune entry points return
    NQ_EINVAL (or their documented no-op result) before any HIP call."""
    lib = nq.lib()
    u32a = lambda *v: (ct.c_uint32 * len(v))(*v)
    handle = ct.c_void_p()
    totals = (ct.c_uint64 * 4)()
    # ragged batches
    assert lib.nq_count_batch(0, None, None, None, None) == 0       # nothing to count
    assert lib.nq_count_batch(3, None, None, None, totals) == -1
    assert lib.nq_count_batch(2, u32a(8, 29), None, None, totals) == -1
    assert lib.nq_count_batch(2, u32a(8, 9), u32a(3, 10), None, totals) == -1
    assert lib.nq_batch_create(0, u32a(8), None, None, ct.byref(handle)) == -1
    assert lib.nq_batch_create(1, u32a(0), None, None, ct.byref(handle)) == -1
    assert lib.nq_batch_create(1, u32a(8), None, None, None) == -1
    assert lib.nq_batch_run(None, totals, None) == -1
    assert lib.nq_batch_entries(None) == 0
    assert lib.nq_batch_destroy(None) == -1
    # serving: no server, no request, no output
    res = nq._native.NqResult()
    req = nq._native.NqRequest()
    tk = ct.c_uint64()
    assert lib.nq_serve_create(None, 0, None) == -1
    # unknown flag bits are refused before any device work, and the serving
    # flag by the counting entry points
    srv = ct.c_void_p()
    so = nq._native.NqOpts()
    so.flags = 16
    assert lib.nq_serve_create(ct.byref(so), 0, ct.byref(srv)) == -1
    assert lib.nq_count(12, ct.byref(so), ct.byref(tk)) == -1
    so.flags = nq._native.FLAG_SERVE_RESERVE
    assert lib.nq_count(12, ct.byref(so), ct.byref(tk)) == -1
    assert lib.nq_count_subproblems(12, None, None, None, None, 0, None, None,
                                    ct.byref(so)) == -1
    assert lib.nq_count_batch(1, (ct.c_uint32 * 1)(12), None, ct.byref(so),
                              (ct.c_uint64 * 1)()) == -1
    assert lib.nq_serve_submit(None, ct.byref(req), ct.byref(tk)) == -1
    assert lib.nq_serve_poll(None, 0, ct.byref(res)) == -1
    assert lib.nq_serve_wait(None, 0, ct.byref(res), 1000) == -1
    assert lib.nq_serve_destroy(None) == -1
    # autotune: board too small or too large, no output, empty depth range
    tuned = nq._native.NqTuned()
    assert lib.nq_autotune(3, 0, 0, 0.0, ct.byref(tuned)) == -1
    assert lib.nq_autotune(29, 0, 0, 0.0, ct.byref(tuned)) == -1
    assert lib.nq_autotune(20, 0, 0, 0.0, None) == -1
    assert lib.nq_autotune(20, 9, 6, 0.0, ct.byref(tuned)) == -1
    assert lib.nq_autotune(20, 6, 21, 0.0, ct.byref(tuned)) == -1
    # chunked boards (21..23): chunk depths start at the host depth 5
    assert lib.nq_autotune(21, 3, 4, 0.0, ct.byref(tuned)) == -1
    assert lib.nq_autotune(22, 11, 10, 0.0, ct.byref(tuned)) == -1
    assert lib.nq_autotune(23, 9, 24, 0.0, ct.byref(tuned)) == -1


def test_frontier_runs_cover_row0_columns():
    for n, k in [(20, 6), (17, 5), (9, 3)]:
        runs = nq.frontier_runs(n, k)
        pre, _ = oracle.frontier(n, k)
        starts = [i for i in range(len(pre)) if i == 0 or pre[i][0] != pre[i - 1][0]]
        assert runs == starts + [len(pre)]


def test_loop_form_setter_validates_and_restores():
    """nq_set_loop_form touches no device: unknown forms are refused, and -1
    restores the default."""
    import paper_2511_12009_amd as nq
    prev = nq.set_loop_form(-1)
    default = nq.set_loop_form(-1)
    try:
        assert default in (1, 3, 7)
        for bad in (-2, 8, 100):
            with pytest.raises(nq.NQError):
                nq.set_loop_form(bad)
        assert nq.set_loop_form(4) == default
        assert nq.set_loop_form(3) == 4
        assert nq.set_loop_form(5) == 3
        assert nq.set_loop_form(6) == 5
        assert nq.set_loop_form(7) == 6
        assert nq.set_loop_form(-1) == 7
        assert nq.set_loop_form(-1) == default
    finally:
        nq.set_loop_form(prev)


def test_perm_step_setter_validates_and_restores():
    """nq_perm_set_step touches no device: unknown steps are refused, and -1
    restores the default (step 2 unless NQ_PERM_STEP selects 0 or 1)."""
    import paper_2511_12009_amd as nq
    prev = nq.perm_set_step(-1)
    default = nq.perm_set_step(-1)
    try:
        assert default in (0, 1, 2)
        for bad in (-2, 3, 100):
            with pytest.raises(nq.NQError):
                nq.perm_set_step(bad)
        assert nq.perm_set_step(0) == default
        assert nq.perm_set_step(1) == 0
        assert nq.perm_set_step(2) == 1
        assert nq.perm_set_step(-1) == 2
        assert nq.perm_set_step(-1) == default
    finally:
        nq.perm_set_step(prev)


def _progress_record(n, depth, host_depth, chunks, done, total):
    """The text of one nq_count_resumable progress record (its file format)."""
    body = (f"nq-progress 1 n={n} depth={depth} host_depth={host_depth} chunks={chunks} "
            f"done={done} total={total}")
    h = 0xcbf29ce484222325
    for ch in body.encode():
        h = ((h ^ ch) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return f"{body} check={h:016x}\n"


def test_resumable_count_file_handling_without_a_gpu(tmp_path):
    """nq_count_resumable reads and checks its progress file before any device
    work: bad arguments, a damaged file and the file of another count are
    refused (the file is left as it was); a finished record is answered from
    the file alone."""
    path = str(tmp_path / "progress")
    with pytest.raises(nq.NQError):
        nq.count_resumable(0, path, depth=3)
    with pytest.raises(nq.NQError):
        nq.count_resumable(29, path, depth=3)
    with pytest.raises(nq.NQError):
        nq.count_resumable(12, "", depth=3)
    for bad in ("garbage\n", "",
                _progress_record(12, 4, 4, 8, 3, 100).replace("done=3", "done=4"),
                _progress_record(12, 4, 4, 8, 9, 100)):
        with open(path, "w") as f:
            f.write(bad)
        with pytest.raises(nq.NQError):
            nq.count_resumable(12, path, chunks=8, depth=4)
        with open(path) as f:
            assert f.read() == bad
    other = _progress_record(13, 4, 4, 8, 3, 100)
    with open(path, "w") as f:
        f.write(other)
    with pytest.raises(nq.NQError):
        nq.count_resumable(12, path, chunks=8, depth=4)
    with pytest.raises(nq.NQError):
        nq.count_resumable(13, path, chunks=16, depth=4)
    with pytest.raises(nq.NQError):
        nq.count_resumable(13, path, chunks=8, depth=5)
    with open(path, "w") as f:
        f.write(_progress_record(12, 4, 4, 8, 8, 14200))
    assert nq.count_resumable(12, path, chunks=8, depth=4) == (14200, 8, True)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 11, 13, 16])
def test_kings_frontier_matches_oracle(n):
    """nq_kings_frontier (bitmask enumeration) against the kings oracle (board
    arrays): the same prefixes in the same order, masks by definition, weights."""
    for k in sorted({1, 2, 3, min(n, 5)} | ({n} if n <= 8 else set())):
        if k > n:
            continue
        c, l, r, w = nq.frontier(n, k, kings=True)
        pre, pw = oracle.kings_frontier(n, k)
        assert len(c) == len(pre), (n, k)
        if len(pre):
            oc, ol, orr = oracle.kings_prefixes_masks(n, pre)
            np.testing.assert_array_equal(c, oc)
            np.testing.assert_array_equal(l, ol)
            np.testing.assert_array_equal(r, orr)
            np.testing.assert_array_equal(w, pw)


def test_kings_flag_refused_where_unsupported(tmp_path):
    """Resumable counts refuse the kings search before touching any file or device."""
    with pytest.raises(nq.NQError):
        nq._native.lib()
        o = nq._native._opts(3, "persistent", 0, 0, 0, None, nq._native.FLAG_KINGS, 0)
        import ctypes as c_
        t, d = c_.c_uint64(), c_.c_uint32()
        rc = nq._native.lib().nq_count_resumable(12, c_.byref(o), str(tmp_path / "p").encode(), 4,
                                                  0, c_.byref(t), c_.byref(d))
        nq._native._check(rc, "nq_count_resumable")
    assert not (tmp_path / "p").exists()


def test_wide_resumable_totals_without_a_gpu(tmp_path):
    """nq_count_resumable_wide keeps 128-bit totals in its progress record: a
    finished record of any total up to 2^128 - 1 is answered exactly from the
    file alone (decimal text across the 2^64 carry), a total of 2^128 or more
    is refused; the 64-bit entry point answers NQ_ERANGE for a total of 2^64 or
    more and refuses boards beyond 28; the domain of the wide entry point is
    checked before any device work."""
    path = str(tmp_path / "wide")
    for total in (0, 14200, 2**64 - 1, 2**64, 2**64 + 12345, 2**127 + 3, 2**128 - 1):
        with open(path, "w") as f:
            f.write(_progress_record(30, 10, 5, 8, 8, total))
        assert nq.count_resumable(30, path, chunks=8, depth=10, wide=True) == (total, 8, True)
        # depth 0 continues the record's count
        assert nq.count_resumable(30, path, chunks=8, wide=True) == (total, 8, True)
    with pytest.raises(nq.NQError):
        nq.count_resumable(30, path, chunks=8, depth=10)          # 64-bit entry: n <= 28
    for bad in (str(2**128), "1" + "0" * 39, "-1", "12a"):
        text = _progress_record(30, 10, 5, 8, 8, 0).replace("total=0 ", f"total={bad} ")
        with open(path, "w") as f:
            f.write(text)
        with pytest.raises(nq.NQError):
            nq.count_resumable(30, path, chunks=8, depth=10, wide=True)
        with open(path) as f:
            assert f.read() == text
    big = 2**64 + 7
    with open(path, "w") as f:
        f.write(_progress_record(12, 4, 4, 8, 8, big))
    with pytest.raises(nq.NQError) as e:
        nq.count_resumable(12, path, chunks=8, depth=4)
    assert e.value.status == nq._native.NQ_ERANGE
    assert nq.count_resumable(12, path, chunks=8, depth=4, wide=True) == (big, 8, True)
    fresh = str(tmp_path / "none")
    for n, depth in ((32, 12), (0, 3), (30, 9), (31, 10), (29, 8)):
        with pytest.raises(nq.NQError):
            nq.count_resumable(n, fresh, chunks=8, depth=depth, wide=True)
    assert not os.path.exists(fresh)


def test_wide_boards_validate_before_touching_the_gpu():
    """Boards beyond 28: nq_count refuses them (its total is 64 bits) and so does
    nq_count_subproblems without a 128-bit total or with more than 20 rows
    below the prefixes; nq_expand accepts up to 31."""
    lib = nq.lib()
    out = ct.c_uint64()
    o = nq._native._opts(10, "persistent", 0, 0, 0, None, 0, 0)
    fake = ct.c_void_p(16)                    # never dereferenced: refused first
    assert lib.nq_count(29, ct.byref(o), ct.byref(out)) == -1
    assert lib.nq_count_subproblems(30, fake, fake, fake, None, 1, None, fake, ct.byref(o)) == -1
    o.flags = nq._native.FLAG_WIDE_TOTAL
    o.depth = 9
    assert lib.nq_count_subproblems(30, fake, fake, fake, None, 1, None, fake, ct.byref(o)) == -1
    assert lib.nq_count_subproblems(32, fake, fake, fake, None, 1, None, fake, ct.byref(o)) == -1
    o.depth = 10
    assert lib.nq_count_subproblems(30, fake, fake, fake, None, 0, None, fake, ct.byref(o)) == 0
    assert lib.nq_count(12, ct.byref(o), ct.byref(out)) == -1    # no device total to widen
    o.flags = nq._native.FLAG_KINGS                            # kings(22) > 2^64
    assert lib.nq_count(22, ct.byref(o), ct.byref(out)) == -1
    assert lib.nq_expand(32, 1, None, None, None, None, 0, None, None, None, None, 0,
                         ct.byref(out), None) == -1


def test_ubench_arguments_are_checked_before_any_device_work():
    """The microbenchmark entry points refuse arguments outside their stated
    ranges before touching a device."""
    L = nq.lib()
    d1, d2 = ct.c_double(), ct.c_double()
    for op, chains, wps, iters in ((12, 8, 1, 8), (0, 2, 1, 8), (0, 8, 0, 8), (0, 8, 9, 8),
                                   (0, 8, 1, 0), (0, 8, 1, 12)):
        assert L.nq_ubench_valu(op, chains, wps, iters, ct.byref(d1), ct.byref(d2)) == -1
    assert L.nq_ubench_valu(0, 8, 1, 8, None, ct.byref(d2)) == -1
    for layout, op, active, wpc, frames in ((2, 0, 64, 4, 10), (0, 13, 64, 4, 10),
                                            (0, 0, 0, 4, 10), (0, 0, 65, 4, 10),
                                            (0, 0, 64, 0, 10), (0, 0, 64, 33, 10),
                                            (0, 0, 64, 4, 1), (0, 0, 64, 4, 33)):
        assert L.nq_ubench_lds(layout, op, active, wpc, frames, 16, ct.byref(d1)) == -1


@pytest.mark.skipif(__import__("shutil").which("gcc") is None, reason="needs gcc")
def test_binding_structures_have_the_header_layout(tmp_path):
    """Every structure the binding passes by pointer has the size and field
    offsets that a C compiler gives the header's declaration."""
    import subprocess
    from paper_2511_12009_amd import _native as nat
    pairs = [("nq_opts", nat.NqOpts), ("nq_tuned", nat.NqTuned),
             ("nq_tune_trial", nat.NqTuneTrial), ("nq_request", nat.NqRequest),
             ("nq_result", nat.NqResult)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "nq.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        cname, field, v = line.split()
        got[(cname, field)] = int(v)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ct.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


@pytest.mark.parametrize("n,dens,seed", [(1, 1.0, 0), (2, 0.7, 1), (7, 0.6, 2), (10, 0.5, 3),
                                         (12, 0.8, 4)])
def test_perm_frontier_matches_oracle(n, dens, seed):
    """The permanent search's frontier: the used-column set of every prefix the
    oracle enumerates, in the same (lexicographic) order, at every depth."""
    import seeded_inputs
    a = np.array(seeded_inputs.matrix01(n, dens, seeded_inputs.MATRIX_SEED + seed), np.uint8)
    for k in range(0, min(n, 6) + 1):
        got = nq.perm_frontier(a, k)
        ref = oracle.perm_prefixes_cols(n, oracle.perm_frontier(a, k))
        np.testing.assert_array_equal(got, ref)


def test_perm_entry_points_validate_before_touching_the_gpu():
    lib = nq.lib()
    rows = (ct.c_uint32 * 32)(*([0b111] * 3 + [0] * 29))
    out = ct.c_uint64()
    cols = (ct.c_uint32 * 8)()
    assert lib.nq_perm_frontier(3, rows, 2, cols, 8, ct.byref(out)) == 0 and out.value == 6
    assert lib.nq_perm_frontier(3, rows, 2, cols, 4, ct.byref(out)) == -2   # NQ_ERANGE
    assert lib.nq_perm_frontier(3, rows, 2, None, 0, ct.byref(out)) == 0 and out.value == 6
    assert lib.nq_perm_frontier(0, rows, 0, None, 0, ct.byref(out)) == -1
    assert lib.nq_perm_frontier(21, rows, 0, None, 0, ct.byref(out)) == -1
    assert lib.nq_perm_frontier(3, rows, 4, None, 0, ct.byref(out)) == -1
    assert lib.nq_perm_frontier(3, None, 1, None, 0, ct.byref(out)) == -1
    assert lib.nq_perm_frontier(3, rows, 1, None, 0, None) == -1
    wide = (ct.c_uint32 * 3)(0b111, 0b1000, 0b111)                      # a column off the board
    assert lib.nq_perm_frontier(3, wide, 1, None, 0, ct.byref(out)) == -1
    total = ct.c_uint64()
    assert lib.nq_perm_count(0, rows, None, ct.byref(total)) == -1
    assert lib.nq_perm_count(3, wide, None, ct.byref(total)) == -1
    assert lib.nq_perm_count(3, rows, None, None) == -1
    o = nq._native.NqOpts()
    o.flags = 1
    assert lib.nq_perm_count(3, rows, ct.byref(o), ct.byref(total)) == -1
    assert lib.nq_perm_count_subproblems(3, rows, None, 5, 1, None, None, None) == -1
    assert lib.nq_perm_count_subproblems(3, rows, None, 0, 4, None, None, None) == -1
    assert lib.nq_perm_count_subproblems(21, rows, None, 0, 1, None, None, None) == -1
    with pytest.raises(ValueError):
        nq.perm_rows(np.ones((3, 4)))
    assert nq.perm_rows([[1, 0, 1], [0, 1, 0], [1, 1, 1]]).tolist() == [0b101, 0b010, 0b111]
