"""Host code under the sanitizers (no GPU): the frontier enumeration of the
library (nq_frontier.cpp, threaded for large frontiers) and the oracle
(threaded prefix counts) are rebuilt with AddressSanitizer + UndefinedBehavior-
Sanitizer and with ThreadSanitizer, run through small drivers, and must report
nothing and print the same results as the normal builds."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_2511_12009_amd as nq
from conftest import ROOT

HERE = os.path.join(ROOT, "tests", "sanitize")
SANITIZERS = [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
              ["-fsanitize=thread"]]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc")


def _run(cmd, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "WARNING: ThreadSanitizer" not in p.stderr, \
        p.stderr[-4000:]
    return p.stdout


def _digest(c, l, r, w):
    """sum over i of (i + 1) * (c + 3 l + 5 r + 7 w), modulo 2^64 (as the driver)."""
    i = np.arange(1, len(c) + 1, dtype=np.uint64)
    v = (c.astype(np.uint64) + np.uint64(3) * l.astype(np.uint64) +
         np.uint64(5) * r.astype(np.uint64) + np.uint64(7) * w.astype(np.uint64))
    with np.errstate(over="ignore"):
        return int(np.sum(i * v, dtype=np.uint64))


@pytest.mark.parametrize("flags", SANITIZERS, ids=["asan-ubsan", "tsan"])
def test_frontier_enumeration_under_sanitizers(tmp_path, flags):
    exe = str(tmp_path / "frontier_driver")
    _run(["g++", "-std=c++17", "-O1", "-g", "-pthread", *flags,
          "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "paper_2511_12009_amd", "csrc", "nq_frontier.cpp"),
          os.path.join(HERE, "frontier_driver.cpp"), "-o", exe])
    out = _run([exe], {"ASAN_OPTIONS": "detect_leaks=1", "TSAN_OPTIONS": "halt_on_error=1"})
    lines = out.strip().splitlines()
    assert len(lines) == 13
    for line in lines[:-1]:
        tag, n, depth, F, cap, digest = line.split()
        n, depth, F, cap = int(n), int(depth), int(F), int(cap)
        c, l, r, w = nq.frontier(n, depth, kings=(tag == "kings"))
        assert len(c) == F and cap <= F
        assert int(digest, 16) == _digest(c[:cap], l[:cap], r[:cap], w[:cap]), line
    assert lines[-1].split()[:3] == ["runs", "20", "6"]
    assert int(lines[-1].split()[4]) == nq.frontier_size(20, 6)


@pytest.mark.parametrize("flags", SANITIZERS, ids=["asan-ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, flags):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", "-O1", "-g", "-pthread", *flags,
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-o", exe])
    out = _run([exe], {"ASAN_OPTIONS": "detect_leaks=1", "TSAN_OPTIONS": "halt_on_error=1"})
    rows = [l.split() for l in out.strip().splitlines()]
    for tag, *vals in rows:
        v = [int(x) for x in vals]
        if tag == "queens":
            assert tuple(v[1:]) == oracle.queens(v[0])
        elif tag == "brute":
            assert v[1] == oracle.brute_count(v[0])
        elif tag == "frontier":
            pre, w = oracle.frontier(v[0], v[1])
            c, nd = oracle.count_prefixes(v[0], pre, threads=8)
            assert v[2:] == [int((c * w.astype(np.uint64)).sum()), int(nd.sum())]
        elif tag == "kings":
            pre, w = oracle.kings_frontier(v[0], v[1])
            c, nd = oracle.kings_count_prefixes(v[0], pre, threads=8)
            assert v[2:] == [int((c * w.astype(np.uint64)).sum()), int(nd.sum())]
    assert [r[0] for r in rows].count("queens") == 11
