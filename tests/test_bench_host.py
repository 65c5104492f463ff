"""Host-side logic of bench.py: the one-GPU guard, the golden lookups behind
its nodes/s, and the reading of the committed counter records (HBM traffic and
executed VALU rate are reported only while the record matches the kernel's
current sources).  Nothing here touches a GPU."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_golden_nodes_lookup():
    # nodes(20, 6) is an oracle run; nodes(20, 9) is derived from it by taking
    # away the weighted placements of rows 6..8, which become prefix rows.
    assert bench.golden_nodes(20, 6) == 1865470950135
    assert bench.golden_nodes(20, 9) == 1864488301015
    # deeper pre-placement leaves fewer nodes below the frontier
    seq = [bench.golden_nodes(20, k) for k in range(4, 11)]
    assert all(a > b for a, b in zip(seq, seq[1:]))
    assert bench.golden_nodes(99, 3) is None


def test_known_counts_lookup(known_counts):
    kc = bench.known_counts()
    assert kc == known_counts
    assert kc[20] == bench.EXPECT


def _record():
    path = os.path.join(ROOT, "profiles", "nq_dfs_n20_k9.md")
    with open(path) as f:
        lines = [l for l in f if l.startswith("counters:")]
    assert len(lines) == 1
    return dict(x.split("=", 1) for x in lines[0].split()[1:])


def test_counter_record_is_read_when_the_digest_matches(monkeypatch):
    rec = _record()
    for v in ("NQ_DFS_LOOP", "NQ_IDLE_MIN", "NQ_CLAIM"):
        monkeypatch.delenv(v, raising=False)
    monkeypatch.setattr(bench, "kernel_digest", lambda: rec["kernel_sha256"])
    kv = bench.profiled_counters(20, 9)
    assert kv is not None and kv["source"] == os.path.join("profiles", "nq_dfs_n20_k9.md")
    assert bench.profiled_traffic(20, 9) == int(rec["fetch_bytes"]) + int(rec["write_bytes"])
    ex = bench.profiled_executed(20, 9)
    rate = int(rec["valu_lane_ops"]) / (int(rec["kernel_ns"]) / 1e9)
    assert ex["lane_ops_per_s"] == pytest.approx(rate)
    assert 0.0 < ex["frac"] <= 1.0
    clk = bench.profiled_clock(20, 9)
    assert clk == pytest.approx(int(rec["grbm_gui_active"]) / 8 / (int(rec["kernel_ns"]) / 1e9))
    assert 1.0e9 < clk < 2.5e9
    lds = bench.profiled_lds(20, 9, 1000.0)
    assert lds["instr_per_launch"] == int(rec["lds_instructions"])
    assert lds["per_cu_per_s"] == pytest.approx(int(rec["lds_instructions"]) / 256 / 1.0)
    assert lds["frac"] == pytest.approx(lds["per_cu_per_s"] / float(rec["lds_ceiling_per_cu"]))
    # another workload has no record
    assert bench.profiled_counters(20, 8) is None
    assert bench.profiled_counters(21, 9) is None


def test_counter_record_is_ignored_for_other_sources_or_overrides(monkeypatch):
    rec = _record()
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 64)
    assert bench.profiled_counters(20, 9) is None
    assert bench.profiled_traffic(20, 9) is None
    assert bench.profiled_executed(20, 9) is None
    assert bench.profiled_clock(20, 9) is None and bench.profiled_lds(20, 9, 1000.0) is None
    monkeypatch.setattr(bench, "kernel_digest", lambda: rec["kernel_sha256"])
    monkeypatch.setenv("NQ_DFS_LOOP", "2")
    assert bench.profiled_counters(20, 9) is None


def test_kernel_digest_covers_the_kernel_sources():
    d = bench.kernel_digest()
    assert len(d) == 64 and int(d, 16) >= 0
    for rel in bench.KERNEL_FILES:
        assert os.path.exists(os.path.join(ROOT, rel))


def test_stored_permanent_lookup():
    stored = bench.perm_stored()
    assert stored[(20, 0.5, 0)] == 1910787252054
    assert all(v > 0 for v in stored.values())
