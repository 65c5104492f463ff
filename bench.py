"""Benchmark: DFS nodes/s of the N=20 count on one MI355X, batched vs plain.

One step = the whole device path over the resident N=20 frontier (pre-placement
depth k, built before the timed region): zero the total, one persistent DFS
launch over every subproblem (weighted total; per-subproblem counts are not
requested), and the copy of the 8-byte total into that step's own slot of a
pinned host array; after the timed loop every slot is checked against
Q(20) = 39,029,188,884.

value = DFS nodes per second = nodes(20, k) / step time, where nodes(20, k) is
the oracle's node count (queens placed in rows k..18 below every pre-placed
prefix), read from tests/golden/oracle_runs.txt.

The pre-placement depth and launch shape come from nq_autotune over depths
5..10 (the workload's stated depths 5..8 and the two beyond them, which win on
this GPU) unless --depth is given; every trial is reported, with the best
within 5..8 beside the overall best.  Frontiers deeper than 8 rows are built on the host at
depth k-2 and expanded on the device (nq_expand) before the timed region.  Printed: one JSON line with the metric, the "plain"
form (one launch per row-0 column over the same frontier), the end-to-end
nq_count wall time, the int-ALU roofline of the DFS kernel, the ragged
256-instance batch (one graph replay), the kings search (a second DFS on the
same engine, n = 16), the permanent of a seeded 20 x 20 0/1 matrix (a third
DFS, with two-word frames), one GPU's share of an N=21 count
dealt round-robin over 8 GPUs (all 8 shares run in turn; their totals must add
up to Q(21)), the serving loop at a few request rates (p50/p99 latency,
throughput; then the latency-first server, NQ_FLAG_SERVE_RESERVE, at one
rate) and the oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, EXPECT = 20, 39029188884
# Algorithmic int32 operations of one DFS node (one queen placement):
# lowest free column (negate, and) 2, remove it from the candidates 1, update
# cols 1, ld (or, shift) 2, rd (or, shift) 2, free squares of the next row
# (or, or, not, and) 4, last-row test (popcount, compare) 2.
OPS_PER_NODE = 14
# MI355X int32 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s.
INT_PEAK = 256 * 4 * 16 * 2.4e9


def golden_nodes(n, k):
    """nodes(n, k) stored by tests/golden/make_golden.py (oracle runs, and for even n
    the other depths derived from them with the node identity), or None."""
    for name in ("oracle_runs.txt", "oracle_nodes.txt"):
        path = os.path.join(ROOT, "tests", "golden", name)
        if not os.path.exists(path):
            continue
        with open(path) as f:
            for line in f:
                if line.startswith("#") or not line.strip():
                    continue
                r = line.split()
                if int(r[0]) == n and int(r[1]) == k:
                    return int(r[4] if name == "oracle_runs.txt" else r[2])
    return None


KERNEL_FILES = ("paper_2511_12009_amd/csrc/nq_dfs.hip", "paper_2511_12009_amd/csrc/nq_kernel.h",
                "paper_2511_12009_amd/csrc/nq_wave.h", "paper_2511_12009_amd/build.py")


def kernel_digest():
    """sha256 over the DFS kernel's source, its parameter header and the build
    script (compiler flags), in that order."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_FILES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_counters(n, k):
    """The counter record of the default persistent DFS kernel at (n, k) from the
    committed summary (profiles/), as a dict, or None when there is none, when
    the kernel's source, header or build flags have changed since the counters
    were taken (the summary records their kernel_digest), or when an environment
    override selects another kernel form or scheduler setting."""
    if any(os.environ.get(v) for v in ("NQ_DFS_LOOP", "NQ_IDLE_MIN", "NQ_CLAIM")):
        return None
    import glob
    digest = kernel_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("counters:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:] if "=" in x)
                if (kv.get("kernel_sha256") == digest and int(kv.get("n", -1)) == n and
                        int(kv.get("depth", -1)) == k):
                    kv["source"] = os.path.relpath(path, ROOT)
                    return kv
    return None


def profiled_traffic(n, k):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    committed counters, or None (see profiled_counters)."""
    kv = profiled_counters(n, k)
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"]) if kv else None


def profiled_executed(n, k):
    """VALU lane-operations the kernel executed per second under the counters
    (SQ_THREAD_CYCLES_VALU, the active lanes summed over its VALU instructions,
    over the duration of the same profiled dispatch), against the same int32
    peak, or None.  Beside `achieved` (the algorithmic operations) it shows how
    much of the issued work is overhead."""
    kv = profiled_counters(n, k)
    if not kv or "valu_lane_ops" not in kv:
        return None
    rate = int(kv["valu_lane_ops"]) / (int(kv["kernel_ns"]) / 1e9)
    return {"lane_ops_per_s": rate, "frac": rate / INT_PEAK, "source": kv["source"]}


def profiled_clock(n, k):
    """The shader clock during the profiled DFS dispatch (GRBM_GUI_ACTIVE of the
    8 XCDs over the dispatch's duration), in Hz, or None."""
    kv = profiled_counters(n, k)
    if not kv or "grbm_gui_active" not in kv:
        return None
    return int(kv["grbm_gui_active"]) / 8 / (int(kv["kernel_ns"]) / 1e9)


def profiled_lds(n, k, kernel_ms):
    """The DFS kernel's LDS instruction rate per CU (SQ_INSTS_LDS of the
    committed counter run, per launch, over this run's kernel time) against
    the ceiling the LDS microbenchmark measured for the same access pair (one
    ds_write_b128 and one ds_read_b128 per wave-step, interleaved layout, 16
    waves per CU), or None."""
    kv = profiled_counters(n, k)
    if not kv or "lds_instructions" not in kv or "lds_ceiling_per_cu" not in kv:
        return None
    rate = int(kv["lds_instructions"]) / 256 / (kernel_ms / 1e3)
    ceiling = float(kv["lds_ceiling_per_cu"])
    return {"instr_per_launch": int(kv["lds_instructions"]), "per_cu_per_s": rate,
            "ceiling_per_cu_per_s": ceiling, "frac": rate / ceiling, "source": kv["source"]}


def known_counts():
    """Expected Q(n): the oracle's weighted total where tests/golden/oracle_runs.txt
    holds an oracle run of n (written by tests/golden/make_golden.py), else the
    published count (tests/golden/known_counts.txt).  The two agree wherever
    both exist (tests/test_oracle.py)."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "known_counts.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                n, c = line.split()[:2]
                out[int(n)] = int(c)
    with open(os.path.join(ROOT, "tests", "golden", "oracle_runs.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r = line.split()
                out[int(r[0])] = int(r[3])
    return out


def oracle_checked():
    """Board sizes whose expected count comes from an oracle run (see known_counts)."""
    with open(os.path.join(ROOT, "tests", "golden", "oracle_runs.txt")) as f:
        return sorted({int(ln.split()[0]) for ln in f if ln.strip() and not ln.startswith("#")})


def bench_batch(nq, known):
    """Ragged batch: 256 board sizes N_i uniform in 8..19 (seeded), one graph replay."""
    import seeded_inputs
    ns = seeded_inputs.ragged_batch_ns()
    t = time.perf_counter()
    with nq.Batch(ns) as b:
        build_ms = (time.perf_counter() - t) * 1e3
        got, ms = b.run(timing=True)      # first replay (warm)
        got, ms = b.run(timing=True)
        entries = b.entries
    ok = got == [known[n] for n in ns]
    if not ok:
        raise SystemExit("bench.py: ragged batch totals differ from the expected counts")
    by_oracle = oracle_checked()
    return {"instances": len(ns), "subproblems": entries, "replay_ms": ms,
            "build_ms": build_ms, "exact": ok,
            "checked_by_oracle_runs": sum(1 for n in ns if n in by_oracle),
            "oracle_sizes": [n for n in sorted(set(ns)) if n in by_oracle],
            "form": "one persistent launch over every instance's frontier, HIP graph replay"}


def bench_shards(nq, torch, known, shares=8, n=21, k=6, deepen=3):
    """One GPU's share of a count sharded over `shares` GPUs: the N=21 depth-6
    frontier dealt round-robin, each share deepened on the device and searched
    by one persistent launch.  Per-share kernel times; the share totals must
    add up to Q(21)."""
    dev = torch.device("cuda:0")
    cols, ld, rd, w = nq.frontier(n, k)
    ms, entries, grand = [], [], 0
    for r in range(shares):
        t = [torch.from_numpy(np.ascontiguousarray(x[r::shares]).view(np.int32)).to(dev)
             for x in (cols, ld, rd)]
        tw = torch.from_numpy(np.ascontiguousarray(w[r::shares])).to(dev)
        c, l, rr, ww = nq.expand(n, deepen, t[0], t[1], t[2], tw)
        tot = torch.zeros(1, dtype=torch.int64, device=dev)
        _, _, m = nq.count_subproblems(n, c, l, rr, weight=ww, counts=False, total=tot,
                                       depth=k + deepen, timing=True)
        grand += int(tot.item())
        ms.append(m)
        entries.append(c.numel())
        del c, l, rr, ww, t, tw
        print(f"[bench] share {r}/{shares}: {entries[-1]} subproblems, {m:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    if grand != known[n]:
        raise SystemExit(f"bench.py: shares of N={n} add up to {grand}, not {known[n]}")
    return {"n": n, "frontier_depth": k, "shares": shares, "search_depth": k + deepen,
            "split": "round-robin over the frontier", "share_ms": ms, "share_subproblems": entries,
            "max_over_mean": max(ms) / (sum(ms) / len(ms)), "sum_exact": True}


def kings_count(n):
    """The king-placement count a(n) from a(0..3) = 1, 1, 0, 0 by its recurrence
    (pinned against the kings oracle in tests/test_oracle_kings.py)."""
    a = [1, 1, 0, 0]
    for m in range(4, n + 1):
        a.append((m + 1) * a[m - 1] - (m - 2) * a[m - 2] - (m - 5) * a[m - 3] + (m - 3) * a[m - 4])
    return a[n]


def bench_kings(nq, n=16):
    """The second search on the same engine: n non-attacking kings, one per row
    and column, automatic depth (host frontier), one persistent launch."""
    want = kings_count(n)

    def best_ms():
        best = None
        for _ in range(2):
            got, ms = nq.count(n, kings=True, timing=True)
            if got != want:
                raise SystemExit(f"bench.py: kings({n}) = {got}, not {want}")
            best = ms if best is None else min(best, ms)
        return best

    best = best_ms()                      # the default step (form 7, popcount leaf test)
    nq.set_loop_form(1)                   # the kings run form 1 while the queens do
    try:
        form1 = best_ms()
    finally:
        nq.set_loop_form(-1)
    return {"n": n, "solutions": want, "kernel_ms": best, "solutions_per_s": want / (best / 1e3),
            "form1_kernel_ms": form1, "exact": True,
            "form": "kings search on the queens lane-stack engine (NQ_FLAG_KINGS), step of form 7"}


def perm_stored():
    """Stored permanents of seeded 0/1 matrices (tests/golden/perm_totals.txt,
    the oracle's Ryser routine): {(n, density, seed): permanent}."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "perm_totals.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[(int(line[0]), float(line[1]), int(line[2]))] = int(line[3])
    return out


def bench_perm(nq, torch, n=20, density=0.5, depths=(10,), reps=2):
    """The third search on the same engine: the permanent of the seeded n x n
    0/1 matrix of the given density (two-word frames, two-row leaf rule), one
    persistent launch over the host frontier resident on the device, at the
    given depths (the line: 10, the best; --perm-only: 7..10; at depth 6 the
    330,541 subtrees of n = 20 leave most lanes idle behind the largest);
    kernel time from HIP events (best of `reps`), nodes (placements in rows
    k..n-3) from one node-counting launch per depth, the total checked
    against the stored permanent."""
    import seeded_inputs
    a = np.array(seeded_inputs.matrix01(n, density), np.uint8)
    want = perm_stored()[(n, density, 0)]
    rows = []
    for k in depths:
        print(f"[bench] permanent n={n} depth {k}", file=sys.stderr, flush=True)
        cols = nq.perm_frontier(a, k)
        d = torch.from_numpy(np.ascontiguousarray(cols).view(np.int32)).cuda()
        nodes = torch.empty(len(cols), dtype=torch.int64, device="cuda")
        _, tot = nq.perm_count_subproblems(a, d, k, counts=False, nodes=nodes)
        torch.cuda.synchronize()
        if int(tot.item()) != want:
            raise SystemExit(f"bench.py: permanent {int(tot.item())} != {want} (node run, k={k})")
        below = int(nodes.sum().item())
        best = None
        for _ in range(reps):
            _, tot, ms = nq.perm_count_subproblems(a, d, k, counts=False, timing=True)
            if int(tot.item()) != want:
                raise SystemExit(f"bench.py: permanent {int(tot.item())} != {want} (k={k})")
            best = ms if best is None else min(best, ms)
        rows.append({"depth": k, "subproblems": len(cols), "kernel_ms": best, "nodes": below,
                     "nodes_per_s": below / (best / 1e3)})
        del d, nodes
        torch.cuda.empty_cache()
    top = min(rows, key=lambda r: r["kernel_ms"])
    return {"n": n, "density": density, "permanent": want, "exact": True,
            "best_depth": top["depth"], "kernel_ms": top["kernel_ms"],
            "nodes_per_s": top["nodes_per_s"], "depths": rows,
            "form": "permanent search on the lane-stack engine (8-byte frames, two-row leaf)"}


def _serve_count_work(nq, torch, n, entries):
    """DFS nodes of a COUNT request of board n that the server searched as
    `entries` subproblems: the frontier depth with that many entries, searched
    by nq_count_subproblems with per-entry node counts (the node-counting
    kernel is checked against the oracle's nodes in the parity tests)."""
    dev = torch.device("cuda:0")
    for d in range(1, n + 1):
        if nq.frontier_size(n, d) == entries:
            cols, ld, rd, w = nq.frontier(n, d)
            t = [torch.from_numpy(x.view(np.int32)).to(dev) for x in (cols, ld, rd)]
            nodes = torch.zeros(len(cols), dtype=torch.int64, device=dev)
            nq.count_subproblems(n, *t, weight=torch.from_numpy(w).to(dev), counts=False,
                                 depth=d, nodes=nodes)
            return int(nodes.sum())
    raise SystemExit(f"bench.py: no frontier depth of N={n} has {entries} entries")


def _slice_check(nq, torch, n, k, cols, ld, rd, w, start, length, entries):
    """A second path for one slice: its entries expanded by as many rows as the
    server expanded them (the rows whose child count is the `entries` the
    server searched), searched by nq_count_subproblems with node counts;
    returns (weighted total, entries searched, DFS nodes)."""
    dev = torch.device("cuda:0")
    sl = slice(start, start + length)
    t = [torch.from_numpy(np.ascontiguousarray(x[sl]).view(np.int32)).to(dev)
         for x in (cols, ld, rd)]
    tw = torch.from_numpy(np.ascontiguousarray(w[sl])).to(dev)
    for rows in (3, 2, 1):
        c, l, r, ww = nq.expand(n, rows, t[0], t[1], t[2], tw)
        if c.numel() == entries:
            break
    else:
        c, l, r, ww, rows = t[0], t[1], t[2], tw, 0
    nodes = torch.zeros(c.numel(), dtype=torch.int64, device=dev)
    _, tot = nq.count_subproblems(n, c, l, r, weight=ww, counts=False, depth=k + rows,
                                  nodes=nodes)
    return int(tot.item()), c.numel(), int(nodes.sum())


def bench_serving(nq, torch, known, rates, seconds, waves_per_cu=0, reserve=False):
    """Poisson COUNT(N in 10..18) requests with N=21 depth-6 4096-entry slices
    interleaved; per rate: p50/p99 latency (all COUNTs, per N, slices),
    throughput in requests/s and in served DFS nodes/s.  Every COUNT result is
    checked against the published count; every slice against a second device
    path over the same entries (nq_expand + nq_count_subproblems), whose node
    counts also give the served nodes.  Solo latency per N (one request on an
    idle server) is measured first."""
    import seeded_inputs
    n21, k21, slen = 21, 6, 4096
    F21 = nq.frontier_size(n21, k21)
    c21, l21, r21, w21 = nq.frontier(n21, k21)
    res = {"solo_count_ms": {}, "rates": []}
    count_nodes, slice_ref = {}, {}
    if waves_per_cu:
        res["waves_per_cu"] = waves_per_cu                 # cap on each epoch's resident waves
    if reserve:
        res["reserve"] = True                              # NQ_FLAG_SERVE_RESERVE
    with nq.Server(hbm_budget=64 << 30, waves_per_cu=waves_per_cu, reserve=reserve) as srv:
        srv.wait(srv.submit_slice(n21, k21, 0, 1))          # builds the resident frontier
        for n in range(10, 19):
            srv.wait(srv.submit_count(n))                     # builds this N's frontier
            r = srv.wait(srv.submit_count(n))
            if r["status"] != 0 or r["count"] != known[n]:
                raise SystemExit(f"bench.py: serving result wrong (solo N={n})")
            res["solo_count_ms"][n] = (r["t_done_ns"] - r["t_submit_ns"]) / 1e6
            count_nodes[n] = (r["entries"], _serve_count_work(nq, torch, n, r["entries"]))
        for rate in rates:
            n_req = max(1, int(rate * seconds))
            arr = seeded_inputs.poisson_arrivals(n_req, rate)
            ns = seeded_inputs.serve_count_ns(n_req)
            s_rate = max(1.0, rate / 8)
            s_arr = seeded_inputs.poisson_arrivals(max(1, int(s_rate * seconds)), s_rate,
                                                   seed=seeded_inputs.SERVE_SEED + 1)
            events = sorted([(t, "count", i) for i, t in enumerate(arr)] +
                            [(t, "slice", i) for i, t in enumerate(s_arr)])
            tickets = []
            t0 = time.perf_counter()
            for t, kind, i in events:
                dt = t - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                if kind == "count":
                    tickets.append(("count", ns[i], srv.submit_count(ns[i])))
                else:
                    start = (i * slen) % F21
                    ln = min(slen, F21 - start)
                    tickets.append(("slice", (start, ln), srv.submit_slice(n21, k21, start, ln)))
            lat = {"count": [], "slice": []}
            per_n = {}
            served_nodes = 0
            results = []
            for kind, arg, tk in tickets:
                r = srv.wait(tk, timeout_s=300)
                results.append((kind, arg, r))
            wall = time.perf_counter() - t0
            for kind, arg, r in results:
                if r["status"] != 0:
                    raise SystemExit(f"bench.py: serving request failed ({kind}, {arg})")
                ms = (r["t_done_ns"] - r["t_submit_ns"]) / 1e6
                lat[kind].append(ms)
                if kind == "count":
                    if r["count"] != known[arg] or r["entries"] != count_nodes[arg][0]:
                        raise SystemExit(f"bench.py: serving result wrong (count, N={arg})")
                    per_n.setdefault(arg, []).append(ms)
                    served_nodes += count_nodes[arg][1]
                else:
                    if arg not in slice_ref:
                        slice_ref[arg] = _slice_check(nq, torch, n21, k21, c21, l21, r21, w21,
                                                      *arg, r["entries"])
                    want, entries, nd = slice_ref[arg]
                    if r["count"] != want or r["entries"] != entries:
                        raise SystemExit(f"bench.py: serving slice {arg} = {r['count']}, "
                                         f"second path {want}")
                    served_nodes += nd
            row = {"rate_count_per_s": rate, "rate_slice_per_s": s_rate,
                   "requests": len(tickets), "wall_s": wall,
                   "throughput_req_per_s": len(tickets) / wall,
                   "served_nodes": served_nodes, "nodes_per_s": served_nodes / wall}
            for kind in ("count", "slice"):
                if lat[kind]:
                    row[f"{kind}_p50_ms"] = float(np.percentile(lat[kind], 50))
                    row[f"{kind}_p99_ms"] = float(np.percentile(lat[kind], 99))
            row["count_by_n"] = {
                n: {"requests": len(v), "p50_ms": float(np.percentile(v, 50)),
                    "p99_ms": float(np.percentile(v, 99)),
                    "p50_over_solo": float(np.percentile(v, 50)) / res["solo_count_ms"][n]}
                for n, v in sorted(per_n.items())}
            res["rates"].append(row)
            print(f"[bench] serving {json.dumps(row)}", file=sys.stderr, flush=True)
    res["checked"] = ("every COUNT against the published count; every slice against nq_expand + "
                      "nq_count_subproblems over the same entries")
    return res


def device_frontier(nq, torch, dev, k, n=N):
    """The depth-k frontier of an n board (default N=20) as device tensors
    (cols, ld, rd int32, weight uint8): built on the host, and for k > 8 at
    depth k-2 and expanded by two rows on the device."""
    hk = k if k <= 8 else k - 2
    cols, ld, rd, w = nq.frontier(n, hk)
    t = [torch.from_numpy(x.view(np.int32)).to(dev) for x in (cols, ld, rd)]
    tw = torch.from_numpy(w).to(dev)
    if hk == k:
        return t[0], t[1], t[2], tw
    out = nq.expand(n, k - hk, t[0], t[1], t[2], tw)
    torch.cuda.synchronize()
    return out


def profile_run(nq, torch, k, args):
    """A short program for rocprofv3 counter passes: a plain copy of known size,
    then one DFS launch of the benchmark workload."""
    dev = torch.device("cuda:0")
    src = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)                                   # 256 MiB read + 256 MiB written
    torch.cuda.synchronize()
    del src, dst
    c, l, r, tw = device_frontier(nq, torch, dev, k)
    t = [c, l, r]
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    _, _, ms = nq.count_subproblems(N, *t, weight=tw, counts=False, total=total, depth=k,
                                    timing=True, waves_per_cu=args.waves_per_cu,
                                    refill_every=args.refill, claim=args.claim)
    if int(total.item()) != EXPECT:
        raise SystemExit(f"bench.py: profile total {int(total.item())} != {EXPECT}")
    print(f"[bench] profile: copy 256 MiB, DFS N={N} k={k} F={c.numel()} kernel {ms:.1f} ms",
          file=sys.stderr, flush=True)


UB_OPS = {0: "v_add3_u32", 1: "v_bitop3_b32", 2: "v_cndmask_b32 (SGPR mask)",
          3: "v_addc_co_u32 (SGPR carry-in)", 4: "v_add_lshl_u32", 5: "v_xad_u32",
          6: "v_and_b32", 7: "v_xor_b32", 8: "v_or3_b32", 9: "v_sub_u32", 10: "v_lshrrev_b32",
          11: "v_add_u32"}
UB_LDS_OPS = {0: ("write b128 + read b128", 2), 1: ("read b128", 1), 2: ("write b128", 1),
              3: ("exchange 16 B (wrxchg2_rtn_b64)", 1), 4: ("write b64 + read b64", 2),
              5: ("write b32 + read b32", 2), 6: ("write b64", 1), 7: ("write b32", 1),
              8: ("write b96", 1), 9: ("write 16 B as write2_b64", 1), 10: ("read b96", 1),
              11: ("read 16 B as read2_b64", 1), 12: ("write b96 + read b96", 2)}


def run_ubench(nq, args, occupancy_only=False):
    """The microbenchmarks behind the roofline (include/nq_ubench.h): the int32
    VALU rate of the DFS step's operations with eight independent chains per
    lane at 1..8 waves per SIMD (and one chain, one wave: the dependent
    latency), the shader clock during those runs (s_memtime cycles over event
    time), and the LDS stack accesses in the interleaved and contiguous
    layouts at several occupancies and active-lane counts."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"valu": [], "lds": [], "cus": cus}

    def valu(op, chains, wps, iters):
        ms, cyc = nq.ubench_valu(op, chains, wps, iters)
        lane_ops = cus * 4 * wps * 64 * chains * iters
        row = {"op": UB_OPS[op], "chains": chains, "waves_per_simd": wps, "iters": iters,
               "kernel_ms": ms, "lane_ops_per_s": lane_ops / (ms / 1e3),
               "frac_of_peak": lane_ops / (ms / 1e3) / INT_PEAK,
               "clock_ghz": cyc / (ms * 1e6),
               "cycles_per_instr_per_wave": cyc / (chains * iters)}
        out["valu"].append(row)
        print(f"[bench] ubench valu {json.dumps(row)}", file=sys.stderr, flush=True)
        return row

    for op in (() if occupancy_only else range(len(UB_OPS))):
        valu(op, 8, 1, 1 << 16)                              # warm the code object
        for wps in (1, 2, 4, 8):
            valu(op, 8, wps, 1 << 19)
        valu(op, 1, 1, 1 << 19)

    def lds(layout, op, wpc, active, frames=10):
        iters = 1 << 16
        nq.ubench_lds(layout, active, wpc, frames, 1 << 10, op=op)  # warm the code object
        ms = nq.ubench_lds(layout, active, wpc, frames, iters, op=op)
        name, per_iter = UB_LDS_OPS[op]
        instr = cus * wpc * iters * per_iter
        row = {"layout": "interleaved" if layout == 0 else "contiguous", "op": name,
               "waves_per_cu": wpc, "active_lanes": active, "frames": frames, "iters": iters,
               "kernel_ms": ms, "lds_instr_per_cu_per_s": instr / cus / (ms / 1e3),
               "cycles_per_instr_per_cu_at_2_4GHz": 2.4e9 / (instr / cus / (ms / 1e3))}
        out["lds"].append(row)
        print(f"[bench] ubench lds {json.dumps(row)}", file=sys.stderr, flush=True)

    # the write + read pairs beyond 16 waves per CU: 5 frames (5 KB) per wave;
    # 16-byte frames (the stack's), 12- and 8-byte frames for comparison
    for op in (0, 12, 4):
        for wpc in (8, 12, 16, 20, 24, 28, 32):
            lds(0, op, wpc, 64, frames=5)
    if occupancy_only:
        return out
    for layout in (0, 1):
        for wpc in (4, 8, 16):
            for active in (64, 32, 16):
                lds(layout, 0, wpc, active)
    for op in range(1, len(UB_LDS_OPS)):
        for wpc in (8, 16):
            for active in (64, 16):
                lds(0, op, wpc, active)
    clocks = [r["clock_ghz"] for r in out["valu"] if r["waves_per_simd"] == 8]
    out["clock_ghz_under_load"] = float(np.median(clocks)) if clocks else None
    best = max(r["lane_ops_per_s"] for r in out["valu"])
    out["best_lane_ops_per_s"] = best
    out["peak_at_measured_clock"] = (cus * 4 * 16 * out["clock_ghz_under_load"] * 1e9
                                     if out["clock_ghz_under_load"] else None)
    return out


ABLATION_PLAN = {
    # n: (pre-placement depths, depth of the plain block-size sweep, repetitions)
    17: (range(3, 10), 5, 2),
    18: (range(3, 10), 5, 2),
    19: (range(4, 10), 5, 2),
    20: (range(5, 11), 6, 2),
    21: (range(7, 11), None, 1),
}
FORM_NAMES = {0: "registers, compiler-scheduled step", 1: "registers, hand-placed exec masks",
              2: "registers, negated untried set", 3: "registers, no selects (push, pop back)",
              4: "frame re-read from LDS every step", 5: "registers, no last-row step",
              6: "registers, no selects, push without exec mask",
              7: "registers, no selects, push without exec mask, no sentinel frame"}


def run_ablation(nq, torch, n):
    """The paper's design choices measured on this GPU for one board size (one
    launch over the resident frontier, kernel time from HIP events; every run
    checked against the expected count): the pre-placement depth (its Table
    3), the block size of the plain launch (its Table 4), and, at the best
    depth, every inner-loop form: the frame kept in registers or re-read from
    the LDS stack every step, the last-row step on or off (its Table 5), and
    the hand-scheduled steps (its inline assembly, Table 6)."""
    dev = torch.device("cuda:0")
    expect = known_counts()[n]
    depths, plain_k, reps = ABLATION_PLAN[n]
    out = {"n": n, "expected": expect, "depth_sweep": [], "plain_block_sweep": [], "forms": []}

    def once(t, k, **kw):
        total = torch.zeros(1, dtype=torch.int64, device=dev)
        _, _, ms = nq.count_subproblems(n, t[0], t[1], t[2], weight=t[3], counts=False,
                                        total=total, depth=k, timing=True, **kw)
        if int(total.item()) != expect:
            raise SystemExit(f"bench.py: ablation N={n} total {int(total.item())} != {expect} "
                             f"({kw})")
        return ms

    def best_of(t, k, **kw):
        return min(once(t, k, **kw) for _ in range(reps))

    for k in depths:
        t = device_frontier(nq, torch, dev, k, n)
        ms = best_of(t, k)
        nodes = golden_nodes(n, k)
        out["depth_sweep"].append({"depth": k, "subproblems": t[0].numel(), "kernel_ms": ms,
                                   "nodes_per_s": nodes / (ms / 1e3) if nodes else None})
        print(f"[bench] ablation N={n} depth {k}: {ms:.1f} ms", file=sys.stderr, flush=True)
        if k == plain_k:
            for wg in (64, 128, 256, 512, 1024):
                try:
                    pm = once(t, k, mode="plain", wg_size=wg)
                except nq.NQError as e:               # stacks exceed the LDS of a workgroup
                    pm = None
                    print(f"[bench] ablation N={n} plain k={k} wg {wg}: {e}", file=sys.stderr,
                          flush=True)
                out["plain_block_sweep"].append({"depth": k, "wg_size": wg, "kernel_ms": pm})
                if pm is not None:
                    print(f"[bench] ablation N={n} plain k={k} wg {wg}: {pm:.1f} ms",
                          file=sys.stderr, flush=True)
        del t
        torch.cuda.empty_cache()
    best = min(out["depth_sweep"], key=lambda r: r["kernel_ms"])["depth"]
    t = device_frontier(nq, torch, dev, best, n)
    for form in (7, 1, 0, 2, 3, 4, 5, 6):
        nq.set_loop_form(form)
        try:
            fm = best_of(t, best)
        finally:
            nq.set_loop_form(-1)
        out["forms"].append({"form": form, "what": FORM_NAMES[form], "depth": best,
                             "kernel_ms": fm})
        print(f"[bench] ablation N={n} form {form}: {fm:.1f} ms", file=sys.stderr, flush=True)
    del t
    torch.cuda.empty_cache()
    return out


def run_form_sweep(nq, torch, spec, reps):
    """Kernel time of the N=20 count for each (depth, inner-loop form, waves
    per CU[, claim]) of `spec` ("k:form:waves[:claim],...", waves 0 = as many
    as the LDS allows, claim 0 or absent = the library's block size),
    `reps` launches each over one resident frontier per depth, every total
    checked against Q(20); one JSON line per launch."""
    dev = torch.device("cuda:0")
    plan = [tuple(int(v) for v in x.split(":")) for x in spec.split(",") if x.strip()]
    plan = [p if len(p) == 4 else p + (0,) for p in plan]
    cur_k, t = None, None
    try:
        for k, form, waves, claim in sorted(plan, key=lambda x: x[0]):
            if k != cur_k:
                t = None
                torch.cuda.empty_cache()
                t = device_frontier(nq, torch, dev, k)
                cur_k = k
            nq.set_loop_form(form)
            for rep in range(reps):
                total = torch.zeros(1, dtype=torch.int64, device=dev)
                _, _, ms = nq.count_subproblems(N, t[0], t[1], t[2], weight=t[3], counts=False,
                                                total=total, depth=k, timing=True,
                                                waves_per_cu=waves, claim=claim)
                got = int(total.item())
                if got != EXPECT:
                    raise SystemExit(f"bench.py: sweep k={k} form={form} waves={waves}: "
                                     f"{got} != {EXPECT}")
                print(json.dumps({"n": N, "depth": k, "form": form, "waves_per_cu": waves,
                                  "claim": claim, "rep": rep, "kernel_ms": round(ms, 2),
                                  "exact": True}), flush=True)
    finally:
        nq.set_loop_form(-1)


def cpu_baseline(k, budget_s):
    """The oracle on a seeded sample of the N=20 frontier (depth min(k, 8), so
    that the prefix list stays small), one thread per host core this process
    may run on."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    k = min(k, 8)
    pre, _ = oracle.frontier(N, k)
    rng = np.random.default_rng(20251112)
    order = rng.permutation(len(pre))
    # size the sample from a short probe so the run takes about budget_s
    probe = pre[order[:64]]
    t = time.perf_counter()
    _, nd = oracle.count_prefixes(N, probe, threads=cores)
    dt = max(time.perf_counter() - t, 1e-3)
    per_entry = dt / 64
    m = int(min(len(pre), max(64, budget_s / per_entry)))
    sample = pre[order[:m]]
    t = time.perf_counter()
    _, nd = oracle.count_prefixes(N, sample, threads=cores)
    dt = time.perf_counter() - t
    return {"value": float(nd.sum()) / dt, "unit": "DFS nodes/s", "cores": cores,
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{m} seeded subproblems of the N=20 depth-{k} frontier "
                      f"({int(nd.sum())} nodes, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--depth", type=int, default=0, help="0 = autotune over 5..10")
    ap.add_argument("--tune-ms", type=float, default=40000.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--serve-rates", default="25,100,200", help="COUNT requests/s, comma list")
    ap.add_argument("--perm-only", action="store_true",
                    help="only the permanent search (third DFS workload; one JSON line)")
    ap.add_argument("--perm-depths", default="7,8,9,10", help="with --perm-only: depths")
    ap.add_argument("--perm-reps", type=int, default=3, help="with --perm-only: timed runs")
    ap.add_argument("--kings-only", type=int, default=0, metavar="N",
                    help="only the kings search on an N x N board (second DFS workload; one JSON line)")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--serve-reserve", action="store_true",
                    help="with --serving-only: a server created with NQ_FLAG_SERVE_RESERVE")
    ap.add_argument("--serve-reserve-rates", default="200",
                    help="COUNT requests/s for the latency-first server in the full run")
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--claim", type=int, default=0, help="entries per work-head claim (0 = auto)")
    ap.add_argument("--forward", action="store_true", help="claim entries in frontier order")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-shards", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="measure the paper's design choices (depth, plain block size, loop "
                         "forms) and print them as one JSON line instead")
    ap.add_argument("--ablation-n", default="20",
                    help="board sizes of --ablation, comma list from 17..21")
    ap.add_argument("--big-counts", default=None,
                    help="comma list of boards (21..23) counted whole by nq_count's automatic "
                         "chunked path; one JSON line per board")
    ap.add_argument("--resumable", type=int, default=0,
                    help="count this board with nq_count_resumable, --resumable-batch chunks "
                         "per call, printing a line per call (with --resumable-path, "
                         "--resumable-upto)")
    ap.add_argument("--resumable-batch", type=int, default=4,
                    help="chunks per nq_count_resumable call (its buffers live for one call)")
    ap.add_argument("--chunked-repeat", default=None,
                    help="N:depth:chunks:reps - time `reps` whole chunked counts (fresh "
                         "progress files, all chunks in one call) in this process")
    ap.add_argument("--resumable-path", default="n.progress")
    ap.add_argument("--resumable-upto", type=int, default=0, help="stop after this many chunks")
    ap.add_argument("--resumable-chunks", type=int, default=64)
    ap.add_argument("--resumable-depth", type=int, default=0)
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving loop at --serve-rates (one JSON line)")
    ap.add_argument("--ubench", action="store_true",
                    help="the VALU and LDS microbenchmarks behind the roofline, as one JSON line")
    ap.add_argument("--form-sweep", default=None,
                    help="k:form:waves,... - N=20 kernel time per depth, inner-loop form and "
                         "waves per CU (0 = the LDS limit), --form-sweep-reps launches each")
    ap.add_argument("--form-sweep-reps", type=int, default=2)
    ap.add_argument("--ubench-lds-occupancy", action="store_true",
                    help="only the LDS write + read pair at 8..32 waves per CU (one JSON line)")
    ap.add_argument("--ubench-counters", action="store_true",
                    help="one launch of each LDS layout and one VALU launch, for counter passes")
    ap.add_argument("--profile", action="store_true",
                    help="counter runs: one 256 MiB device copy (calibrates the HBM byte "
                         "counters), then one persistent DFS launch at --depth; no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(subproblems are independent: the path would shard by splitting the frontier)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_12009_amd as nq

    if args.profile:
        profile_run(nq, torch, args.depth or 8, args)
        return
    if args.ablation:
        res = [run_ablation(nq, torch, int(x)) for x in args.ablation_n.split(",") if x.strip()]
        print(json.dumps({"ablation": res}), flush=True)
        return
    if args.form_sweep:
        run_form_sweep(nq, torch, args.form_sweep, args.form_sweep_reps)
        return
    if args.ubench or args.ubench_lds_occupancy:
        print(json.dumps({"ubench": run_ubench(nq, args, args.ubench_lds_occupancy)}),
              flush=True)
        return
    if args.big_counts:
        known = known_counts()
        for n in (int(x) for x in args.big_counts.split(",") if x.strip()):
            t = time.perf_counter()
            got, ms = nq.count(n, timing=True)
            row = {"n": n, "count": got, "exact": got == known.get(n), "kernel_ms": ms,
                   "wall_s": time.perf_counter() - t}
            if got != known.get(n):
                raise SystemExit(f"bench.py: Q({n}) = {got}, expected {known.get(n)}")
            print(json.dumps(row), flush=True)
        return
    if args.chunked_repeat:
        import tempfile
        n, depth, chunks, reps = (int(x) for x in args.chunked_repeat.split(":"))
        for rep in range(reps):
            path = os.path.join(tempfile.mkdtemp(), "count.progress")
            t = time.perf_counter()
            total, done, fin = nq.count_resumable(n, path, chunks=chunks, depth=depth)
            wall = time.perf_counter() - t
            if not fin or total != known_counts()[n]:
                raise SystemExit(f"bench.py: chunked Q({n}) = {total}, expected {known_counts()[n]}")
            print(json.dumps({"n": n, "depth": depth, "chunks": chunks, "rep": rep,
                              "wall_s": wall, "exact": True}), flush=True)
        return
    if args.resumable:
        t0 = time.perf_counter()
        while True:
            t = time.perf_counter()
            total, done, fin = nq.count_resumable(args.resumable, args.resumable_path,
                                                  chunks=args.resumable_chunks,
                                                  max_chunks=max(1, args.resumable_batch),
                                                  depth=args.resumable_depth)
            print(json.dumps({"n": args.resumable, "chunks_done": done, "total": total,
                              "chunk_s": time.perf_counter() - t,
                              "elapsed_s": time.perf_counter() - t0, "finished": fin}),
                  flush=True)
            if fin or (args.resumable_upto and done >= args.resumable_upto):
                break
        if fin and total != known_counts().get(args.resumable, total):
            raise SystemExit(f"bench.py: Q({args.resumable}) = {total}, expected "
                             f"{known_counts()[args.resumable]}")
        return
    if args.perm_only:
        depths = tuple(int(x) for x in args.perm_depths.split(",") if x.strip())
        print(json.dumps({"perm": bench_perm(nq, torch, depths=depths, reps=args.perm_reps)}),
              flush=True)
        return
    if args.kings_only:
        print(json.dumps({"kings": bench_kings(nq, args.kings_only)}), flush=True)
        return
    if args.serving_only:
        rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
        print(json.dumps({"serving": bench_serving(nq, torch, known_counts(), rates,
                                                   args.serve_seconds, args.waves_per_cu,
                                                   args.serve_reserve)}),
              flush=True)
        return
    if args.ubench_counters:
        for layout in (0, 1):
            ms = nq.ubench_lds(layout, 64, 16, 10, 1 << 14)
            print(f"[bench] ubench lds layout {layout}: {ms:.2f} ms", file=sys.stderr, flush=True)
        ms = nq.ubench_lds(0, 64, 16, 10, 1 << 14, op=3)
        print(f"[bench] ubench lds exchange: {ms:.2f} ms", file=sys.stderr, flush=True)
        ms, cyc = nq.ubench_valu(0, 8, 8, 1 << 16)
        print(f"[bench] ubench valu v_add3 8 waves/SIMD: {ms:.2f} ms", file=sys.stderr, flush=True)
        return

    tuned = None
    if args.depth == 0:
        print("[bench] autotune N=20 over depths 5..10", file=sys.stderr, flush=True)
        tuned = nq.autotune(N, 5, 10, budget_ms=args.tune_ms, table=True)
        print(f"[bench] tuned { {k: v for k, v in tuned.items() if k != 'table'} }",
              file=sys.stderr, flush=True)
        if tuned["count"] != EXPECT:
            raise SystemExit(f"bench.py: autotune count {tuned['count']} != {EXPECT}")
        stated = [r for r in tuned["table"] if 5 <= r["depth"] <= 8]
        if stated:
            b = min(stated, key=lambda r: r["ms"])
            nodes_b = golden_nodes(N, b["depth"])
            tuned["best_within_stated_depths_5_8"] = dict(
                b, nodes_per_s=(nodes_b / (b["ms"] / 1e3)) if nodes_b else None)
        k = tuned["depth"]
        if not args.wg:
            args.wg = tuned["wg_size"]
        if not args.waves_per_cu:
            args.waves_per_cu = tuned["waves_per_cu"]
        if not args.refill:
            args.refill = tuned["refill_every"]
        if not args.claim:
            args.claim = tuned["claim"]
    else:
        k = args.depth
    dev = torch.device("cuda:0")
    t_cols, t_ld, t_rd, t_w = device_frontier(nq, torch, dev, k)
    F = t_cols.numel()
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    # one pinned slot per timed step: each step's total is checked after the loop
    host_totals = torch.zeros(max(args.steps, args.plain_steps, 1), dtype=torch.int64).pin_memory()
    stream = torch.cuda.current_stream()
    kw = dict(depth=k, wg_size=args.wg, waves_per_cu=args.waves_per_cu,
              refill_every=args.refill, forward=args.forward, claim=args.claim)

    runs = nq.frontier_runs(N, k)

    def step(mode, slot):
        total.zero_()
        if mode == "plain":
            # one launch per row-0 column, each over its run of the frontier
            for lo, hi in zip(runs[:-1], runs[1:]):
                nq.count_subproblems(N, t_cols[lo:hi], t_ld[lo:hi], t_rd[lo:hi],
                                     weight=t_w[lo:hi], counts=False, total=total,
                                     mode=mode, stream=stream, **kw)
        else:
            nq.count_subproblems(N, t_cols, t_ld, t_rd, weight=t_w, counts=False, total=total,
                                 mode=mode, stream=stream, **kw)
        host_totals[slot:slot + 1].copy_(total, non_blocking=True)

    def timed(mode, steps, warmup):
        host_totals.zero_()
        for _ in range(warmup):
            step(mode, 0)
        torch.cuda.synchronize()
        bad = [int(x) for x in host_totals[:min(warmup, 1)] if int(x) != EXPECT]
        if bad:
            raise SystemExit(f"bench.py: {mode} warm-up total {bad[0]} != {EXPECT}")
        host_totals.zero_()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t0 = time.perf_counter()
        for i, (a, b) in enumerate(evs):
            a.record(stream)
            step(mode, i)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        got = [int(x) for x in host_totals[:steps]]
        wrong = [(i, g) for i, g in enumerate(got) if g != EXPECT]
        if wrong:
            raise SystemExit(f"bench.py: {mode} step {wrong[0][0]} total {wrong[0][1]} != {EXPECT}")
        ev_ms = [a.elapsed_time(b) for a, b in evs]
        return wall, ev_ms

    print(f"[bench] N={N} k={k} F={F}: persistent warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    wall, ev_ms = timed("persistent", args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    print(f"[bench] persistent {ms_step:.1f} ms/step (events {np.mean(ev_ms):.1f} ms)",
          file=sys.stderr, flush=True)
    plain_wall, plain_ev = timed("plain", args.plain_steps, 1)
    plain_ms = plain_wall / args.plain_steps * 1e3
    print(f"[bench] plain {plain_ms:.1f} ms/step over {args.plain_steps} steps (events "
          f"{min(plain_ev):.1f}..{max(plain_ev):.1f} ms)", file=sys.stderr, flush=True)

    t = time.perf_counter()
    e2e_total = nq.count(N, depth=k, mode="persistent")
    e2e_ms = (time.perf_counter() - t) * 1e3
    if e2e_total != EXPECT:
        raise SystemExit(f"bench.py: nq_count total {e2e_total} != {EXPECT}")

    nodes = golden_nodes(N, k)
    src = "oracle (tests/golden)" if nodes else None
    kern_ms = float(np.mean(ev_ms))
    out = {
        "metric": "DFS nodes/s + N=20 count wall time on 1 MI355X, batched vs plain, bit-exact",
        "value": (nodes / (ms_step / 1e3)) if nodes else None,
        "unit": "DFS nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"N-Queens N={N} full count, pre-placement depth {k}"
                               f"{' (autotuned over 5..10)' if tuned else ''}, {F} subproblems "
                               "resident in HBM, one persistent launch",
                   "n": N, "depth": k, "subproblems": F, "solutions": EXPECT,
                   "nodes": nodes, "nodes_source": src},
        "plain": {"ms_per_step": plain_ms, "steps": args.plain_steps, "warmup": 1,
                  "event_ms": plain_ev,
                  "value": (nodes / (plain_ms / 1e3)) if nodes else None,
                  "form": "one launch per row-0 column over the same resident frontier"},
        "batched_over_plain": plain_ms / ms_step,
        "end_to_end_ms": e2e_ms,
        "solutions_per_s": EXPECT / (ms_step / 1e3),
    }
    if nodes:
        achieved = nodes * OPS_PER_NODE / (kern_ms / 1e3)
        clk = profiled_clock(N, k)
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_PEAK / 1e12,
                           "unit": "Tint32op/s", "frac": achieved / INT_PEAK,
                           "traffic": profiled_traffic(N, k),
                           "executed": profiled_executed(N, k),
                           "ops_per_node": OPS_PER_NODE, "kernel_ms": kern_ms,
                           "clock_ghz": clk / 1e9 if clk else None,
                           "peak_at_measured_clock": (256 * 64 * clk / 1e12) if clk else None,
                           "frac_at_measured_clock": (achieved / (256 * 64 * clk)) if clk else None,
                           "lds": profiled_lds(N, k, kern_ms)}
    out["launch"] = {"waves_per_cu": args.waves_per_cu, "refill_every": args.refill,
                     "claim": args.claim,
                     "wg_size": args.wg, "autotune": tuned}
    del t_cols, t_ld, t_rd, t_w
    torch.cuda.empty_cache()
    known = known_counts()
    if not args.no_batch:
        print("[bench] ragged batch (256 instances)", file=sys.stderr, flush=True)
        out["batch"] = bench_batch(nq, known)
    print("[bench] kings search (second DFS workload)", file=sys.stderr, flush=True)
    out["kings"] = bench_kings(nq)
    print("[bench] permanent search (third DFS workload)", file=sys.stderr, flush=True)
    out["perm"] = bench_perm(nq, torch)
    if not args.no_shards:
        print("[bench] one GPU's share of N=21 over 8 GPUs", file=sys.stderr, flush=True)
        out["shard"] = bench_shards(nq, torch, known)
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    if rates:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = bench_serving(nq, torch, known, rates, args.serve_seconds)
    rates = [float(x) for x in args.serve_reserve_rates.split(",") if x.strip()]
    if rates:
        print("[bench] serving, latency-first server (NQ_FLAG_SERVE_RESERVE)", file=sys.stderr,
              flush=True)
        out["serving_reserve"] = bench_serving(nq, torch, known, rates, args.serve_seconds,
                                               reserve=True)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(k, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
