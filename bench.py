"""Benchmark: DFS nodes/s of the N=20 count on one MI355X, batched vs plain.

One step = the whole device path over the resident N=20 frontier (pre-placement
depth k, built once on the host and copied to HBM before the timed region):
zero the total, one persistent DFS launch over every subproblem (per-entry
counts + weighted total), and the copy of the 8-byte total back to the host,
which is checked against Q(20) = 39,029,188,884 every step.

value = DFS nodes per second = nodes(20, k) / step time, where nodes(20, k) is
the oracle's node count (queens placed in rows k..18 below every pre-placed
prefix), read from tests/golden/oracle_runs.txt.

Printed: one JSON line (rank 0) with the metric, the "plain" form (one launch
per row-0 column over the same frontier), the end-to-end nq_count wall time,
the int-ALU roofline of the DFS kernel and the oracle timed on the host cores.
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


def cpu_baseline(k, budget_s):
    """The oracle on a seeded sample of the N=20 frontier, all host cores."""
    import oracle
    cores = min(os.cpu_count() or 1, 16)
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
            "kind": "oracle",
            "sample": f"{m} seeded subproblems of the N=20 depth-{k} frontier "
                      f"({int(nd.sum())} nodes, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--depth", type=int, default=6)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--forward", action="store_true", help="claim entries in frontier order")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by splitting the frontier, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_12009_amd as nq

    k = args.depth
    cols, ld, rd, w = nq.frontier(N, k)
    F = len(cols)
    dev = torch.device("cuda:0")
    t_cols = torch.from_numpy(cols.view(np.int32)).to(dev)
    t_ld = torch.from_numpy(ld.view(np.int32)).to(dev)
    t_rd = torch.from_numpy(rd.view(np.int32)).to(dev)
    t_w = torch.from_numpy(w).to(dev)
    counts = torch.empty(F, dtype=torch.int64, device=dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    host_total = torch.zeros(1, dtype=torch.int64).pin_memory()
    stream = torch.cuda.current_stream()
    kw = dict(depth=k, wg_size=args.wg, waves_per_cu=args.waves_per_cu,
              refill_every=args.refill, forward=args.forward)

    runs = nq.frontier_runs(N, k)

    def step(mode):
        total.zero_()
        if mode == "plain":
            # one launch per row-0 column, each over its run of the frontier
            for lo, hi in zip(runs[:-1], runs[1:]):
                nq.count_subproblems(N, t_cols[lo:hi], t_ld[lo:hi], t_rd[lo:hi],
                                     weight=t_w[lo:hi], counts=counts[lo:hi], total=total,
                                     mode=mode, stream=stream, **kw)
        else:
            nq.count_subproblems(N, t_cols, t_ld, t_rd, weight=t_w, counts=counts, total=total,
                                 mode=mode, stream=stream, **kw)
        host_total.copy_(total, non_blocking=True)

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            step(mode)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if int(host_total.item()) != EXPECT:
            raise SystemExit(f"bench.py: {mode} total {int(host_total.item())} != {EXPECT}")
        ev_ms = [a.elapsed_time(b) for a, b in evs]
        return wall, ev_ms

    print(f"[bench] N={N} k={k} F={F}: persistent warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    wall, ev_ms = timed("persistent", args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    print(f"[bench] persistent {ms_step:.1f} ms/step (events {np.mean(ev_ms):.1f} ms)",
          file=sys.stderr, flush=True)
    plain_wall, plain_ev = timed("plain", args.plain_steps, 0)
    plain_ms = plain_wall / args.plain_steps * 1e3
    print(f"[bench] plain {plain_ms:.1f} ms/step", file=sys.stderr, flush=True)

    t = time.perf_counter()
    e2e_total = nq.count(N, depth=k, mode="persistent")
    e2e_ms = (time.perf_counter() - t) * 1e3
    if e2e_total != EXPECT:
        raise SystemExit(f"bench.py: nq_count total {e2e_total} != {EXPECT}")

    nodes = golden_nodes(N, k)
    src = "oracle (tests/golden)" if nodes else None
    kern_ms = float(np.mean(ev_ms))
    out = {
        "metric": "DFS nodes/s (N=20 count, 1 MI355X, batched persistent launch, bit-exact)",
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
        "config": {"workload": f"N-Queens N={N} full count, pre-placement depth {k}, "
                               f"{F} subproblems, persistent launch",
                   "n": N, "depth": k, "subproblems": F, "solutions": EXPECT,
                   "nodes": nodes, "nodes_source": src},
        "plain": {"ms_per_step": plain_ms,
                  "value": (nodes / (plain_ms / 1e3)) if nodes else None,
                  "form": "one launch per row-0 column over the same resident frontier"},
        "batched_over_plain": plain_ms / ms_step,
        "end_to_end_ms": e2e_ms,
        "solutions_per_s": EXPECT / (ms_step / 1e3),
    }
    if nodes:
        achieved = nodes * OPS_PER_NODE / (kern_ms / 1e3)
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_PEAK / 1e12,
                           "unit": "Tint32op/s", "frac": achieved / INT_PEAK, "traffic": None,
                           "ops_per_node": OPS_PER_NODE, "kernel_ms": kern_ms}
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(k, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
