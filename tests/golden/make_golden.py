"""Writes oracle_runs.txt: per-frontier oracle results used as stored expected values.

Calls only the oracle package.  For each (N, k) it enumerates the symmetry-reduced
frontier, counts every prefix's completions and nodes with the oracle, and
records: F, the weighted total, the node total, and SHA-256 digests of the
per-prefix counts and nodes (little-endian uint64 in canonical frontier order),
so that a test can check every per-subproblem result without rerunning the
oracle.  Usage:  python tests/golden/make_golden.py N:k [N:k ...] [--threads T]
An existing line for the same (N, k) is replaced.

With --slices N:k:len:count it instead writes oracle_slices.txt: the oracle's
counts of `count` seeded slices of `len` entries of the (N, k) frontier (slice
indices from seeded_inputs.sample_slices, plus the last, short slice), one line
per slice: N k start len weighted_total node_total sha256(counts u64 LE).

With --perm N:density[:seed] ... it writes perm_totals.txt: the permanent of
the seeded 0/1 matrix (seeded_inputs.matrix01 with seed MATRIX_SEED + seed)
by the oracle's Ryser routine, and for N <= 15 also by its search (both must
agree): N density seed permanent.
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import seeded_inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_runs.txt")
SLICES_OUT = os.path.join(HERE, "oracle_slices.txt")
SLICES_HEADER = """# Oracle counts of seeded slices of a frontier (canonical order), written by
# tests/golden/make_golden.py --slices (oracle only).
# N k start len weighted_total node_total sha256(counts u64 LE)
"""
NODES_OUT = os.path.join(HERE, "oracle_nodes.txt")
NODES_HEADER = """# Node counts nodes(N, k) (queens placed in rows k..N-2 below every frontier
# prefix), written by tests/golden/make_golden.py.  "run" lines repeat an
# oracle run of oracle_runs.txt; "derived" lines (even N only) follow from one by
# the node identity nodes(k) = nodes(j) + F(k+1) + ... + F(j) for k < j (and the
# same with the sign reversed for k > j), with F from the oracle's frontier.
# N k nodes source
"""
PERM_OUT = os.path.join(HERE, "perm_totals.txt")
PERM_HEADER = """# Permanents of seeded 0/1 matrices (seeded_inputs.matrix01(N, density,
# MATRIX_SEED + seed)), written by tests/golden/make_golden.py --perm (oracle only:
# Ryser's formula, and the oracle's search where it finishes).
# N density seed permanent
"""
HEADER = """# Oracle results per frontier, written by tests/golden/make_golden.py (oracle only).
# N k F weighted_total node_total sha256(counts u64 LE) sha256(nodes u64 LE) oracle_seconds threads
"""


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def run(n, k, threads):
    t0 = time.time()
    pre, w = oracle.frontier(n, k)
    counts, nodes = oracle.count_prefixes(n, pre, threads=threads)
    secs = time.time() - t0
    total = int(np.sum(counts.astype(object) * w.astype(object))) if len(w) else 0
    return (f"{n} {k} {len(w)} {total} {int(nodes.sum())} {digest(counts)} {digest(nodes)} "
            f"{secs:.1f} {threads}")


def write_nodes():
    """Node counts at depths j-2..j+4 for every even N with an oracle run at depth j."""
    runs = []
    with open(OUT) as f:
        runs = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    lines = []
    for r in runs:
        n, j, nodes = int(r[0]), int(r[1]), int(r[4])
        lines.append((n, j, nodes, "run"))
        if n % 2:
            continue
        for k in range(max(1, j - 2), min(n, j + 5)):
            if k == j or any(x[0] == n and x[1] == k for x in runs):
                continue
            if k < j:
                v = nodes + sum(oracle.frontier_size(n, d) for d in range(k + 1, j + 1))
            else:
                v = nodes - sum(oracle.frontier_size(n, d) for d in range(j + 1, k + 1))
            lines.append((n, k, v, f"derived-from-k{j}"))
    lines.sort()
    with open(NODES_OUT, "w") as f:
        f.write(NODES_HEADER)
        for n, k, v, src in lines:
            f.write(f"{n} {k} {v} {src}\n")


def write_slices(spec, threads):
    n, k, length, count = (int(x) for x in spec.split(":"))
    pre, w = oracle.frontier(n, k)
    nslices = (len(pre) + length - 1) // length
    picks = sorted(set(seeded_inputs.sample_slices(count, nslices)) | {nslices - 1})
    lines = []
    if os.path.exists(SLICES_OUT):
        with open(SLICES_OUT) as f:
            lines = [ln for ln in f if ln.strip() and not ln.startswith("#")]
    for j in picks:
        lo, hi = j * length, min(len(pre), (j + 1) * length)
        counts, nodes = oracle.count_prefixes(n, pre[lo:hi], threads=threads)
        total = int(np.sum(counts.astype(object) * w[lo:hi].astype(object)))
        line = f"{n} {k} {lo} {hi - lo} {total} {int(nodes.sum())} {digest(counts)}"
        print(line, flush=True)
        lines = [ln for ln in lines if ln.split()[:4] != line.split()[:4]] + [line + "\n"]
    lines.sort(key=lambda ln: tuple(int(x) for x in ln.split()[:4]))
    with open(SLICES_OUT, "w") as f:
        f.write(SLICES_HEADER)
        f.writelines(lines)


def write_perm(specs):
    lines = []
    if os.path.exists(PERM_OUT):
        with open(PERM_OUT) as f:
            lines = [ln for ln in f if ln.strip() and not ln.startswith("#")]
    for spec in specs:
        parts = spec.split(":")
        n, dens = int(parts[0]), float(parts[1])
        seed = int(parts[2]) if len(parts) > 2 else 0
        a = np.array(seeded_inputs.matrix01(n, dens, seeded_inputs.MATRIX_SEED + seed), np.uint8)
        value = oracle.permanent_ryser(a)
        if n <= 15 and oracle.permanent(a)[0] != value:
            raise SystemExit(f"oracle search and Ryser disagree for {spec}")
        line = f"{n} {dens} {seed} {value}"
        print(line, flush=True)
        lines = [ln for ln in lines if ln.split()[:3] != line.split()[:3]] + [line + "\n"]
    lines.sort(key=lambda ln: (int(ln.split()[0]), float(ln.split()[1]), int(ln.split()[2])))
    with open(PERM_OUT, "w") as f:
        f.write(PERM_HEADER)
        f.writelines(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--slices", default=None, help="N:k:len:count")
    ap.add_argument("--perm", nargs="+", default=None, help="N:density[:seed] ...")
    args = ap.parse_args()
    if args.slices:
        write_slices(args.slices, args.threads)
        return
    if args.perm:
        write_perm(args.perm)
        return
    for case in args.cases:
        n, k = (int(x) for x in case.split(":"))
        line = run(n, k, args.threads)
        print(line, flush=True)
        lines = []
        if os.path.exists(OUT):
            with open(OUT) as f:
                lines = [ln for ln in f if ln.strip() and not ln.startswith("#")]
        lines = [ln for ln in lines if ln.split()[:2] != [str(n), str(k)]] + [line + "\n"]
        lines.sort(key=lambda ln: (int(ln.split()[0]), int(ln.split()[1])))
        with open(OUT, "w") as f:
            f.write(HEADER)
            f.writelines(lines)
    write_nodes()


if __name__ == "__main__":
    main()
