"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

Holds no part of the counting method: only the random draws that define the
workloads (board sizes of a ragged batch, request streams of the serving loop,
the 0/1 matrices of the permanent search).
The generator is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written from its published
definition; a draw for index i is the SplitMix64 output of state seed + i.
"""
import math

MASK64 = (1 << 64) - 1

RAGGED_SEED = 0x251112009
SERVE_SEED = 0x5E4E
SLICE_SAMPLE_SEED = 0x5E21
MATRIX_SEED = 0x9E12


def splitmix64(state: int) -> int:
    """One SplitMix64 output for the given 64-bit state (the state is advanced
    by the golden-ratio increment, then mixed)."""
    z = (state + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform01(state: int) -> float:
    """A double in (0, 1] from the top 53 bits of one SplitMix64 output."""
    return ((splitmix64(state) >> 11) + 1) * (1.0 / (1 << 53))


def ragged_batch_ns(count: int = 256, lo: int = 8, hi: int = 19, seed: int = RAGGED_SEED):
    """Board sizes of a ragged batch: N_i uniform in [lo, hi], seeded."""
    span = hi - lo + 1
    return [lo + splitmix64((seed + i) & MASK64) % span for i in range(count)]


def poisson_arrivals(count: int, rate_per_s: float, seed: int = SERVE_SEED):
    """Arrival times (seconds from 0) of a Poisson stream: inter-arrival -ln(U)/rate."""
    t, out = 0.0, []
    for i in range(count):
        t += -math.log(uniform01((seed + 2 * i) & MASK64)) / rate_per_s
        out.append(t)
    return out


def serve_count_ns(count: int, lo: int = 10, hi: int = 18, seed: int = SERVE_SEED):
    """Board sizes of the COUNT requests of the serving workload: uniform in [lo, hi]."""
    span = hi - lo + 1
    return [lo + splitmix64((seed + 2 * i + 1) & MASK64) % span for i in range(count)]


def sample_slices(count: int, nslices: int, seed: int = SLICE_SAMPLE_SEED):
    """`count` distinct slice indices in [0, nslices), seeded (the oracle checks
    of the serving workload's N=21 slices use them), in ascending order."""
    picked, i = set(), 0
    while len(picked) < min(count, nslices):
        picked.add(splitmix64((seed + i) & MASK64) % nslices)
        i += 1
    return sorted(picked)


def matrix01(n: int, density: float, seed: int = MATRIX_SEED):
    """An n x n 0/1 matrix (list of rows of ints 0/1): entry (r, c) is 1 when
    the uniform draw of index r * n + c is at most `density`."""
    return [[1 if uniform01((seed + r * n + c) & MASK64) <= density else 0 for c in range(n)]
            for r in range(n)]
