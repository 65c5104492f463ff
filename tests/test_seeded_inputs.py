"""The seeded workload generators (shared by the tests and the benchmark)."""
import seeded_inputs as si


def test_splitmix64_reference_outputs():
    # The first outputs of SplitMix64 started from state 0, as printed by the
    # generator's published reference implementation.
    g = 0x9E3779B97F4A7C15
    got = [si.splitmix64((i * g) & si.MASK64) for i in range(4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                   0xF88BB8A8724C81EC]


def test_ragged_batch_sizes():
    ns = si.ragged_batch_ns()
    assert len(ns) == 256 and min(ns) >= 8 and max(ns) <= 19
    assert set(ns) == set(range(8, 20))              # every size occurs
    assert ns == si.ragged_batch_ns()                  # deterministic


def test_poisson_arrivals():
    a = si.poisson_arrivals(2000, 100.0)
    assert all(x < y for x, y in zip(a, a[1:]))
    mean_gap = a[-1] / len(a)
    assert 0.009 < mean_gap < 0.011                    # 1 / rate within 10 %
    ns = si.serve_count_ns(500)
    assert min(ns) >= 10 and max(ns) <= 18 and set(ns) == set(range(10, 19))
