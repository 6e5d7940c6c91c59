"""The seeded workloads bench.py measures, checked on the CPU: the uneven batch (classes 2..100 with the per-shape
encoding every product's preconditions accept) and the serving mix built from it."""
import numpy as np

import bench


def test_uneven_requests_cover_the_stated_ranges_with_valid_encodings():
    spec = bench.uneven_requests(bench.SEEDS["data"] + 7, 64, True)
    assert len(spec) == 64
    assert [r["op"] for r in spec] == ["abt", "atb"] * 32
    assert all(32 <= r["rows"] <= 512 and 64 <= r["inner"] <= 1024 and 2 <= r["classes"] <= 100 for r in spec)
    assert max(r["classes"] for r in spec) > 64          # the large-c' classes are exercised
    for r in spec:
        s0, c = r["s0"], r["c"]
        s1 = 32768 // s0
        assert s0 * s1 == 32768 and s0 & (s0 - 1) == 0 and c & (c - 1) == 0
        assert c >= r["classes"] and c // 2 < r["classes"] or c == 2   # the next power of two
        assert 1 < c <= s0 and s1 % c == 0                    # DiagABT's and DiagATB's preconditions
        assert s0 >= min(r["rows"], 32768 // c) or s0 == 32768 // c


def test_uneven_requests_are_seeded_and_the_standard_encoding_is_uniform():
    a = bench.uneven_requests(11, 16, True)
    assert a == bench.uneven_requests(11, 16, True)
    assert a != bench.uneven_requests(12, 16, True)
    std = bench.uneven_requests(11, 16, False)
    assert all(r["s0"] == bench.S0 and r["c"] == 128 for r in std)
    assert [(r["rows"], r["inner"], r["classes"]) for r in std] == [(r["rows"], r["inner"], r["classes"]) for r in a]


def test_serving_mix_gives_every_client_two_products_of_each_kind():
    spec = bench.uneven_requests(bench.SEEDS["data"] + 7, 4 * 16, True)
    for cl in range(16):
        mine = spec[4 * cl:4 * cl + 4]
        assert sorted(r["op"] for r in mine) == ["abt", "abt", "atb", "atb"]
    rng = np.random.default_rng(0)
    assert len(set(int(x) for x in rng.integers(0, 16, size=2000))) == 16
