"""The autotuner's host logic (no GPU): the joint sweep, its tie rule, the
size buckets and the JSON cache that lets a repeated bucket skip the sweep."""
import json
from types import SimpleNamespace

import pytest

from paper_2109_14814_amd import tune


def _pairs(*sizes):
    return [(SimpleNamespace(n_tris=a), SimpleNamespace(n_tris=b)) for a, b in sizes]


def test_auto_table_matches_the_library_rule():
    # bits of the triangle count + 2, clamped to [12, 25]; 2 x 524,288 -> 23
    assert tune.auto_table_log2(2 * 524288) == 23
    assert tune.auto_table_log2(100) == 12
    assert tune.auto_table_log2(1 << 30) == 25


def test_bucket_rounds_sizes_to_powers_of_two():
    k1 = tune.bucket(_pairs((524288, 524288)), "gfx950x256")
    k2 = tune.bucket(_pairs((600000, 500000)), "gfx950x256")
    k3 = tune.bucket(_pairs((524288, 524288)) * 200, "gfx950x256")
    assert k1 == k2 and k1 != k3
    assert k1.startswith("gfx950x256|pairs~2^0|")


def test_sweep_finds_the_minimum_and_breaks_ties_stably():
    calls = []

    def measure(k, t, s):
        calls.append((k, t, s))
        return abs(k - 1.5) + 0.1 * abs(t - 22) + (0.05 if s != 3 else 0.0) + 1.0

    choice, times = tune.sweep(measure, (0.5, 1.0, 1.5, 2.0), (22, 23, 24), default_table=23)
    assert (choice["kappa"], choice["table_log2"], choice["enum_shape"]) == (1.5, 22, 3)
    assert len(set(calls)) == len(calls) == 4 + 2 * 3 * 3 - 2   # each best kappa reuses its stage-1 tuple
    # exact ties resolve to the smallest kappa, then the default table and tile
    flat = lambda k, t, s: 1.0
    choice, _ = tune.sweep(flat, (1.0, 2.0), (22, 23), default_table=23)
    assert (choice["kappa"], choice["table_log2"], choice["enum_shape"]) == (1.0, 23, tune.DEFAULT_SHAPE)


def test_cache_hit_skips_the_sweep(tmp_path):
    path = str(tmp_path / "cache.json")
    pairs = _pairs((5000, 7000))
    n = []

    def measure(k, t, s):
        n.append(1)
        return 1.0 + abs(k - 2.0)

    c1, times = tune.tune(pairs, measure, "dev", batch=False, path=path)
    assert c1["cache"] == "miss" and c1["kappa"] == 2.0 and times and n
    stored = json.load(open(path))
    assert stored[c1["key"]]["kappa"] == 2.0

    def boom(*a):
        raise AssertionError("the sweep ran on a cache hit")

    c2, times2 = tune.tune(pairs, boom, "dev", batch=False, path=path)
    assert c2["cache"] == "hit" and times2 == {}
    assert (c2["kappa"], c2["table_log2"], c2["enum_shape"]) == (c1["kappa"], c1["table_log2"], c1["enum_shape"])
    # another device or size misses
    with pytest.raises(AssertionError):
        tune.tune(pairs, boom, "other", batch=False, path=path)


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert tune.load_cache(str(p)) == {}


def test_tables_reach_one_above_the_largest_automatic_size():
    """Above the automatic ceiling (2^25) the sweep still tries one size more
    (the library takes up to 2^27), and keeps it when it is the fastest."""
    seen = set()

    def measure(k, t, s):
        seen.add(t)
        return 1.0 - 0.5 * (t == 26) + 0.1 * abs(k - 1.5)

    choice, _ = tune.tune(_pairs((1 << 24, 1 << 24)), measure, "dev", batch=True, use_cache=False)
    assert seen == {24, 25, 26}
    assert choice["table_log2"] == 26 and choice["kappa"] == 1.5
