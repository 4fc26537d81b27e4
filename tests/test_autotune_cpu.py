"""Autotuner host logic (no GPU): buckets, keys, choice rule, cache file."""
import os

from paper_2410_01752_amd import autotune as A


def test_n_bucket_and_key():
    assert A.n_bucket(50) == "n<=64"
    assert A.n_bucket(500) == "n<=512"
    assert A.n_bucket(2000) == "n<=2048"
    assert A.n_bucket(2048) == "n<=2048"
    assert A.cache_key("gfx950", "7.0", "k_score_rect", "fp32", 2000) == "gfx950|7.0|k_score_rect|fp32|n<=2048"


def test_pick_fastest_and_ties_go_first():
    t = {(0, 0): 3.0, (1, 256): 2.0, (2, 512): 2.0, (0, 768): 5.0}
    assert A.pick(t) == (1, 256)


def test_cache_round_trip(tmp_path):
    path = os.path.join(str(tmp_path), "sub", "at.json")
    c = A.Cache(path)
    assert c.get("k") is None
    c.put("k", A.Choice(1, 512, 12.5, {"tile1_grid512": 12.5}))
    c2 = A.Cache(path)
    ch = c2.get("k")
    assert (ch.tile, ch.grid, ch.ms) == (1, 512, 12.5)
    with open(path, "w") as f:
        f.write("not json")
    assert A.Cache(path).get("k") is None      # unreadable cache is ignored
