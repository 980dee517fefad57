"""Autotuner table lookup (host logic only)."""
import json

from paper_2312_13117_amd import autotune


def test_lookup_picks_smallest_tuned_order_at_least_n(tmp_path):
    t = {"device": "x", "entries": [
        {"n": 256, "precision": 0, "batch": 512, "streams": 2, "graph": 0},
        {"n": 1024, "precision": 0, "batch": 472, "streams": 2, "graph": 0},
        {"n": 1024, "precision": 1, "batch": 256, "streams": 1, "graph": 1},
    ]}
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps(t))
    assert autotune.lookup(100, 0, str(p))["n"] == 256
    assert autotune.lookup(256, 0, str(p))["n"] == 256
    assert autotune.lookup(257, 0, str(p))["n"] == 1024
    assert autotune.lookup(4000, 0, str(p))["n"] == 1024      # beyond the table: largest
    assert autotune.lookup(64, 1, str(p))["batch"] == 256
    assert autotune.lookup(64, 5, str(p)) is None
    assert autotune.lookup(64, 0, str(tmp_path / "missing.json")) is None


def test_select_prefers_lightest_within_margin():
    from paper_2312_13117_amd import autotune
    c = [{"batch": 0, "streams": 1, "graph": 0, "solves_per_s": 90.0},
         {"batch": 0, "streams": 2, "graph": 0, "solves_per_s": 99.0},
         {"batch": 0, "streams": 3, "graph": 0, "solves_per_s": 100.0},
         {"batch": 512, "streams": 2, "graph": 0, "solves_per_s": 99.5},
         {"batch": 0, "streams": 1, "graph": 1, "solves_per_s": 130.0}]   # graph mode: not applied
    b = autotune.select(c)
    assert (b["batch"], b["streams"], b["graph"]) == (0, 2, 0)
    c[2]["solves_per_s"] = 110.0                                          # a clear win for three streams
    assert autotune.select(c)["streams"] == 3
