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
