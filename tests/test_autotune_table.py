"""The autotuner's shipped table (host only): every entry is a configuration the library
accepts, under a key in the tuner's own format."""

import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2509_14442_amd",
                     "autotune_table.json")


def _entries():
    with open(TABLE) as f:
        return json.load(f)


def test_table_entries_are_valid_configurations():
    from paper_2509_14442_amd import autotune

    db = _entries()
    assert db, "empty table"
    launches = {(tuple(t), w, p, b) for t, w, p, b in autotune.LAUNCHES}
    for key, e in db.items():
        parts = key.split("|")
        assert parts[0] == "v4" and parts[1].startswith("gfx") and parts[-1] in ("fwd", "fwd+adj"), key
        assert parts[2] in ("f32", "f16", "bf16") and parts[3] in ("t0", "t1"), key
        assert e["ckpt_stride"] in autotune.STRIDES, key
        assert e["layout"] in autotune.LAYOUTS, key
        assert e["ms"] > 0, key
        for which in ("fwd", "adj") if parts[-1] == "fwd+adj" else ("fwd",):
            l = e[which]
            assert (tuple(l["tile"]), l["waves_per_block"], l["persistent"], l["blocks_per_cu"]) in launches, key
        assert "source" not in e, key  # added on return, never stored


def test_table_covers_the_benchmark_workloads():
    """The room at FP32, FP16 and BF16 (1M rays, 128^3), the quasi-linear tracer, 4 rays per
    pixel, the 64-scene batch and the 256x256x192 room."""
    keys = list(_entries())
    wanted = [("f32", "t0", "spp1", "g21", "r20", "n1"), ("f16", "t0", "spp1", "g21", "r20", "n1"),
              ("bf16", "t0", "spp1", "g21", "r20", "n1"), ("f32", "t1", "spp1", "g21", "r20", "n1"),
              ("f32", "t0", "spp4", "g21", "r22", "n1"), ("f32", "t0", "spp1", "g21", "r24", "n64"),
              ("f32", "t0", "spp1", "g24", "r22", "n1")]
    for w in wanted:
        assert any(all(part in k.split("|") for part in w) for k in keys), w
