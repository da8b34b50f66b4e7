"""The committed launch-shape cache that bench.py's ensemble reads holds an
entry for that ensemble (64 uneven ducts, FP32) at the current source of the
step: the cache key carries the source digest, so a change to the step
kernel or its layout code needs a re-tune (bench.py --tune on a GPU), or the
benchmark falls back to an untuned shape."""
import bench
from paper_1711_03254_amd import autotune, inputs


def test_committed_cache_matches_the_current_step():
    doms = inputs.ensemble_case(64)
    key = autotune.batch_key(doms, "fp32")
    table = autotune._load(bench.TUNED)
    assert key in table, f"no tuned launch shape under {key}: re-tune with bench.py --tune"
    ent = table[key]
    assert ent["ms"] == min(ent["all_ms"].values())
    best = min(ent["all_ms"], key=ent["all_ms"].get)
    assert best == f"{ent['tile'][0]}x{ent['tile'][1]}/{ent['zchunk']}"
