"""Host logic of the batch autotuner: size classes, the JSON cache and the
candidate sweep (timings injected, no GPU)."""
import json

from paper_2607_02749_amd import autotune


def test_size_class_groups_similar_batches():
    a = autotune.size_class([12, 15, 20], [2, 3, 4])
    b = autotune.size_class([12, 15, 20], [2, 3, 4])
    c = autotune.size_class([12, 15, 21], [2, 3, 4])
    assert a == b and a != c
    assert a.startswith("n12-20_L2-4_c4_")


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(p) == {}
    autotune.store_cache("gfx950/c64/batch/x", {"blocks_per_cu": 3, "order": 1, "ms": 1.5}, p)
    autotune.store_cache("gfx950/c64/batch/y", {"blocks_per_cu": 1, "order": 0, "ms": 2.0}, p)
    d = json.load(open(p))
    assert d["gfx950/c64/batch/x"]["blocks_per_cu"] == 3
    assert set(autotune.load_cache(p)) == {"gfx950/c64/batch/x", "gfx950/c64/batch/y"}


def test_cache_ignores_corrupt_file(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert autotune.load_cache(str(p)) == {}


def test_sweep_picks_fastest():
    fake = {(1, 0, 17, 12): 3.0, (1, 1, 17, -1): 2.5, (2, 0, 31, 12): 1.25, (2, 1, 15, -1): 4.0}
    r = autotune.sweep(sorted(fake), lambda b, o, sp, ld: fake[(b, o, sp, ld)])
    assert (r["blocks_per_cu"], r["order"], r["split_n"], r["lds_n"], r["ms"]) == (2, 0, 31, 12, 1.25)
    assert len(r["timings"]) == 4
