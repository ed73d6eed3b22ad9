"""Host-side behaviour of the autotuner's cache (no GPU needed)."""
import importlib
import json

import pytest


@pytest.fixture
def tune(tmp_path, monkeypatch):
    monkeypatch.setenv("GR_TUNE_CACHE", str(tmp_path / "t.json"))
    import paper_2602_01057_amd.tune as t
    return importlib.reload(t)


def test_cache_roundtrip_and_buckets(tune):
    k1 = tune.cache_key("gfx950|cu256", "ct", "fwd", 50_000, 3_276_800)
    k2 = tune.cache_key("gfx950|cu256", "ct", "fwd", 60_000, 3_000_000)   # same power-of-two buckets
    k3 = tune.cache_key("gfx950|cu256", "ct", "fwd", 500_000, 3_276_800)
    assert k1 == k2 and k1 != k3
    assert tune.load_cache() == {}
    cfg = {"leaf": 32, "waves": 2, "remap": 1, "persistent": 0, "tile": [8, 8], "ms": 1.0}
    tune.store(k1, cfg)
    assert json.load(open(tune.cache_path()))[k1] == cfg
    assert tune.load_cache()[k1]["leaf"] == 32
    assert tune.launch_kwargs(cfg) == {"waves_per_group": 2, "xcd_remap": 1, "persistent": False,
                                       "traversal": 2}
    assert tune.launch_kwargs(dict(cfg, traversal=1))["traversal"] == 1
    g = {"kind": "pet", "tile_radial": 8, "tile_axial": 8}
    t = tune.apply_tile(g, {"tile": [16, 4]})
    assert (t["tile_radial"], t["tile_axial"], t["tile_views"]) == (16, 4, 1)
    t = tune.apply_tile(g, {})  # the PET default: 8 radial x 1 plane x 8 views
    assert (t["tile_radial"], t["tile_axial"], t["tile_views"]) == (8, 1, 8)
    assert tune.apply_tile({"kind": "ct"}, {})["tile_u"] == 8
