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


def test_search_space_and_tie_break_on_a_fake_device(tune, monkeypatch):
    """The fused search space runs every listed combination, and the default
    configuration wins unless another is faster by more than the margin."""
    import types

    class FakeScene:
        def __init__(self, *a, kappa=3.0, leaf_size=0):
            self.n, self.leaf = 10, leaf_size

        def status_flags(self):
            return 0

    class FakeTensor:
        def __init__(self, m):
            self.shape = (3, m)

        def numel(self):
            return self.shape[1]

    times = {}

    def fake_time(fn, reps):
        return fn()

    calls = []

    def fake_backward(scene, ro, rd, loss, target, scratch, waves_per_group, xcd_remap, persistent, traversal):
        calls.append((scene.leaf, waves_per_group, traversal))
        key = (scene.leaf, waves_per_group, traversal)
        return times.get(key, 10.0)

    fake_api = types.SimpleNamespace(
        make_rays=lambda g, dev, planes=None: (FakeTensor(640), FakeTensor(640)), Scene=FakeScene,
        fused_scratch_bytes=lambda n, w: 64, project_backward=fake_backward,
        ray_count=lambda g, planes=None: 640)
    monkeypatch.setattr(tune, "api", fake_api)
    monkeypatch.setattr(tune, "_time", fake_time)
    monkeypatch.setattr(tune.torch, "empty", lambda *a, **k: None)
    monkeypatch.setattr(tune.torch, "zeros", lambda m, device=None: FakeTensor(m))
    params = [types.SimpleNamespace(device="cpu")] * 4
    geom = {"kind": "ct", "n_views": 4}
    times[(64, 1, 2)] = 10.0
    times[(32, 2, 1)] = 9.6          # within 5 %: the default stays
    best = tune.tune(params, geom, op="bwd", max_rays=None, search=tune.SEARCH_FUSED, save=False)
    assert (best["leaf"], best["waves"], best["traversal"], best["tile"]) == (64, 1, 2, [8, 8])
    assert len(calls) == 3 * 2 * 2 * 2   # tiles x leaves x waves x traversals
    times[(32, 2, 1)] = 9.0          # clearly faster (> 5 %): it wins
    best = tune.tune(params, geom, op="bwd", max_rays=None, search=tune.SEARCH_FUSED, save=False)
    assert (best["leaf"], best["waves"], best["traversal"]) == (32, 2, 1)


def test_tuning_slices(tune):
    """A CT slice is the views that fit. A PET slice keeps every view (their
    angular spacing depends on their count, and view-blocked packets on it)
    and takes whole blocks of 8 of the default ring pairs."""
    from paper_2602_01057_amd import api
    from paper_2602_01057_amd.inputs import CT_CONE_500K, PET_200K
    ct, none = tune._slice_geom(CT_CONE_500K["geom"], 1_500_000)
    assert none is None and ct["n_views"] == 1_500_000 // (512 * 512)
    g = PET_200K["geom"]
    pet, planes = tune._slice_geom(g, 1_500_000)   # 17 planes' worth of lines
    assert pet["n_views"] == g["n_views"] and len(planes) == 16
    assert planes[:3] == [(0, 0), (1, 1), (2, 2)] and planes[-1] == (15, 15)
    allp = tune._pet_planes(g, 1 << 30)
    assert api.ray_count(g) == len(allp) * g["n_radial"] * g["n_views"]
    assert len(set(allp)) == len(allp) and all(abs(a - b) <= g["max_ring_diff"] for a, b in allp)
    assert allp[g["n_rings"]] == (0, 1) and allp[2 * g["n_rings"] - 1] == (1, 0)
    assert tune._slice_geom(g, None) == (g, None)
    assert tune._slice_geom(g, 10 ** 12)[1] is None
