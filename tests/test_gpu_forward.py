"""Forward parity of the HIP path against the FP64 oracle (same seeded FP32
inputs on both sides), plus edge cases and exact invariances."""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_2602_01057_amd.inputs import CT_CONE_50K, CT_PARALLEL_SMALL, Scene, preset_scene, sample_scene
from parity import assert_forward

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def dev_scene(gr, sc, kappa=3.0, leaf=0):
    S = gr.Scene(to_dev(sc.mean.astype(np.float32)), to_dev(sc.scale.astype(np.float32)),
                    to_dev(sc.quat.astype(np.float32)), to_dev(sc.density.astype(np.float32)),
                    kappa=kappa, leaf_size=leaf)
    assert S.status_flags() == 0
    return S


def gpu_project(gr, sc, o, d, kappa=3.0, leaf=0, **kw):
    import torch
    S = dev_scene(gr, sc, kappa, leaf)
    out = gr.project(S, to_dev(o.astype(np.float32)), to_dev(d.astype(np.float32)), **kw)
    torch.cuda.synchronize()
    assert S.status_flags() == 0
    return out.cpu().numpy()


def test_parallel_beam_512_all_rays(gr):
    """Parallel-beam CT, 512 Gaussians, 32 views of 64x64: every ray vs oracle."""
    p = CT_PARALLEL_SMALL
    sc = preset_scene(p)
    o, d = G.rays32(p["geom"])
    ref = oracle.project(sc, o, d)
    I = gpu_project(gr, sc, o, d)
    worst = assert_forward(I, ref, what="ct_parallel_512")
    print(f"max rel err {worst:.2e}; hits {int(ref['hits'].sum())}; rays with hits "
          f"{int((ref['hits'] > 0).sum())}/{o.shape[1]}")
    assert (ref["hits"] > 0).sum() > 10000


@pytest.mark.parametrize("traversal", [1, 2])
@pytest.mark.parametrize("leaf", [1, 2, 7, 16, 33, 64])
def test_leaf_sizes_and_ragged_tail(gr, leaf, traversal):
    """Several leaf sizes, both traversals (binary LBVH, 64-wide hierarchy);
    1000 rays (15 full packets + a ragged tail of 40)."""
    sc = sample_scene(777, seed=5, radius=60.0, scale_range=(1.0, 9.0))
    geom = dict(kind="ct", cone=1, n_views=3, nu=20, nv=17, angle0=0.3, angle_range=5.0, dso=400.0,
                dsd=700.0, pitch_u=4.0, pitch_v=4.0, offset_u=1.0, offset_v=-2.0, tile_u=8, tile_v=8)
    o, d = G.rays32(geom)
    o, d = o[:, :1000], d[:, :1000]
    ref = oracle.project(sc, o, d)
    assert_forward(gpu_project(gr, sc, o, d, leaf=leaf, traversal=traversal), ref,
                   what=f"leaf {leaf} traversal {traversal}")


def test_incoherent_rays_and_non_unit_directions(gr):
    """Random lines in random order (degenerate packet beams) with |d| != 1."""
    rng = np.random.default_rng(3)
    sc = sample_scene(400, seed=6, radius=40.0, scale_range=(1.0, 8.0))
    m = 3000
    o = rng.uniform(-60, 60, (3, m)).astype(np.float32)
    d = (rng.standard_normal((3, m)) * rng.uniform(0.2, 4.0, m)).astype(np.float32)
    ref = oracle.project(sc, o, d)
    assert_forward(gpu_project(gr, sc, o, d), ref, what="incoherent")


def test_far_origins(gr):
    """Origins at the cone-beam source (|o| = 1000 mm), where the literal
    C - B^2/A cancels in FP32."""
    sc = sample_scene(3000, seed=7, radius=100.0, scale_range=(0.8, 6.0))
    g = dict(CT_CONE_50K["geom"], n_views=2, nu=64, nv=64, pitch_u=6.4, pitch_v=6.4)
    o, d = G.rays64(g)
    v = np.arange(o.shape[1]) // (64 * 64)
    ang = v * (2 * math.pi / 2)
    S = 1000.0 * np.stack([np.cos(ang), np.sin(ang), 0 * ang])
    o32 = S.astype(np.float32)
    d32 = d.astype(np.float32)
    ref = oracle.project(sc, o32, d32)
    assert (ref["hits"] > 0).sum() > 1000
    assert_forward(gpu_project(gr, sc, o32, d32), ref, what="far origins")


def test_edge_cases(gr):
    import torch
    rng = np.random.default_rng(9)
    o = rng.uniform(-30, 30, (3, 130)).astype(np.float32)
    d = rng.standard_normal((3, 130)).astype(np.float32)
    # empty scene: all zeros
    e = Scene(np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32),
              np.zeros(0, np.float32))
    assert np.all(gpu_project(gr, e, o, d) == 0)
    # one Gaussian
    s1 = sample_scene(1, seed=1, radius=5.0, scale_range=(5.0, 10.0))
    assert_forward(gpu_project(gr, s1, o, d), oracle.project(s1, o, d), what="n=1")
    # zero rays
    S = dev_scene(gr, s1)
    out = gr.project(S, torch.empty(3, 0, device="cuda"), torch.empty(3, 0, device="cuda"))
    assert out.numel() == 0
    # invalid Gaussians are excluded and counted
    sc = sample_scene(200, seed=2, radius=30.0, scale_range=(1.0, 6.0))
    bad_s = sc.scale.copy()
    bad_q = sc.quat.copy()
    bad_m = sc.mean.copy()
    bad_s[0, 3] = 0.0
    bad_s[1, 10] = -1.0
    bad_q[:, 20] = 0.0
    bad_m[2, 30] = np.nan
    bad_s[2, 40] = np.inf
    bad = Scene(bad_m, bad_s, bad_q, sc.density)
    ref = oracle.project(bad, o, d)
    S = dev_scene(gr, bad)
    assert S.invalid_count() == 5
    I = gr.project(S, to_dev(o), to_dev(d)).cpu().numpy()
    assert_forward(I, ref, what="invalid gaussians")
    # kappa other than 3
    ref2 = oracle.project(sc, o, d, kappa=1.7)
    assert_forward(gpu_project(gr, sc, o, d, kappa=1.7), ref2, what="kappa 1.7")
    # all Gaussians in one leaf position (identical Morton codes)
    same = Scene(np.zeros((3, 100), np.float32) + 1.0, sc.scale[:, :100], sc.quat[:, :100],
                 sc.density[:100])
    assert_forward(gpu_project(gr, same, o, d), oracle.project(same, o, d), what="coincident means")


def test_deterministic_and_exact_invariances(gr):
    """Repeat runs are bitwise equal; FP32-exact transforms of the inputs give
    exactly related outputs (d -> 2d halves I; d -> -d and axis permutations
    keep I within tolerance)."""
    sc = sample_scene(2000, seed=11, radius=80.0, scale_range=(1.0, 7.0))
    g = dict(CT_CONE_50K["geom"], n_views=3, nu=48, nv=48, pitch_u=8.0, pitch_v=8.0)
    o, d = G.rays32(g)
    a = gpu_project(gr, sc, o, d)
    b = gpu_project(gr, sc, o, d)
    assert np.array_equal(a, b)
    h = gpu_project(gr, sc, o, 2 * d)
    ref = oracle.project(sc, o, d)
    assert_forward(h * 2, ref, what="2d")
    assert_forward(gpu_project(gr, sc, o, -d), ref, what="-d")
    perm = [2, 0, 1]
    # permuting world axes: mean/rays permuted, rotation conjugated by the permutation
    from scipy.spatial.transform import Rotation
    P = np.eye(3)[perm]
    q = sc.quat.astype(np.float64)
    rq = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], 1))
    rp = Rotation.from_matrix(P) * rq
    qq = rp.as_quat()
    sc_p = Scene(sc.mean[perm], sc.scale, np.stack([qq[:, 3], qq[:, 0], qq[:, 1], qq[:, 2]]).astype(np.float32),
                 sc.density)
    ref_p = oracle.project(sc_p, o[perm], d[perm])
    assert_forward(gpu_project(gr, sc_p, o[perm], d[perm]), ref_p, what="axis permutation")


@pytest.mark.timeout(600)
def test_cone_beam_50k_full_size_whole_views(gr):
    """Cone-beam CT at full size (50k Gaussians, 3.28M rays, the benchmark
    launch); the oracle checks two seeded whole views (131,072 rays, every
    64-ray packet of them complete) one ray at a time."""
    p = CT_CONE_50K
    sc = preset_scene(p)
    o, d = G.rays32(p["geom"])
    I = gpu_project(gr, sc, o, d)
    per = o.shape[1] // int(p["geom"]["n_views"])
    views = np.sort(np.random.default_rng(4).choice(int(p["geom"]["n_views"]), 2, replace=False))
    idx = np.concatenate([np.arange(v * per, (v + 1) * per) for v in views])
    ref = oracle.project(sc, o[:, idx], d[:, idx])
    worst = assert_forward(I[idx], ref, what=f"ct_cone_50k views {views.tolist()}")
    print(f"max rel err {worst:.2e} on views {views.tolist()}, pairs {int(ref['hits'].sum())}")
    assert np.isfinite(I).all() and (I >= 0).all()


def test_batched_equals_single(gr):
    """Two scenes and three segments in one launch equal separate launches."""
    import torch
    s1 = sample_scene(500, seed=21, radius=50.0, scale_range=(1.0, 6.0))
    s2 = sample_scene(900, seed=22, radius=70.0, scale_range=(0.5, 4.0))
    g = dict(CT_CONE_50K["geom"], n_views=2, nu=32, nv=30, pitch_u=8.0, pitch_v=8.0)
    o, d = G.rays32(g)
    m = o.shape[1]
    S1, S2 = dev_scene(gr, s1), dev_scene(gr, s2)
    ro, rd = to_dev(o), to_dev(d)
    a = gr.project(S1, ro, rd)
    b = gr.project(S2, ro, rd)
    out = torch.full((3 * m,), -1.0, device="cuda")
    ro2, rd2 = ro[:, 50:].contiguous(), rd[:, 50:].contiguous()   # a second, separate ray array
    out2 = torch.full((1000,), -1.0, device="cuda")
    gr.project_batched([S1, S2], [(0, ro, rd, 0, m, out, 0), (1, ro, rd, 0, m, out, m),
                                  (0, ro, rd, 100, 777, out, 2 * m), (1, ro2, rd2, 3, 500, out2, 10)])
    torch.cuda.synchronize()
    assert torch.equal(out[:m], a)
    assert torch.equal(out[m:2 * m], b)
    c = gr.project(S1, ro[:, 100:877].contiguous(), rd[:, 100:877].contiguous())
    assert torch.equal(out[2 * m:2 * m + 777], c)
    assert torch.all(out[2 * m + 777:] == -1.0)
    e = gr.project(S2, ro2[:, 3:503].contiguous(), rd2[:, 3:503].contiguous())
    assert torch.equal(out2[10:510], e) and torch.all(out2[:10] == -1) and torch.all(out2[510:] == -1)


def test_launch_options_do_not_change_results(gr):
    sc = sample_scene(3000, seed=12, radius=80.0, scale_range=(1.0, 7.0))
    g = dict(CT_CONE_50K["geom"], n_views=2, nu=40, nv=40, pitch_u=8.0, pitch_v=8.0)
    o, d = G.rays32(g)
    base = gpu_project(gr, sc, o, d)
    for w, x in ((1, 2), (2, 1), (8, 1), (16, 2)):
        assert np.array_equal(gpu_project(gr, sc, o, d, waves_per_group=w, xcd_remap=x), base)
    # the binary traversal visits the same pairs in another order (FP64 sum)
    bin_ = gpu_project(gr, sc, o, d, traversal=1)
    assert np.allclose(bin_, base, rtol=1e-6, atol=0)


def test_work_counters_match_oracle_hits(gr):
    """gr_project_stats: same projection as gr_project, and its included-pair
    count lies between the oracle's counts at kappa^2 (1 -+ 1e-5)."""
    import torch
    p = CT_PARALLEL_SMALL
    sc = preset_scene(p)
    o, d = G.rays32(p["geom"])
    S = dev_scene(gr, sc)
    ro, rd = to_dev(o), to_dev(d)
    a = gr.project(S, ro, rd)
    b, st = gr.project_stats(S, ro, rd)
    assert torch.equal(a, b)
    lo = int(oracle.project(sc, o, d, kappa=3.0 * math.sqrt(1 - 1e-5))["hits"].sum())
    hi = int(oracle.project(sc, o, d, kappa=3.0 * math.sqrt(1 + 1e-5))["hits"].sum())
    assert lo <= st["pairs"] <= hi
    assert st["packets"] == (o.shape[1] + 63) // 64
    assert st["pairs"] <= st["evaluated"]
    # both traversals are conservative, so they include exactly the same pairs
    _, st1 = gr.project_stats(S, ro, rd, traversal=1)
    assert st1["pairs"] == st["pairs"]
    print(f"binary traversal: evaluated {st1['evaluated']} leaves/packet {st1['leaves'] / st1['packets']:.1f}")
    print(f"pairs {st['pairs']} evaluated {st['evaluated']} utilisation "
          f"{st['pairs'] / st['evaluated']:.3f} leaves/packet {st['leaves'] / st['packets']:.1f}")


def test_persistent_and_per_view_launches_equal(gr):
    """The persistent launch (waves pulling packets from a counter) and one
    launch per view give bitwise the same forward as the single grid launch
    over all views (the packets are identical); the backward agrees to FP32
    atomic-order rounding."""
    import torch
    sc = sample_scene(3000, seed=13, radius=80.0, scale_range=(1.0, 7.0))
    g = dict(CT_CONE_50K["geom"], n_views=4, nu=48, nv=48, pitch_u=8.0, pitch_v=8.0)
    o, d = G.rays32(g)
    S = dev_scene(gr, sc)
    ro, rd = to_dev(o), to_dev(d)
    base = gr.project(S, ro, rd)
    for w in (1, 2, 4):
        assert torch.equal(gr.project(S, ro, rd, persistent=True, waves_per_group=w), base)
    assert torch.equal(gr.project(S, ro, rd, persistent=7), base)   # few groups, many packets each
    per = 48 * 48
    views = [gr.project(S, ro[:, v * per:(v + 1) * per].contiguous(), rd[:, v * per:(v + 1) * per].contiguous())
             for v in range(4)]
    assert torch.equal(torch.cat(views), base)
    w = to_dev(np.random.default_rng(0).uniform(-1, 1, o.shape[1]).astype(np.float32))
    g1 = gr.project_backward(S, ro, rd, w)
    g2 = gr.project_backward(S, ro, rd, w, persistent=True, waves_per_group=2)
    for k in g1:
        assert torch.allclose(g1[k], g2[k], rtol=1e-5, atol=1e-6 * float(g1[k].abs().max()))
    assert S.status_flags() == 0


def test_autotuner_small_search(gr, tmp_path, monkeypatch):
    monkeypatch.setenv("GR_TUNE_CACHE", str(tmp_path / "tune.json"))
    import importlib
    import paper_2602_01057_amd.tune as tune
    tune = importlib.reload(tune)
    sc = sample_scene(2000, seed=14, radius=80.0, scale_range=(1.0, 7.0))
    params = [to_dev(a) for a in (sc.mean, sc.scale, sc.quat, sc.density)]
    g = dict(CT_CONE_50K["geom"], n_views=3, nu=64, nv=64, pitch_u=6.0, pitch_v=6.0)
    best = tune.tune(params, g, op="fwd", search={"leaf": [32, 64], "waves": [1, 2], "tile": [[8, 8], [16, 4]]})
    assert best["ms"] > 0 and best["leaf"] in (32, 64)
    import torch
    assert tune.lookup(torch.device("cuda:0"), "ct", "fwd", 2000, 3 * 64 * 64)["leaf"] == best["leaf"]
    best_b = tune.tune(params, g, op="bwd", search={"leaf": [64], "waves": [1], "remap": [1], "tile": [[8, 8]]})
    assert best_b["ms"] > 0
