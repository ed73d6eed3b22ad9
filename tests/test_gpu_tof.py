"""Time-of-flight / attenuation projector on the GPU against the FP64 oracle
(the extensions the paper names as future work, Sec. 5): forward per (bin,
ray), gradient, TOF centres of PET lines, loss weights with per-element
randoms + scatter, and one TOF training step through the library only."""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_2602_01057_amd.inputs import PET_200K, preset_scene, sample_scene
from parity import FWD_TOL, assert_grad, gpu_grad_rows

pytestmark = pytest.mark.gpu

# a small cylindrical scanner: 96 crystals x 8 rings, radius 120 mm
SMALL_PET = dict(kind="pet", ring_radius=120.0, ring_pitch=4.0, n_crystals=96, n_rings=8, n_radial=40,
                 n_views=48, max_ring_diff=7, arc_correct=1, tile_radial=8, tile_axial=8)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def f32(x):
    return float(np.float32(x))


def dev_scene(gr, sc, leaf=0):
    S = gr.Scene(to_dev(sc.mean), to_dev(sc.scale), to_dev(sc.quat), to_dev(sc.density), leaf_size=leaf)
    assert S.status_flags() == 0
    return S


def small_problem(seed=61, n=400, nsub=6000):
    sc = sample_scene(n, seed=seed, region="cylinder", radius=70.0, length=28.0, scale_range=(1.0, 7.0))
    idx = np.sort(np.random.default_rng(seed + 1).choice(G.count(SMALL_PET), nsub, replace=False))
    o, d = G.rays32(SMALL_PET, idx)
    c = G.pet_tof_centers64(SMALL_PET, idx).astype(np.float32)
    a = np.random.default_rng(seed + 2).uniform(0.05, 1.0, o.shape[1]).astype(np.float32)
    return sc, o, d, c, a


# FP32's smallest normal number: a true value below it may come out as 0 or as
# a subnormal, so an absolute slack of this size covers the flush and nothing
# more (every normal value keeps the relative bar)
TINY = float(np.finfo(np.float32).tiny)


def assert_bins(I_gpu, ref, what):
    """Each (bin, ray) within [I_in (1 - tol), I_hi (1 + tol)] widened by
    TINY; exactly 0 where nothing is in reach."""
    I = np.asarray(I_gpu, np.float64)
    lo = ref["I_in"] * (1 - FWD_TOL) - TINY
    hi = ref["I_hi"] * (1 + FWD_TOL) + TINY
    bad = (I < lo) | (I > hi) | ((ref["I_hi"] == 0) & (I != 0))
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {I.size} outside; e.g. gpu {I[bad][:4]} "
                           f"ref {ref['I_kappa'][bad][:4]}")
    nz = ref["I_kappa"] > 0
    return float((np.abs(I[nz] - ref["I_kappa"][nz]) / ref["I_kappa"][nz]).max()) if nz.any() else 0.0


@pytest.mark.parametrize("n_bins,sigma,width,leaf", [(0, 0, 0, 16), (1, 30.0, 25.0, 16), (13, 25.0, 12.0, 64),
                                                     (9, 8.0, 6.0, 1), (32, 20.0, 6.5, 16), (32, 0.6, 1.5, 16),
                                                     (16, 40.0, 25.0, 64), (5, 10.0, 8.0, 16), (17, 22.0, 9.0, 64)])
def test_tof_forward_matches_oracle(gr, n_bins, sigma, width, leaf):
    sc, o, d, c, a = small_problem()
    S = dev_scene(gr, sc, leaf)
    out = gr.project_tof(S, to_dev(o), to_dev(d), n_bins, sigma, width, center=to_dev(c), atten=to_dev(a))
    ref = oracle.project_tof(sc, o, d, n_bins, f32(sigma), f32(width), center=c, atten=a)
    worst = assert_bins(out.cpu().numpy(), ref, f"{n_bins} bins")
    assert S.status_flags() == 0
    print(f"{n_bins} bins x {o.shape[1]} lines: max rel err {worst:.2e}")


def test_tof_bins_sum_to_the_plain_projection(gr):
    """Bins spaced at most 2 sigma apart covering the scanner sum to the
    attenuated non-TOF projection (up to the bins' FP32 rounding)."""
    import torch
    sc, o, d, c, a = small_problem(n=300)
    S = dev_scene(gr, sc)
    nb, sigma, width = 25, 14.0, 11.0  # +-138 mm around the centre
    tof = gr.project_tof(S, to_dev(o), to_dev(d), nb, sigma, width, center=to_dev(c), atten=to_dev(a))
    plain = gr.project(S, to_dev(o), to_dev(d))
    s = tof.double().sum(dim=0)
    ref = plain.double() * to_dev(a).double()
    assert torch.allclose(s, ref, rtol=3e-5, atol=1e-30)


@pytest.mark.parametrize("n_bins,sigma,width", [(0, 0, 0), (13, 25.0, 12.0), (32, 20.0, 6.5), (2, 30.0, 20.0),
                                                (17, 22.0, 9.0), (24, 0.8, 2.0)])
def test_tof_backward_matches_oracle(gr, n_bins, sigma, width):
    import torch
    sc, o, d, c, a = small_problem(n=250, nsub=3000)
    S = dev_scene(gr, sc)
    nb = max(1, n_bins)
    w = np.random.default_rng(62).uniform(-1, 1, (nb, o.shape[1])).astype(np.float32)
    w[:, ::7] = 0.0  # rays with no weight
    grads = gr.project_tof_backward(S, to_dev(o), to_dev(d), to_dev(w), n_bins, sigma, width,
                                    center=to_dev(c), atten=to_dev(a))
    torch.cuda.synchronize()
    ref = oracle.grad_tof(sc, o, d, w.astype(np.float64), n_bins, f32(sigma), f32(width), center=c, atten=a)
    worst = assert_grad(gpu_grad_rows(grads, np.arange(sc.n)), ref, what=f"tof {n_bins} bins")
    print(f"worst normwise rel err {worst:.2e}")


def test_tof_training_step_poisson_with_randoms(gr):
    """Forward TOF -> Poisson loss weights with per-bin randoms + scatter ->
    TOF backward, all in the library, against the oracle computing the same
    chain from its own projection."""
    import torch
    sc, o, d, c, a = small_problem(n=250, nsub=3000)
    tgt = sample_scene(250, seed=63, region="cylinder", radius=70.0, length=28.0, scale_range=(1.0, 7.0))
    nb, sigma, width = 13, 25.0, 12.0
    ref_t = oracle.project_tof(tgt, o, d, nb, f32(sigma), f32(width), center=c, atten=a)["I_kappa"]
    rng = np.random.default_rng(64)
    cscale = 40.0
    bg = (0.02 * cscale * rng.uniform(0.5, 1.5, ref_t.shape) * ref_t.mean()).astype(np.float32)
    y = rng.poisson(cscale * ref_t + bg).astype(np.float32)
    scc = type(sc)(sc.mean, sc.scale, sc.quat, (cscale * sc.density).astype(np.float32))
    S = dev_scene(gr, scc)
    ro, rd, ct, at = to_dev(o), to_dev(d), to_dev(c), to_dev(a)
    I = gr.project_tof(S, ro, rd, nb, sigma, width, center=ct, atten=at)
    wgt, loss = gr.loss_weights("poisson", I, to_dev(y), background=to_dev(bg))
    grads = gr.project_tof_backward(S, ro, rd, wgt, nb, sigma, width, center=ct, atten=at)
    torch.cuda.synchronize()
    I_ref = oracle.project_tof(scc, o, d, nb, f32(sigma), f32(width), center=c, atten=a)["I_kappa"]
    L_ref, w_ref = oracle.loss_weights("poisson", I_ref, y, bg)
    assert abs(loss.item() - L_ref) <= 1e-5 * abs(L_ref) + 1e-3
    ref = oracle.grad_tof(scc, o, d, w_ref, nb, f32(sigma), f32(width), center=c, atten=a)
    worst = assert_grad(gpu_grad_rows(grads, np.arange(sc.n)), ref, what="tof poisson step")
    print(f"loss {loss.item():.6g} (oracle {L_ref:.6g}); worst normwise rel err {worst:.2e}")


def test_loss_weights_match_oracle(gr):
    rng = np.random.default_rng(65)
    m = 10_000
    I = rng.uniform(0.0, 20.0, m).astype(np.float32)
    y = rng.poisson(8.0, m).astype(np.float32)
    bg = rng.uniform(0.05, 1.0, m).astype(np.float32)
    for kind, b in (("l2", 0.0), ("poisson", 0.3), ("poisson", bg)):
        w, loss = gr.loss_weights(kind, to_dev(I), to_dev(y), to_dev(b) if isinstance(b, np.ndarray) else b)
        L_ref, w_ref = oracle.loss_weights(kind, I, y, np.float32(b) if not isinstance(b, np.ndarray) else b)
        assert np.allclose(w.cpu().numpy(), w_ref, rtol=2e-7, atol=1e-6)
        assert abs(loss.item() - L_ref) <= 1e-9 * abs(L_ref)


def test_tof_centres_match_oracle_geometry(gr):
    import torch
    for g in (SMALL_PET, dict(SMALL_PET, arc_correct=0), PET_200K["geom"]):
        m = G.count(g)
        idx = np.sort(np.random.default_rng(66).choice(m, min(m, 200_000), replace=False))
        o, d = G.rays32(g, idx)
        c = gr.tof_centers(to_dev(o), to_dev(d))
        ref = G.pet_tof_centers64(g, idx)
        # the FP32 rays move the closest approach by ~eps32 x radius
        assert np.abs(c.cpu().numpy() - ref).max() <= 2e-4
    z = torch.zeros(3, 0, device="cuda")
    assert gr.tof_centers(z, z).numel() == 0


def test_tof_edge_cases(gr):
    import torch
    sc, o, d, c, a = small_problem(n=100, nsub=200)
    S = dev_scene(gr, sc)
    z3 = torch.zeros(3, 0, device="cuda")
    assert gr.project_tof(S, z3, z3, 7, 20.0, 10.0).shape == (7, 0)
    e = type(sc)(np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32),
                 np.zeros(0, np.float32))
    E = dev_scene(gr, e)
    assert torch.all(gr.project_tof(E, to_dev(o), to_dev(d), 7, 20.0, 10.0) == 0)
    # all-zero weights give zero gradients; no centres and no attenuation = 0 and 1
    grads = gr.project_tof_backward(S, to_dev(o), to_dev(d), torch.zeros(7, o.shape[1], device="cuda"), 7, 20.0,
                                    10.0)
    assert all(float(v.abs().max()) == 0 for v in grads.values())
    out = gr.project_tof(S, to_dev(o), to_dev(d), 7, 20.0, 10.0)
    ref = oracle.project_tof(sc, o, d, 7, 20.0, 10.0)
    assert_bins(out.cpu().numpy(), ref, "no centre / attenuation")


def test_tof_full_size_pet_sampled(gr):
    """PET 200k Gaussians, the full 344 x 252 x 752 geometry with 13 TOF bins
    (sigma 25 mm, bins 12 mm), launched over all 65M lines like the
    projector's bench; 300 sampled lines checked against the oracle."""
    import torch
    from paper_2602_01057_amd.inputs import PET_200K as P
    sc = preset_scene(P)
    g = P["geom"]
    S = dev_scene(gr, sc, 64)
    m = gr.ray_count(g)
    ro = torch.empty(3, m, device="cuda")
    rd = torch.empty(3, m, device="cuda")
    gr.make_rays(g, "cuda", out=(ro, rd))
    ct = gr.tof_centers(ro, rd)
    # the sampled lines take the oracle geometry's FP32 rays and centres, so
    # that both sides see the same inputs inside the full-size launch
    idx = np.sort(np.random.default_rng(67).choice(m, 300, replace=False))
    o, d = G.rays32(g, idx)
    c = G.pet_tof_centers64(g, idx).astype(np.float32)
    ii = torch.from_numpy(idx).cuda()
    ro[:, ii] = to_dev(o)
    rd[:, ii] = to_dev(d)
    ct[ii] = to_dev(c)
    nb = 13
    out = gr.project_tof(S, ro, rd, nb, 25.0, 12.0, center=ct)
    got = out[:, ii].cpu().numpy()
    assert S.status_flags() == 0
    del out
    ref = oracle.project_tof(sc, o, d, nb, 25.0, 12.0, center=c)
    worst = assert_bins(got, ref, "pet_200k tof sampled")
    print(f"max rel err {worst:.2e}")


def test_tof_launch_forms_agree(gr):
    """Binary-LBVH traversal, two waves per group and the persistent launch
    give the default launch's TOF bins (same pairs, summation order aside)."""
    import torch
    sc, o, d, c, a = small_problem(n=300, nsub=4000)
    S = dev_scene(gr, sc, 16)
    ro, rd, ct, at = to_dev(o), to_dev(d), to_dev(c), to_dev(a)
    ref = gr.project_tof(S, ro, rd, 13, 25.0, 12.0, center=ct, atten=at)
    for kw in ({"traversal": 1}, {"waves_per_group": 2}, {"persistent": True}, {"waves_per_group": 4, "persistent": 64}):
        out = gr.project_tof(S, ro, rd, 13, 25.0, 12.0, center=ct, atten=at, **kw)
        assert torch.allclose(out, ref, rtol=1e-6, atol=1e-30), kw
    w = torch.from_numpy(np.random.default_rng(68).uniform(-1, 1, (13, o.shape[1])).astype(np.float32)).cuda()
    g0 = gr.project_tof_backward(S, ro, rd, w, 13, 25.0, 12.0, center=ct, atten=at)
    g1 = gr.project_tof_backward(S, ro, rd, w, 13, 25.0, 12.0, center=ct, atten=at, traversal=1, persistent=True)
    for k in g0:
        assert float((g1[k] - g0[k]).norm()) <= 1e-5 * float(g0[k].norm()), k
    assert S.status_flags() == 0
