"""The continuous-batching server on the GPU: every result is the same alone
and in the mix (forward bit for bit, since each request's packets are those of
a stand-alone launch; gradients to FP32 atomic-order rounding), and served
forward and gradient results match the FP64 oracle."""
import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_2602_01057_amd.inputs import CT_CONE_500K, PET_200K, preset_scene
from parity import assert_forward, assert_grad, gpu_grad_rows

pytestmark = pytest.mark.gpu


def test_results_alone_equal_results_in_the_mix(gr):
    import torch
    from paper_2602_01057_amd import serve
    dev = torch.device("cuda:0")
    scenes = {}
    for k, (preset, n) in enumerate([(CT_CONE_500K, 20_000), (CT_CONE_500K, 5_000), (PET_200K, 15_000)]):
        sc = preset_scene(preset, seed=200 + k, n=n)
        scenes[k] = gr.Scene(*[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                               (sc.mean, sc.scale, sc.quat, sc.density)])
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(30):
        grad = i % 5 == 4
        if i % 2 == 0:
            n = int(rng.choice([64, 96, 128]))
            g = dict(CT_CONE_500K["geom"], nu=n, nv=n, pitch_u=409.6 / n, pitch_v=409.6 / n,
                     n_views=int(rng.integers(1, 6)), angle0=float(rng.uniform(0, 6.28)))
            reqs.append(serve.Request(int(rng.integers(0, 2)), g, kind="gradient" if grad else "forward",
                                      target_seed=i))
        else:
            planes = np.array([[3, 5], [10, 10], [20, 18]][: int(rng.integers(1, 4))], dtype=np.int32)
            g = dict(PET_200K["geom"], planes=planes, n_views=24)
            reqs.append(serve.Request(2, g, kind="gradient" if grad else "forward", loss="poisson",
                                      background=0.05, target_seed=i))
    ex = serve.GpuExecutor(scenes, n_streams=2, keep_rays=True)
    sched = serve.Scheduler(ex, hbm_budget=1e9, n_streams=2, tick_rays=100_000)
    srv = serve.Server(sched).start()
    futs = [srv.submit(r) for r in reqs]
    srv.drain(120)
    srv.stop()
    assert all(f.exception() is None for f in futs)
    assert max(len(t) for t in [reqs]) == 30
    for r, f in zip(reqs, futs):
        ro, rd = r.state["ro"], r.state["rd"]
        sc = scenes[r.scene_id]
        if r.kind == "forward":
            alone = gr.project(sc, ro, rd)
            torch.cuda.synchronize()
            assert torch.equal(f.result(), alone), r.rid
        else:
            res = f.result()
            proj = torch.empty_like(res["proj"])
            loss = torch.zeros(1, dtype=torch.float64, device=dev)
            g = gr.project_backward(sc, ro, rd, loss=r.loss, target=r.state["target"],
                                    background=r.background, out_proj=proj, out_loss=loss)
            torch.cuda.synchronize()
            assert torch.equal(res["proj"], proj), r.rid
            assert abs(res["loss"].item() - loss.item()) <= 1e-12 * abs(loss.item()), r.rid
            for k in g:
                assert float((g[k] - res["grads"][k]).norm()) <= 1e-5 * float(g[k].norm()) + 1e-30, k
    st = sched.latency_stats()
    assert st["n"] == 30 and st["p99_s"] >= st["p50_s"] > 0
    for s in scenes.values():
        assert s.status_flags() == 0


def test_served_results_match_the_oracle(gr):
    """Seeded mix of forward and gradient requests (CT and PET, L2 and
    Poisson) served with a small tick, so that gradient requests are cut into
    chunks and batched with others; every served projection is checked ray by
    ray, every served loss value, and the gradients of 16 seeded Gaussians per
    gradient request, against the FP64 oracle. Requests carry the oracle's FP32
    rays, so both sides integrate along the same lines."""
    import torch
    from paper_2602_01057_amd import serve
    dev = torch.device("cuda:0")
    host, scenes = {}, {}
    for k, (preset, n) in enumerate([(CT_CONE_500K, 4000), (CT_CONE_500K, 2500), (PET_200K, 3000)]):
        sc = preset_scene(preset, seed=300 + k, n=n)
        host[k] = sc
        scenes[k] = gr.Scene(*[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                               (sc.mean, sc.scale, sc.quat, sc.density)])
    rng = np.random.default_rng(21)
    reqs, refs = [], []
    for i in range(10):
        grad = i % 3 != 0
        if i % 2 == 0:
            n = int(rng.choice([64, 96]))
            g = dict(CT_CONE_500K["geom"], nu=n, nv=n, pitch_u=409.6 / n, pitch_v=409.6 / n,
                     n_views=int(rng.integers(1, 4)), angle0=float(rng.uniform(0, 6.28)))
            sid, loss, bg = int(rng.integers(0, 2)), "l2", 0.0
        else:
            planes = np.array([[3, 5], [10, 10], [20, 18]][: int(rng.integers(1, 3))], dtype=np.int32)
            g = dict(PET_200K["geom"], planes=planes, n_views=12)
            sid, loss, bg = 2, "poisson", 0.05
        o, d = G.rays32(g)
        ref = oracle.project(host[sid], o, d)
        req = serve.Request(sid, g, kind="gradient" if grad else "forward", loss=loss, background=bg,
                            rays=(o, d))
        if grad:
            m = o.shape[1]
            if loss == "l2":
                # targets a seeded distance away from the oracle's projection
                u = rng.uniform(0.5, 1.5, m) * rng.choice([-1.0, 1.0], m) * max(1e-3, float(ref["I_kappa"].mean()))
                req.target = (ref["I_kappa"] + u).astype(np.float32)
            else:
                req.target = rng.poisson(5.0 * ref["I_kappa"] + 1.0).astype(np.float32)
        reqs.append(req)
        refs.append((o, d, ref))
    ex = serve.GpuExecutor(scenes, n_streams=2)
    sched = serve.Scheduler(ex, hbm_budget=1e9, n_streams=2, tick_rays=8192)
    srv = serve.Server(sched).start()
    futs = [srv.submit(r) for r in reqs]
    srv.drain(120)
    srv.stop()
    assert all(f.exception() is None for f in futs)
    chunked = 0
    for r, f, (o, d, ref) in zip(reqs, futs, refs):
        sc = host[r.scene_id]
        if r.kind == "forward":
            assert_forward(f.result().cpu().numpy(), ref, what=f"served forward {r.rid}")
            continue
        res = f.result()
        assert_forward(res["proj"].cpu().numpy(), ref, what=f"served gradient request {r.rid} projection")
        y = np.asarray(r.target, np.float64)
        L_ref, w_ref = oracle.loss_weights(r.loss, ref["I_kappa"], y, r.background)
        assert abs(res["loss"].item() - L_ref) <= 1e-4 * abs(L_ref), (r.rid, res["loss"].item(), L_ref)
        sel = np.sort(np.random.default_rng(100 + r.rid).choice(sc.n, 16, replace=False))
        gref = oracle.grad(sc, o, d, w_ref, sel=sel)
        assert_grad(gpu_grad_rows(res["grads"], sel), gref, what=f"served gradient request {r.rid}")
        chunked += int(r.n_rays * serve.GRAD_COST > 8192)
    assert chunked >= 2   # gradient requests were cut into several ticks
    for s in scenes.values():
        assert s.status_flags() == 0
