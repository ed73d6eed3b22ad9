"""The continuous-batching server on the GPU: every result is the same alone
and in the mix (forward bit for bit, since each request's packets are those of
a stand-alone launch; gradients to FP32 atomic-order rounding)."""
import numpy as np
import pytest

from paper_2602_01057_amd.inputs import CT_CONE_500K, PET_200K, preset_scene

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
            g = gr.project_backward(sc, ro, rd, loss=r.loss, target=r.state["target"],
                                    background=r.background)
            torch.cuda.synchronize()
            for k in g:
                assert float((g[k] - res["grads"][k]).norm()) <= 1e-5 * float(g[k].norm()) + 1e-30, k
    st = sched.latency_stats()
    assert st["n"] == 30 and st["p99_s"] >= st["p50_s"] > 0
    for s in scenes.values():
        assert s.status_flags() == 0
