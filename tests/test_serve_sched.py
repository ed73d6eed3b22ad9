"""Scheduler of the continuous-batching server, driven on the CPU with a fake
executor and a simulated clock (no GPU)."""
import numpy as np
import pytest

from paper_2602_01057_amd.serve import PACKET, Request, Scheduler, mixed_stream


class FakeExecutor:
    """Each tick takes 1 us per 1000 rays (+20 us) of simulated time."""

    def __init__(self, fail_scene=None):
        self.now = 0.0
        self.launches = []   # (stream, [(rid, first, count)], [rid], t_start, t_end)
        self.fail_scene = fail_scene
        self.setups = []

    def ray_count(self, req):
        return int(req.geom["n_rays"])

    def request_bytes(self, req):
        return 28 * self.ray_count(req) + (1000 if req.kind == "gradient" else 0)

    def setup(self, req):
        self.setups.append((req.rid, self.now))
        req.state = {"covered": []}

    def launch(self, s, segs):
        rays = sum(c * (2 if r.kind == "gradient" else 1) for r, _, c in segs)
        t_end = self.now + 20e-6 + rays * 1e-9
        err = None
        for r, a, c in segs:
            assert 0 <= a and c > 0 and a + c <= r.n_rays, (a, c, r.n_rays)
            r.state["covered"].append((a, c))
            if r.scene_id == self.fail_scene:
                err = RuntimeError("injected device failure")
        self.launches.append((s, [(r.rid, a, c) for r, a, c in segs],
                              [r.rid for r, _, _ in segs if r.kind == "gradient"], self.now, t_end))
        return {"t_end": t_end, "err": err}

    def done(self, h, now):
        return now >= h["t_end"]

    def error(self, h):
        return h["err"]

    def result(self, req):
        return list(req.state["covered"])

    def release(self, req):
        pass


def run(sched, ex, arrivals, dt=5e-6, t_max=10.0):
    """arrivals: [(t, Request)]; advance the simulated clock until idle."""
    futs = []
    pending = sorted(arrivals, key=lambda x: x[0])
    t = 0.0
    while t < t_max:
        while pending and pending[0][0] <= t:
            futs.append(sched.submit(pending.pop(0)[1], t))
        ex.now = t
        busy = sched.step(t)
        if not busy and not pending:
            break
        t += dt
    return futs


def req(n, scene=0, kind="forward"):
    return Request(scene, {"n_rays": n}, kind=kind)


def test_single_request_and_latency():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e9)
    (f,) = run(s, ex, [(0.0, req(1000))])
    assert f.result() == [(0, 1000)]
    st = s.latency_stats()
    assert st["n"] == 1 and 20e-6 <= st["p50_s"] <= 100e-6


def test_chunks_are_whole_packets_and_cover_every_ray_once():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12, tick_rays=1000)
    (f,) = run(s, ex, [(0.0, req(10_000 + 37))])
    cov = f.result()
    assert len(cov) > 5
    pos = 0
    for a, c in cov:
        assert a == pos and a % PACKET == 0
        pos += c
    assert pos == 10_037
    assert all(c % PACKET == 0 for _, c in cov[:-1])


def _assert_tiled(result, n):
    pos = 0
    for a, c in result:
        assert a == pos and a % PACKET == 0 and c > 0
        pos += c
    assert pos == n


def test_short_remainders_and_small_leftover_budgets_stay_inside_each_request():
    """Chunks are whole packets from the request's start and never reach past
    its end, also when fewer than 64 rays are left and the tick's leftover
    budget is smaller still (the fake executor asserts the bounds of every
    chunk it is handed). Sizes include PET-like 64 k + 32 ray requests."""
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12, n_streams=1, tick_rays=1024)
    futs = run(s, ex, [(0.0, req(994)), (0.0, req(50))])
    _assert_tiled(futs[0].result(), 994)
    _assert_tiled(futs[1].result(), 50)
    rng = np.random.default_rng(12)
    for trial in range(20):
        ex = FakeExecutor()
        s = Scheduler(ex, hbm_budget=1e12, n_streams=int(rng.integers(1, 3)),
                      tick_rays=int(rng.choice([64, 100, 1000, 1024, 4096])))
        sizes = [int(x) for x in rng.integers(1, 5000, 12)] + [64 * 7 + 32, 31, 64]
        kinds = ["gradient" if rng.uniform() < 0.3 else "forward" for _ in sizes]
        arr = [(float(rng.uniform(0, 2e-4)), req(n, scene=int(rng.integers(0, 10)), kind=k))
               for n, k in zip(sizes, kinds)]
        futs = run(s, ex, arr)
        for f, (_, r) in zip(futs, sorted(arr, key=lambda x: x[0])):
            _assert_tiled(f.result(), r.n_rays)


def test_gradient_requests_are_chunked_and_share_ticks():
    """Gradient work is cut into whole packets like forward work (each ray
    counting double against the tick's budget), so a long gradient request
    shares ticks with requests that arrive after it."""
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12, n_streams=1, tick_rays=2048)
    futs = run(s, ex, [(0.0, req(10_000, kind="gradient")), (50e-6, req(500)),
                       (60e-6, req(3000, scene=2, kind="gradient"))])
    cov = futs[0].result()
    assert len(cov) > 5
    pos = 0
    for a, c in cov:
        assert a == pos and a % PACKET == 0 and c <= 1024
        pos += c
    assert pos == 10_000
    assert sum(c for _, c in futs[1].result()) == 500 and sum(c for _, c in futs[2].result()) == 3000
    mixed = [segs for _, segs, grads, _, _ in ex.launches if len({rid for rid, _, _ in segs}) > 1 and grads]
    assert mixed
    done = {r.rid: r for r in s.done}
    assert done[1].t_done < done[0].t_done     # the short forward request did not wait for the long one


def test_admission_waits_for_budget_and_rejects_oversize():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=28 * 1500)     # room for one 1000-ray request at a time
    futs = run(s, ex, [(0.0, req(1000)), (0.0, req(1000)), (0.0, req(100_000))])
    assert isinstance(futs[2].exception(), MemoryError)
    done = {r.rid: r for r in s.done}
    assert done[1].t_admit >= done[0].t_done      # second admitted only after the first released
    assert s.used == 0


def test_slots_limit_active_requests():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12, max_slots=2)
    peak = 0
    arrivals = [(0.0, req(5000)) for _ in range(6)]
    pending = list(arrivals)
    t = 0.0
    futs = []
    while True:
        while pending and pending[0][0] <= t:
            futs.append(s.submit(pending.pop(0)[1], t))
        ex.now = t
        busy = s.step(t)
        peak = max(peak, len(s.active))
        if not busy and not pending:
            break
        t += 5e-6
    assert peak == 2 and all(f.done() for f in futs)


def test_continuous_batching_overlaps_streams_and_joins_new_arrivals():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12, n_streams=2, tick_rays=2000)
    arrivals = [(0.0, req(20_000, scene=0)), (0.0, req(20_000, scene=1)),
                (30e-6, req(3000, scene=2)), (31e-6, req(3000, scene=3))]
    futs = run(s, ex, arrivals)
    assert all(f.done() and f.exception() is None for f in futs)
    # ticks on the two streams overlapped in time
    by_stream = {0: [], 1: []}
    for st, segs, grads, t0, t1 in ex.launches:
        by_stream[st].append((t0, t1))
    assert any(a0 < b1 and b0 < a1 for a0, a1 in by_stream[0] for b0, b1 in by_stream[1])
    # a late arrival shared a tick with an earlier, still running request
    shared = [segs for _, segs, _, _, _ in ex.launches if len({rid for rid, _, _ in segs}) > 1]
    assert shared


def test_gradient_requests_and_failure_isolation():
    ex = FakeExecutor(fail_scene=7)
    s = Scheduler(ex, hbm_budget=1e12, n_streams=1)
    # a failed launch fails the requests of its tick; the loop keeps serving
    futs = run(s, ex, [(0.0, req(500, kind="gradient")), (1e-3, req(700, scene=7)),
                       (2e-3, req(300))])
    assert futs[0].result() == [(0, 500)]
    assert isinstance(futs[1].exception(), RuntimeError)
    assert futs[2].result() == [(0, 300)]      # the server kept serving after the failure
    assert s.used == 0 and not s.active


def test_poisson_arrivals_on_a_simulated_clock():
    rng = np.random.default_rng(5)
    t = 0.0
    arrivals = []
    for _ in range(200):
        t += float(rng.exponential(1 / 50.0))
        arrivals.append((t, req(int(rng.integers(1000, 200_000)))))
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=200e9)
    futs = run(s, ex, arrivals, dt=1e-4, t_max=100.0)
    assert all(f.done() for f in futs)
    st = s.latency_stats()
    assert st["n"] == 200 and 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]


def test_mixed_stream_is_seeded():
    a = mixed_stream(50, 50.0, 5, [0, 1], [2])
    b = mixed_stream(50, 50.0, 5, [0, 1], [2])
    assert [(t, r.scene_id, r.kind, r.geom["kind"]) for t, r in a] == \
           [(t, r.scene_id, r.kind, r.geom["kind"]) for t, r in b]
    kinds = [r.geom["kind"] for _, r in a]
    assert 10 < kinds.count("ct") < 40
    grads = sum(r.kind == "gradient" for _, r in a)
    assert 5 < grads < 30
    ts = [t for t, _ in a]
    assert all(x < y for x, y in zip(ts, ts[1:]))


def test_requests_with_array_fields_and_scheduler_fault():
    """Requests compare by identity (geometry dicts may hold arrays), and a
    fault inside a scheduling step fails the admitted requests without
    stopping the loop."""
    from paper_2602_01057_amd.serve import Server
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1e12)
    a = Request(0, {"n_rays": 100, "planes": np.zeros((3, 2))})
    b = Request(0, {"n_rays": 100, "planes": np.zeros((2, 2))})
    futs = run(s, ex, [(0.0, a), (0.0, b)])
    assert all(f.result() for f in futs)
    s2 = Scheduler(ex, hbm_budget=1e12)
    srv = Server(s2)
    bad = Request(0, {"n_rays": 100})
    f = s2.submit(bad, 0.0)
    s2._admit(0.0)
    s2.fail_all(RuntimeError("boom"))
    assert isinstance(f.exception(), RuntimeError) and not s2.active
    del srv


def test_a_stalled_drain_names_what_it_waits_for():
    """A tick that never completes (an executor whose work does not finish)
    makes the threaded server's drain report the scheduler's state while it
    waits and raise with it at the deadline, instead of waiting silently."""
    import time

    from paper_2602_01057_amd.serve import Server

    class Stuck(FakeExecutor):
        def done(self, h, now):
            return False

    ex = Stuck()
    sched = Scheduler(ex, hbm_budget=1e9, n_streams=2, tick_rays=1024)
    srv = Server(sched).start()
    futs = [srv.submit(Request(0, {"n_rays": n})) for n in (100, 5000)]
    logs = []
    t0 = time.perf_counter()
    with pytest.raises(TimeoutError) as e:
        srv.drain(0.5, progress=logs.append, progress_every=0.1)
    srv.stop()
    assert time.perf_counter() - t0 < 5.0
    msg = str(e.value)
    assert "in flight 2" in msg and "stream 0" in msg and "stream 1" in msg, msg
    assert "active 2" in msg and "0 done" in msg, msg
    assert logs and all("draining for" in m for m in logs)
    assert not any(f.done() for f in futs)
