"""Continuous-batching request server for projection and gradient requests.

Requests name a resident scene (Gaussians + LBVH kept on the device) and a
scanner geometry (CT or PET). A host thread runs the scheduling loop:

  admission   a request is admitted when a slot is free and its device memory
              (rays, outputs, targets, gradient accumulators and gradients)
              fits the HBM budget next to the admitted ones; the fused pass's
              hit-list scratch is one buffer per stream, allocated when the
              executor starts;
  set-up      an admitted request gets its buffers and its rays (generated on
              the device) on one of the server's streams, which it keeps;
  ticks       every loop iteration, each stream with nothing in flight gets a
              tick: the pending work of its requests is cut into chunks of
              whole 64-ray packets up to the tick's budget (gradient rays
              count double: the fused pass costs about twice the forward),
              forward chunks go into ONE batched forward launch
              (gr_project_batched) and gradient chunks into ONE batched fused
              forward -> loss -> backward launch (gr_project_backward_batched,
              each chunk adding into its request's per-Gaussian sums); a
              gradient request's last chunk is followed by its epilogue
              (gr_backward_finish) on the same stream. Up to 32 chunks against
              up to 8 scenes share a launch. Chunks start at the request's
              packet boundaries, so the packets, and therefore the results,
              are those of a stand-alone launch (gradients up to the order of
              the FP32 atomics);
  completion  ticks complete through events; a finished request's future
              receives its output and its latency is recorded.

Requests arriving while ticks run join the next tick of some stream, so work
from different requests overlaps on the device (continuous batching, not a
queue in front of one launch at a time), and a long request no longer holds a
stream for its whole duration. The scheduler is separate from the executor:
tests drive it with a simulated clock and a fake executor on the CPU.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import math
import statistics
import threading
import time
from typing import Dict, List, Optional, Sequence

PACKET = 64
MAX_SEGMENTS = 32
MAX_SCENES = 8
GRAD_COST = 2  # tick budget per gradient ray, in forward rays


@dataclasses.dataclass(eq=False)  # requests compare by identity
class Request:
    scene_id: int
    geom: Dict
    kind: str = "forward"            # "forward" or "gradient"
    loss: str = "l2"                 # gradient requests: "l2" or "poisson"
    target: Optional[object] = None  # gradient requests: per-ray target / counts
    background: float = 0.0
    target_seed: int = 0             # seeds synthetic targets when target is None
    rays: Optional[object] = None    # (ray_o, ray_d) arrays of shape (3, m) given by the client,
                                     # used instead of rays generated from geom
    # set by the server
    rid: int = -1
    n_rays: int = 0
    bytes: int = 0
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    stream: int = -1
    next_ray: int = 0                # first ray not yet handed to a tick
    chunks_out: int = 0              # chunks launched and not yet complete
    future: Optional[cf.Future] = None
    state: object = None             # executor-owned buffers


@dataclasses.dataclass
class Tick:
    stream: int
    handle: object
    requests: List[Request]
    chunk_counts: Dict[int, int]
    t_launch: float = 0.0


class Scheduler:
    """Admission, chunking, tick formation and completion; no device calls."""

    def __init__(self, executor, hbm_budget: float = 200e9, max_slots: int = 64,
                 n_streams: int = 2, tick_rays: int = 4_000_000):
        if n_streams < 1:
            raise ValueError("need at least one stream")
        self.ex = executor
        self.budget = float(hbm_budget)
        self.max_slots = int(max_slots)
        self.n_streams = int(n_streams)
        self.tick_rays = max(PACKET, (int(tick_rays) // PACKET) * PACKET)
        self.queue: List[Request] = []
        self.active: List[Request] = []
        self.in_flight: List[Tick] = []
        self.used = 0.0
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self._next_id = 0
        self._lock = threading.Lock()

    # -- client side ---------------------------------------------------------
    def submit(self, req: Request, now: float) -> cf.Future:
        req.future = cf.Future()
        req.rid = self._next_id
        self._next_id += 1
        req.t_submit = now
        req.n_rays = self.ex.ray_count(req)
        req.bytes = self.ex.request_bytes(req)
        if req.bytes > self.budget:
            req.future.set_exception(MemoryError(
                f"request needs {req.bytes} B of device memory, budget is {self.budget:.0f} B"))
            self.rejected.append(req)
            return req.future
        with self._lock:
            self.queue.append(req)
        return req.future

    # -- one scheduling iteration ------------------------------------------------
    def step(self, now: float) -> bool:
        """Admit, launch and complete what is possible at time ``now``.
        Returns True if anything is queued, active or in flight."""
        self._complete(now)
        self._admit(now)
        self._launch()
        return bool(self.queue or self.active or self.in_flight)

    def _admit(self, now: float) -> None:
        with self._lock:
            waiting = list(self.queue)
        for req in waiting:
            if len(self.active) >= self.max_slots or self.used + req.bytes > self.budget:
                break  # first come, first served: later requests wait behind this one
            with self._lock:
                self.queue.remove(req)
            req.t_admit = now
            req.stream = req.rid % self.n_streams
            try:
                self.ex.setup(req)
            except Exception as e:  # device errors become per-request failures
                req.future.set_exception(e)
                self.rejected.append(req)
                continue
            self.used += req.bytes
            self.active.append(req)

    def _launch(self) -> None:
        busy = {t.stream for t in self.in_flight}
        for s in range(self.n_streams):
            if s in busy:
                continue
            reqs = [r for r in self.active if r.stream == s and r.next_ray < r.n_rays]
            if not reqs:
                continue
            # Shortest remaining work first (small requests finish in one or two
            # ticks instead of queueing behind long ones), except that the
            # oldest request is first given a quarter of the tick, so that no
            # request starves under load.
            oldest = min(reqs, key=lambda r: r.rid)

            def cost(r):
                return GRAD_COST if r.kind == "gradient" else 1

            order = [oldest] + sorted(reqs, key=lambda r: ((r.n_rays - r.next_ray) * cost(r), r.rid))
            take_of: Dict[int, int] = {}
            used_scenes: List[int] = []
            budget = self.tick_rays
            for k, r in enumerate(order):
                if budget <= 0:
                    break
                if r.rid not in take_of:
                    if len(take_of) >= MAX_SEGMENTS:
                        continue
                    if r.scene_id not in used_scenes:
                        if len(used_scenes) >= MAX_SCENES:
                            continue
                        used_scenes.append(r.scene_id)
                rem = r.n_rays - r.next_ray - take_of.get(r.rid, 0)
                if rem <= 0:
                    continue
                allow = budget if k > 0 else max(PACKET * cost(r), self.tick_rays // 4)
                take = min(rem, min(allow, budget) // cost(r))
                if take < rem:
                    # whole packets, at least one, never past the request's end
                    take = min(rem, max(PACKET, (take // PACKET) * PACKET))
                take_of[r.rid] = take_of.get(r.rid, 0) + take
                budget -= take * cost(r)
            segs = []
            counts: Dict[int, int] = {}
            for r in reqs:
                take = take_of.get(r.rid, 0)
                if take > 0:
                    segs.append((r, r.next_ray, take))
                    r.next_ray += take
                    counts[r.rid] = 1
            if not segs:
                continue
            handle = self.ex.launch(s, segs)
            involved = {id(r): r for r, _, _ in segs}
            for r in involved.values():
                r.chunks_out += counts[r.rid]
            self.in_flight.append(Tick(s, handle, list(involved.values()), counts, time.perf_counter()))

    def _complete(self, now: float) -> None:
        still = []
        for t in self.in_flight:
            if not self.ex.done(t.handle, now):
                still.append(t)
                continue
            err = self.ex.error(t.handle)
            for r in t.requests:
                r.chunks_out -= t.chunk_counts[r.rid]
                if err is not None:
                    r.next_ray = r.n_rays
                if r.chunks_out == 0 and r.next_ray >= r.n_rays and not r.future.done():
                    r.t_done = now
                    if err is not None:
                        r.future.set_exception(err)
                    else:
                        r.future.set_result(self.ex.result(r))
                    self.active.remove(r)
                    self.used -= r.bytes
                    self.ex.release(r)
                    self.done.append(r)
        self.in_flight = still

    def fail_all(self, err: Exception) -> None:
        """Fail every admitted and in-flight request (scheduler fault)."""
        for r in list(self.active):
            if r.future is not None and not r.future.done():
                r.future.set_exception(err)
            self.ex.release(r)
        self.active.clear()
        self.in_flight.clear()
        self.used = 0.0

    # -- reporting -------------------------------------------------------------
    def describe(self) -> str:
        """One-line state of the scheduler: what a drain is waiting for."""
        now = time.perf_counter()
        ticks = ", ".join(f"stream {t.stream}: requests {[r.rid for r in t.requests]} for {now - t.t_launch:.1f} s"
                          for t in self.in_flight)
        act = ", ".join(f"{r.rid} ({r.kind}, {r.next_ray}/{r.n_rays} rays handed out, {r.chunks_out} chunks out)"
                        for r in self.active[:8])
        return (f"queue {len(self.queue)} (first {[r.rid for r in self.queue[:8]]}), active {len(self.active)} "
                f"[{act}], in flight {len(self.in_flight)} [{ticks}], {len(self.done)} done, "
                f"{self.used / 1e9:.2f} GB of {self.budget / 1e9:.0f} GB in use")

    def latency_stats(self) -> Dict[str, float]:
        lat = sorted(r.t_done - r.t_submit for r in self.done if r.t_done > 0)
        if not lat:
            return {"n": 0}

        def pct(p):
            k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
            return lat[k]

        return {"n": len(lat), "p50_s": pct(50), "p99_s": pct(99), "mean_s": statistics.fmean(lat),
                "max_s": lat[-1]}


class GpuExecutor:
    """Runs ticks on the GPU through the libgr binding, one torch stream per
    scheduler stream (default priority)."""

    def __init__(self, scenes: Dict[int, object], n_streams: int = 2, keep_rays: bool = False,
                 hit_list_cap: int = 0):
        import torch

        from . import api
        self.torch = torch
        self.api = api
        self.scenes = scenes
        self.device = next(iter(scenes.values())).device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.keep_rays = keep_rays
        self.hit_list_cap = hit_list_cap
        # one hit-list scratch per stream (a stream's ticks run one after
        # another); the per-Gaussian sums belong to the requests
        self.scratch = [None] * n_streams
        if hit_list_cap != -1:
            nb = api.fused_scratch_bytes(0, hit_list_cap=hit_list_cap)
            self.scratch = [torch.empty(nb // 4, device=self.device) for _ in range(n_streams)]

    def _planes(self, req: Request, device=None):
        p = req.geom.get("planes")
        if p is None:
            return None
        t = self.torch.as_tensor(p, dtype=self.torch.int32).reshape(-1, 2).contiguous()
        return t if device is None else t.to(device)

    def ray_count(self, req: Request) -> int:
        if req.rays is not None:
            return int(req.rays[0].shape[1])
        return self.api.ray_count(req.geom, self._planes(req))  # host copy: only its length is read

    def request_bytes(self, req: Request) -> int:
        m = self.ray_count(req)
        b = 28 * m  # rays (24 B) + output (4 B)
        if req.kind == "gradient":
            n = self.scenes[req.scene_id].n
            # target, per-Gaussian sums, gradients and the loss (the hit-list
            # scratch is per stream)
            b += 4 * m + self.api.backward_scratch_bytes(n) + 44 * n + 8
        return int(b)

    def setup(self, req: Request) -> None:
        torch = self.torch
        st = self.streams[req.stream]
        with torch.cuda.stream(st):
            m = req.n_rays
            planes = None
            if req.rays is not None:
                ro, rd = (torch.as_tensor(a, dtype=torch.float32).to(self.device).contiguous() for a in req.rays)
                if tuple(ro.shape) != (3, m) or tuple(rd.shape) != (3, m):
                    raise ValueError("request rays must be two (3, m) arrays")
            else:
                planes = self._planes(req, self.device)
                ro = torch.empty(3, m, device=self.device)
                rd = torch.empty(3, m, device=self.device)
                self.api.make_rays(req.geom, self.device, planes=planes, out=(ro, rd))
            state = {"ro": ro, "rd": rd, "out": torch.empty(m, device=self.device), "planes": planes}
            if req.kind == "gradient":
                if req.target is not None:
                    tgt = torch.as_tensor(req.target, dtype=torch.float32).to(self.device)
                else:  # seeded synthetic measurements
                    g = torch.Generator(device=self.device)
                    g.manual_seed(int(getattr(req, "target_seed", 0)))
                    if req.loss == "poisson":
                        tgt = torch.poisson(torch.full((m,), 5.0, device=self.device), generator=g)
                    else:
                        tgt = torch.rand(m, device=self.device, generator=g) * 50.0
                state["target"] = tgt
                sc = self.scenes[req.scene_id]
                state["accum"] = torch.empty(self.api.backward_scratch_bytes(sc.n) // 4, device=self.device)
                self.api.backward_accum_zero(sc, state["accum"], stream=st)
                state["loss"] = torch.zeros(1, dtype=torch.float64, device=self.device)
            req.state = state

    def launch(self, s: int, segs):
        torch = self.torch
        st = self.streams[s]
        err = None
        fwd = [x for x in segs if x[0].kind != "gradient"]
        grad = [x for x in segs if x[0].kind == "gradient"]
        with torch.cuda.stream(st):
            try:
                for part in (fwd[k0:k0 + MAX_SEGMENTS] for k0 in range(0, len(fwd), MAX_SEGMENTS)):
                    scene_ids = []
                    for r, _, _ in part:
                        if r.scene_id not in scene_ids:
                            scene_ids.append(r.scene_id)
                    table = [(scene_ids.index(r.scene_id), r.state["ro"], r.state["rd"], a, c,
                              r.state["out"], a) for r, a, c in part]
                    self.api.project_batched([self.scenes[i] for i in scene_ids], table, stream=st)
                for part in (grad[k0:k0 + MAX_SEGMENTS] for k0 in range(0, len(grad), MAX_SEGMENTS)):
                    scene_ids = []
                    for r, _, _ in part:
                        if r.scene_id not in scene_ids:
                            scene_ids.append(r.scene_id)
                    table = [{"scene": scene_ids.index(r.scene_id), "rays_o": r.state["ro"],
                              "rays_d": r.state["rd"], "ray_offset": a, "n_rays": c, "loss": r.loss,
                              "background": r.background, "target": r.state["target"],
                              "out_proj": r.state["out"], "out_offset": a, "accum": r.state["accum"],
                              "out_loss": r.state["loss"]} for r, a, c in part]
                    self.api.project_backward_batched([self.scenes[i] for i in scene_ids], table,
                                                      scratch=self.scratch[s], hit_list_cap=self.hit_list_cap,
                                                      stream=st)
                    for r, a, c in part:
                        if a + c == r.n_rays:  # the request's last chunk: its epilogue
                            r.state["grads"] = self.api.backward_finish(self.scenes[r.scene_id],
                                                                        r.state["accum"], stream=st)
            except Exception as e:  # a failed launch fails the tick's requests
                err = e
            ev = torch.cuda.Event()
            ev.record(st)
        return {"event": ev, "error": err}

    def done(self, handle, now) -> bool:
        return handle["error"] is not None or handle["event"].query()

    def error(self, handle):
        return handle["error"]

    def result(self, req: Request):
        if req.kind == "gradient":
            return {"proj": req.state["out"], "grads": req.state["grads"], "loss": req.state["loss"]}
        return req.state["out"]

    def release(self, req: Request) -> None:
        if not self.keep_rays:
            req.state = {k: v for k, v in req.state.items() if k not in ("ro", "rd", "target", "accum")}


class Server:
    """Thread wrapper: ``submit`` from any thread, the loop runs on its own."""

    def __init__(self, scheduler: Scheduler, idle_sleep: float = 2e-4):
        self.sched = scheduler
        self.idle_sleep = idle_sleep
        self._stop = threading.Event()
        self._thread: Optional[threading.Thread] = None
        self._t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, req: Request) -> cf.Future:
        return self.sched.submit(req, self.now())

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="gr-serve", daemon=True)
        self._thread.start()
        return self

    def _loop(self) -> None:
        while not self._stop.is_set():
            try:
                busy = self.sched.step(self.now())
            except Exception as e:  # keep serving: fail what was in progress
                self.sched.fail_all(e)
                busy = False
            if not busy:
                time.sleep(self.idle_sleep)

    def drain(self, timeout: float = 600.0, progress=None, progress_every: float = 30.0) -> None:
        """Waits until nothing is queued, active or in flight. ``progress(str)``
        gets the scheduler's state every ``progress_every`` seconds of waiting;
        the TimeoutError names the state at the deadline."""
        t0 = time.perf_counter()
        t_end, t_next = t0 + timeout, t0 + progress_every
        while time.perf_counter() < t_end:
            s = self.sched
            if not (s.queue or s.active or s.in_flight):
                return
            if progress is not None and time.perf_counter() >= t_next:
                progress(f"draining for {time.perf_counter() - t0:.0f} s: {s.describe()}")
                t_next += progress_every
            time.sleep(1e-3)
        raise TimeoutError(f"server did not drain within {timeout:.0f} s: {self.sched.describe()}")

    def stop(self) -> None:
        self._stop.set()
        if self._thread:
            self._thread.join()


# ---------------------------------------------------------------------------
# the served mixed-stream workload
# ---------------------------------------------------------------------------

def mixed_stream(n_requests: int, qps: float, seed: int, ct_scene_ids: Sequence[int],
                 pet_scene_ids: Sequence[int], grad_fraction: float = 0.3):
    """Seeded request stream: Poisson arrivals at ``qps``; half cone-beam CT
    (square detector 128..512 step 32 over 409.6 mm, 1-64 views), half PET
    (1-8 ring-difference planes of the 200k-Gaussian scanner, 86,688 LORs each);
    ``grad_fraction`` of them gradient requests (L2 for CT, Poisson for PET).
    Returns [(arrival_time_s, Request)]."""
    import numpy as np

    from .inputs import CT_CONE_500K, PET_200K
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / qps))
        grad = bool(rng.uniform() < grad_fraction)
        if rng.uniform() < 0.5:
            n = int(rng.choice(np.arange(128, 513, 32)))
            views = int(rng.integers(1, 65))
            g = dict(CT_CONE_500K["geom"], nu=n, nv=n, pitch_u=409.6 / n, pitch_v=409.6 / n,
                     n_views=views, angle0=float(rng.uniform(0, 2 * np.pi)))
            sid = int(rng.choice(ct_scene_ids))
            req = Request(sid, g, kind="gradient" if grad else "forward", loss="l2")
        else:
            k = int(rng.integers(1, 9))
            diffs = rng.choice(np.arange(-15, 16), size=k, replace=False)
            planes = []
            for dlt in diffs:
                r1 = int(rng.integers(max(0, -dlt), min(32, 32 - dlt)))
                planes.append((r1, r1 + int(dlt)))
            g = dict(PET_200K["geom"], planes=np.asarray(planes, dtype=np.int32))
            sid = int(rng.choice(pet_scene_ids))
            req = Request(sid, g, kind="gradient" if grad else "forward", loss="poisson",
                          background=0.05)
        if grad:
            req.target_seed = int(rng.integers(1 << 30))
        out.append((t, req))
    return out


def scene_pool(device, n_scenes: int = 32, seed0: int = 100, n_min: int = 10_000,
               n_max: int = 500_000, pool_seed: int = 5):
    """Resident scenes for the served workload: seeds seed0.., log-uniform
    Gaussian counts in [n_min, n_max]; the first half follow the cone-beam CT
    recipe (ball of radius 100 mm, scales 0.5-4 mm), the second half the PET
    recipe (cylinder r 300 mm, length 250 mm, scales 1-8 mm).
    Returns (scenes, ct_ids, pet_ids)."""
    import numpy as np
    import torch

    from . import api
    from .inputs import CT_CONE_500K, PET_200K, preset_scene
    rng = np.random.default_rng(pool_seed)
    scenes, ct_ids, pet_ids = {}, [], []
    for k in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        pet = k >= n_scenes // 2
        sc = preset_scene(PET_200K if pet else CT_CONE_500K, seed=seed0 + k, n=n)
        t = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in
             (sc.mean, sc.scale, sc.quat, sc.density)]
        scenes[k] = api.Scene(*t)
        (pet_ids if pet else ct_ids).append(k)
    return scenes, ct_ids, pet_ids


def run_served(scenes, stream, n_streams: int = 2, hbm_budget: float = 200e9,
               tick_rays: int = 4_000_000, hit_list_cap: int = 0, progress=None,
               progress_every: int = 500, drain_log=None, drain_timeout: float = 600.0) -> Dict:
    """Serve a list of (arrival_s, Request) in real time; returns latency and
    throughput figures. ``progress(k, n)`` is called after every
    ``progress_every``-th submission; ``drain_log(str)`` gets the scheduler's
    state every 30 s of a drain that takes that long."""
    ex = GpuExecutor(scenes, n_streams=n_streams, hit_list_cap=hit_list_cap)
    sched = Scheduler(ex, hbm_budget=hbm_budget, n_streams=n_streams, tick_rays=tick_rays)
    srv = Server(sched).start()
    futs = []
    t0 = srv.now()
    for t_arr, req in stream:
        delay = t0 + t_arr - srv.now()
        if delay > 0:
            time.sleep(delay)
        futs.append(srv.submit(req))
        if progress is not None and len(futs) % progress_every == 0:
            progress(len(futs), len(stream))
    srv.drain(drain_timeout, progress=drain_log)
    srv.stop()
    wall = srv.now() - t0
    errs = [f.exception() for f in futs if f.exception() is not None]
    st = sched.latency_stats()
    rays = sum(r.n_rays for r in sched.done)
    st.update({"requests": len(futs), "failed": len(errs), "wall_s": wall,
               "requests_per_s": len(futs) / wall, "rays_per_s": rays / wall})
    return st


def run_one_at_a_time(scenes, stream, progress=None, progress_every: int = 25) -> Dict:
    """Baseline: the same arrivals served one request at a time, forward
    requests with one plain gr_project launch per view (per plane for PET),
    gradient requests with their fused launch; the next request starts when
    the previous one has finished (or when it arrives). ``progress(k, n)`` is
    called after every ``progress_every``-th finished request."""
    import numpy as np
    import torch

    from . import api
    dev = next(iter(scenes.values())).device
    t0 = time.perf_counter()
    lat = []
    rays_total = 0
    for t_arr, req in stream:
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        planes = req.geom.get("planes")
        pt = None if planes is None else torch.as_tensor(planes, dtype=torch.int32).reshape(-1, 2).to(dev)
        ro, rd = api.make_rays(req.geom, dev, planes=pt)
        m = ro.shape[1]
        rays_total += m
        sc = scenes[req.scene_id]
        if req.kind == "gradient":
            g = torch.Generator(device=dev)
            g.manual_seed(int(req.target_seed))
            if req.loss == "poisson":
                tgt = torch.poisson(torch.full((m,), 5.0, device=dev), generator=g)
            else:
                tgt = torch.rand(m, device=dev, generator=g) * 50.0
            api.project_backward(sc, ro, rd, loss=req.loss, target=tgt, background=req.background)
        else:
            views = int(req.geom["n_views"])
            per = m // views
            out = torch.empty(m, device=dev)
            for v in range(views):
                a = v * per
                api.project(sc, ro[:, a:a + per].contiguous(), rd[:, a:a + per].contiguous(),
                            out=out[a:a + per])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - t_arr)
        if progress is not None and len(lat) % progress_every == 0:
            progress(len(lat), len(stream))
    wall = time.perf_counter() - t0
    lat = np.sort(np.asarray(lat))

    def pct(p):
        return float(lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))])

    return {"n": len(lat), "p50_s": pct(50), "p99_s": pct(99), "mean_s": float(lat.mean()),
            "max_s": float(lat[-1]), "wall_s": wall, "requests_per_s": len(lat) / wall,
            "rays_per_s": rays_total / wall}


def main(argv=None) -> int:
    """Served mixed-stream benchmark: prints one JSON line."""
    import argparse
    import json

    import torch
    ap = argparse.ArgumentParser(description="continuous-batching server benchmark")
    ap.add_argument("--requests", type=int, default=3000)
    ap.add_argument("--qps", type=float, default=50.0)
    ap.add_argument("--scenes", type=int, default=32)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--no-baseline", action="store_true")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    scenes, ct_ids, pet_ids = scene_pool(dev, n_scenes=args.scenes)
    torch.cuda.synchronize()
    stream = mixed_stream(args.requests, args.qps, args.seed, ct_ids, pet_ids)
    warm = mixed_stream(8, 1000.0, args.seed + 1, ct_ids, pet_ids)
    run_served(scenes, warm)
    out = {"served": run_served(scenes, stream), "requests": args.requests, "qps": args.qps,
           "scenes": args.scenes}
    if not args.no_baseline:
        out["one_at_a_time"] = run_one_at_a_time(scenes, mixed_stream(args.requests, args.qps, args.seed,
                                                                       ct_ids, pet_ids))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
