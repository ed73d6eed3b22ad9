"""Python binding of libgr: torch tensors in, torch tensors out.

Only argument marshalling lives here. Every step of the projection (ray set-up,
acceleration-structure build, forward, backward) runs in the HIP library; if
the library is missing the calls raise.

Array conventions follow include/gr.h: float32, CUDA (HIP) device, SoA shapes
mean (3, n), scale (3, n), quat (4, n) as (w, x, y, z), density (n,), rays
(3, m). Work is enqueued on torch's current stream of the tensors' device.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, name: str, shape: Tuple[int, ...], device=None, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class _Launch:
    """gr_launch options plus the lifetime of a persistent launch's counter."""

    def __init__(self, waves_per_group: int = 0, xcd_remap: int = 0, persistent=0, device=None,
                 traversal: int = 0, hit_list_cap: int = 0, precision: str = "fp64"):
        self.opt = None
        self.counter = None
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        if (not waves_per_group and not xcd_remap and not persistent and not traversal and not hit_list_cap
                and precision == "fp64"):
            return
        opt = L.GrLaunch()
        opt.waves_per_group = int(waves_per_group)
        opt.xcd_remap = int(xcd_remap)
        opt.traversal = int(traversal)
        opt.hit_list_cap = int(hit_list_cap)
        opt.precision = PRECISIONS[precision]
        if persistent:
            # one uint32 ticket counter per call; the library zeroes it on the stream
            self.counter = torch.empty(1, dtype=torch.int32, device=device)
            opt.work_counter = self.counter.data_ptr()
            opt.persistent_groups = 0 if persistent is True else int(persistent)
        self.opt = opt

    @property
    def ref(self):
        return None if self.opt is None else ctypes.byref(self.opt)


# forward arithmetic (gr_launch.precision): Eq. 7 in FP64 from 80-byte records,
# or in FP32 from 64-byte compact records
PRECISIONS = {"fp64": 0, "fp32": 1}


def _launch(waves_per_group: int = 0, xcd_remap: int = 0, persistent=0, device=None,
            traversal: int = 0, hit_list_cap: int = 0, precision: str = "fp64") -> _Launch:
    return _Launch(waves_per_group, xcd_remap, persistent, device, traversal, hit_list_cap, precision)


def accel_bytes(n: int, leaf_size: int = 0) -> int:
    out = ctypes.c_size_t()
    L.check("gr_accel_bytes", L.load().gr_accel_bytes(int(n), int(leaf_size), ctypes.byref(out)))
    return int(out.value)


def backward_scratch_bytes(n: int) -> int:
    out = ctypes.c_size_t()
    L.check("gr_backward_scratch_bytes", L.load().gr_backward_scratch_bytes(int(n), ctypes.byref(out)))
    return int(out.value)


def fused_scratch_bytes(n: int, waves_per_group: int = 0, persistent=0, hit_list_cap: int = 0) -> int:
    """Scratch bytes with which the fused-loss backward records and replays
    hit lists on the current device (gr_fused_scratch_bytes)."""
    opt = L.GrLaunch()
    opt.waves_per_group = int(waves_per_group)
    opt.persistent_groups = 0 if persistent is True or not persistent else int(persistent)
    opt.hit_list_cap = int(hit_list_cap)
    out = ctypes.c_size_t()
    L.check("gr_fused_scratch_bytes", L.load().gr_fused_scratch_bytes(int(n), ctypes.byref(opt), ctypes.byref(out)))
    return int(out.value)


class Scene:
    """A set of Gaussians with its on-device acceleration structure.

    Holds references to the parameter tensors (the library reads them again in
    the backward epilogue) and owns the workspace tensor. ``build()`` re-runs
    the on-device build, e.g. after an optimiser step changed the parameters
    in place."""

    def __init__(self, mean: torch.Tensor, scale: torch.Tensor, quat: torch.Tensor,
                 density: torch.Tensor, kappa: float = 3.0, leaf_size: int = 0, build: bool = True):
        n = int(density.shape[0]) if density.dim() == 1 else -1
        dev = density.device
        _require(density, "density", (n,))
        _require(mean, "mean", (3, n), dev)
        _require(scale, "scale", (3, n), dev)
        _require(quat, "quat", (4, n), dev)
        self.n = n
        self.device = dev
        self.mean, self.scale, self.quat, self.density = mean, scale, quat, density
        self.kappa = float(kappa)
        self.leaf_size = int(leaf_size)
        self.accel = torch.empty(accel_bytes(n, leaf_size), dtype=torch.uint8, device=dev)
        self._c = L.GrScene(n, mean.data_ptr(), scale.data_ptr(), quat.data_ptr(), density.data_ptr(),
                            self.kappa, self.leaf_size, self.accel.data_ptr(), self.accel.numel())
        if build:
            self.build()

    @property
    def c_struct(self) -> L.GrScene:
        return self._c

    def build(self) -> "Scene":
        L.check("gr_build_accel", L.load().gr_build_accel(ctypes.byref(self._c), _stream(self.device)))
        return self

    def refit(self) -> "Scene":
        """Recompute records and boxes for changed parameters, keeping the
        last build's order and tree (gr_refit_accel)."""
        L.check("gr_refit_accel", L.load().gr_refit_accel(ctypes.byref(self._c), _stream(self.device)))
        return self

    def invalid_count(self) -> int:
        out = ctypes.c_int64()
        L.check("gr_scene_invalid_count",
                L.load().gr_scene_invalid_count(ctypes.byref(self._c), ctypes.byref(out),
                                                _stream(self.device)))
        return int(out.value)

    def status_flags(self) -> int:
        """Device-side consistency-check bits since the last build (0 = none)."""
        out = ctypes.c_int32()
        L.check("gr_scene_status", L.load().gr_scene_status(ctypes.byref(self._c), ctypes.byref(out),
                                                            _stream(self.device)))
        return int(out.value)

    def nbytes(self) -> int:
        return int(self.accel.numel())


def project(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor,
            out: Optional[torch.Tensor] = None, waves_per_group: int = 0,
            xcd_remap: int = 0, persistent=0, traversal: int = 0, precision: str = "fp64") -> torch.Tensor:
    """I[r] for every ray (Eq. 12 with the kappa cutoff). precision "fp32"
    selects the compact FP32 records (gr_launch.precision)."""
    m = int(rays_o.shape[1]) if rays_o.dim() == 2 else -1
    _require(rays_o, "rays_o", (3, m), scene.device)
    _require(rays_d, "rays_d", (3, m), scene.device)
    if out is None:
        out = torch.empty(m, dtype=torch.float32, device=scene.device)
    _require(out, "out", (m,), scene.device)
    ln = _launch(waves_per_group, xcd_remap, persistent, scene.device, traversal, precision=precision)
    L.check("gr_project", L.load().gr_project(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d),
                                              m, _ptr(out), ln.ref, _stream(scene.device)))
    return out


def project_stats(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor,
                  out: Optional[torch.Tensor] = None, waves_per_group: int = 0,
                  xcd_remap: int = 0, persistent=0,
                  traversal: int = 0, precision: str = "fp64") -> Tuple[torch.Tensor, Dict[str, int]]:
    """project() plus exact work counters: included pairs, evaluated pairs,
    leaves visited and packets (synchronises to read them)."""
    m = int(rays_o.shape[1])
    _require(rays_o, "rays_o", (3, m), scene.device)
    _require(rays_d, "rays_d", (3, m), scene.device)
    if out is None:
        out = torch.empty(m, dtype=torch.float32, device=scene.device)
    stats = torch.zeros(8, dtype=torch.int64, device=scene.device)
    ln = _launch(waves_per_group, xcd_remap, persistent, scene.device, traversal, precision=precision)
    L.check("gr_project_stats",
            L.load().gr_project_stats(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d), m,
                                      _ptr(out), _ptr(stats), ln.ref, _stream(scene.device)))
    v = stats.cpu().tolist()
    return out, {"pairs": v[0], "evaluated": v[1], "leaves": v[2], "packets": v[3],
                 "candidates": v[4], "candidates_hit": v[5]}


def project_batched(scenes: Sequence[Scene], segments: Sequence[Tuple], waves_per_group: int = 0,
                    xcd_remap: int = 0, persistent=0,
                    stream: Optional[torch.cuda.Stream] = None, traversal: int = 0,
                    precision: str = "fp64") -> None:
    """One launch over several segments. Each segment is
    (scene index, rays_o, rays_d, ray_offset, n_rays, out, out_offset): rays
    [ray_offset, ray_offset + n_rays) of the (3, m) arrays go to
    out[out_offset ...]. Results equal project() on each segment's rays."""
    if not scenes:
        raise ValueError("no scenes")
    dev = scenes[0].device
    SC = (L.GrScene * len(scenes))(*[s.c_struct for s in scenes])
    SG = (L.GrSegment * max(1, len(segments)))()
    keep = []
    for k, (si, ro, rd, off, cnt, out, oo) in enumerate(segments):
        m = int(ro.shape[1])
        _require(ro, "rays_o", (3, m), dev)
        _require(rd, "rays_d", (3, m), dev)
        if out.dtype != torch.float32 or out.device != dev or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor on the scenes' device")
        if not (0 <= off and off + cnt <= m and 0 <= oo and oo + cnt <= out.numel()):
            raise ValueError("segment outside its ray or output array")
        if not 0 <= si < len(scenes):
            raise ValueError("segment scene index out of range")
        SG[k].scene, SG[k].stride, SG[k].ray_offset, SG[k].n_rays = int(si), m, int(off), int(cnt)
        SG[k].ray_o, SG[k].ray_d, SG[k].out, SG[k].out_offset = ro.data_ptr(), rd.data_ptr(), out.data_ptr(), int(oo)
        keep.append((ro, rd, out))
    ln = _launch(waves_per_group, xcd_remap, persistent, dev, traversal, precision=precision)
    st = _stream(dev) if stream is None else ctypes.c_void_p(stream.cuda_stream)
    L.check("gr_project_batched",
            L.load().gr_project_batched(SC, len(scenes), SG, len(segments), ln.ref, st))


def project_backward(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor,
                     grad_out: Optional[torch.Tensor] = None, *, loss: Optional[str] = None,
                     target: Optional[torch.Tensor] = None, background: float = 0.0,
                     out_proj: Optional[torch.Tensor] = None, out_loss: Optional[torch.Tensor] = None,
                     scratch: Optional[torch.Tensor] = None, grads: Optional[Dict] = None,
                     waves_per_group: int = 0, xcd_remap: int = 0,
                     persistent=0, traversal: int = 0, hit_list_cap: int = 0) -> Dict[str, torch.Tensor]:
    """Gradient of L with respect to mean, scale, quat and density.

    Either ``grad_out`` (dL/dI per ray) is given, or ``loss`` is "l2" /
    "poisson" with ``target`` (and ``background`` for Poisson), in which case
    the forward, the loss weight and the backward run fused in one launch;
    ``out_proj`` then receives I and ``out_loss`` (a float64 device scalar) has
    L added to it. Without ``scratch``, the fused form gets the scratch of
    ``fused_scratch_bytes`` (hit lists recorded by its forward half, see
    gr_fused_scratch_bytes; ``hit_list_cap=-1`` re-traverses instead)."""
    dev = scene.device
    m = int(rays_o.shape[1])
    _require(rays_o, "rays_o", (3, m), dev)
    _require(rays_d, "rays_d", (3, m), dev)
    n = scene.n
    if grads is None:
        grads = {"mean": torch.empty(3, n, device=dev), "scale": torch.empty(3, n, device=dev),
                 "quat": torch.empty(4, n, device=dev), "density": torch.empty(n, device=dev)}
    if scratch is None:
        nb = (backward_scratch_bytes(n) if grad_out is not None else
              fused_scratch_bytes(n, waves_per_group, persistent, hit_list_cap))
        scratch = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    lossp = None
    if grad_out is not None:
        _require(grad_out, "grad_out", (m,), dev)
        if loss is not None:
            raise ValueError("give grad_out or loss, not both")
    else:
        kinds = {"l2": L.GR_LOSS_L2, "poisson": L.GR_LOSS_POISSON}
        if loss not in kinds:
            raise ValueError("loss must be 'l2' or 'poisson' when grad_out is None")
        _require(target, "target", (m,), dev)
        if out_proj is not None:
            _require(out_proj, "out_proj", (m,), dev)
        if out_loss is not None:
            _require(out_loss, "out_loss", (1,), dev, torch.float64)
        lc = L.GrLoss(kinds[loss], float(background), target.data_ptr(),
                      None if out_proj is None else out_proj.data_ptr(),
                      None if out_loss is None else out_loss.data_ptr())
        lossp = ctypes.byref(lc)
    ln = _launch(waves_per_group, xcd_remap, persistent, dev, traversal, hit_list_cap)
    L.check("gr_project_backward",
            L.load().gr_project_backward(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d), m,
                                         _ptr(grad_out), lossp, _ptr(grads["mean"]),
                                         _ptr(grads["scale"]), _ptr(grads["quat"]),
                                         _ptr(grads["density"]), _ptr(scratch),
                                         scratch.numel() * scratch.element_size(),
                                         ln.ref, _stream(dev)))
    return grads


def project_backward_static(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor,
                            grad_out: Optional[torch.Tensor] = None, *, loss: Optional[str] = None,
                            target: Optional[torch.Tensor] = None, background: float = 0.0,
                            out_proj: Optional[torch.Tensor] = None, out_loss: Optional[torch.Tensor] = None,
                            grads: Optional[Dict] = None, waves_per_group: int = 0, traversal: int = 0,
                            hit_list_cap: int = 0) -> Dict[str, torch.Tensor]:
    """project_backward through gr_project_backward_static: the library's
    static device scratch instead of a caller buffer (for callers that cannot
    allocate; the caller still provides the gradient outputs through
    ``grads``). Calls on one GPU must not overlap."""
    dev = scene.device
    m = int(rays_o.shape[1])
    _require(rays_o, "rays_o", (3, m), dev)
    _require(rays_d, "rays_d", (3, m), dev)
    n = scene.n
    if grads is None:
        grads = {"mean": torch.empty(3, n, device=dev), "scale": torch.empty(3, n, device=dev),
                 "quat": torch.empty(4, n, device=dev), "density": torch.empty(n, device=dev)}
    lossp = None
    if grad_out is not None:
        _require(grad_out, "grad_out", (m,), dev)
        if loss is not None:
            raise ValueError("give grad_out or loss, not both")
    else:
        kinds = {"l2": L.GR_LOSS_L2, "poisson": L.GR_LOSS_POISSON}
        if loss not in kinds:
            raise ValueError("loss must be 'l2' or 'poisson' when grad_out is None")
        _require(target, "target", (m,), dev)
        if out_proj is not None:
            _require(out_proj, "out_proj", (m,), dev)
        if out_loss is not None:
            _require(out_loss, "out_loss", (1,), dev, torch.float64)
        lc = L.GrLoss(kinds[loss], float(background), target.data_ptr(),
                      None if out_proj is None else out_proj.data_ptr(),
                      None if out_loss is None else out_loss.data_ptr())
        lossp = ctypes.byref(lc)
    ln = _launch(waves_per_group, 0, 0, dev, traversal, hit_list_cap)
    L.check("gr_project_backward_static",
            L.load().gr_project_backward_static(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d), m,
                                                _ptr(grad_out), lossp, _ptr(grads["mean"]), _ptr(grads["scale"]),
                                                _ptr(grads["quat"]), _ptr(grads["density"]), ln.ref, _stream(dev)))
    return grads


def backward_accum_zero(scene: Scene, accum: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> None:
    """Zeroes a request's 10 x n accumulators (gr_backward_accum_zero)."""
    _require(accum, "accum", (backward_scratch_bytes(scene.n) // 4,), scene.device)
    st = _stream(scene.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
    L.check("gr_backward_accum_zero", L.load().gr_backward_accum_zero(scene.n, _ptr(accum), st))


def project_backward_batched(scenes: Sequence[Scene], segments: Sequence[Dict],
                             scratch: Optional[torch.Tensor] = None, waves_per_group: int = 0,
                             traversal: int = 0, hit_list_cap: int = 0,
                             stream: Optional[torch.cuda.Stream] = None) -> None:
    """One fused forward -> loss -> backward launch over several segments
    (gr_project_backward_batched). Each segment is a dict with keys scene
    (index), rays_o, rays_d ((3, m) arrays), ray_offset, n_rays, loss ("l2" /
    "poisson"), target (indexed like out_proj: element out_offset + i),
    accum (the request's accumulators, added to), and optionally background,
    out_proj, out_offset, out_loss (float64, shape (1,), added to). scratch:
    None (re-traversal) or at least fused_scratch_bytes(0, ...) bytes."""
    if not scenes:
        raise ValueError("no scenes")
    dev = scenes[0].device
    kinds = {"l2": L.GR_LOSS_L2, "poisson": L.GR_LOSS_POISSON}
    SC = (L.GrScene * len(scenes))(*[s.c_struct for s in scenes])
    SG = (L.GrBwdSegment * max(1, len(segments)))()
    for k, g in enumerate(segments):
        ro, rd = g["rays_o"], g["rays_d"]
        m = int(ro.shape[1])
        _require(ro, "rays_o", (3, m), dev)
        _require(rd, "rays_d", (3, m), dev)
        si, off, cnt, oo = int(g["scene"]), int(g["ray_offset"]), int(g["n_rays"]), int(g.get("out_offset", 0))
        if not 0 <= si < len(scenes):
            raise ValueError("segment scene index out of range")
        if not (0 <= off and off + cnt <= m and oo >= 0):
            raise ValueError("segment outside its ray array")
        tgt = g["target"]
        if tgt.dtype != torch.float32 or tgt.device != dev or not tgt.is_contiguous() or oo + cnt > tgt.numel():
            raise ValueError("target must be a contiguous float32 device tensor covering the segment")
        op = g.get("out_proj")
        if op is not None and (op.dtype != torch.float32 or op.device != dev or not op.is_contiguous()
                               or oo + cnt > op.numel()):
            raise ValueError("out_proj must be a contiguous float32 device tensor covering the segment")
        _require(g["accum"], "accum", (backward_scratch_bytes(scenes[si].n) // 4,), dev)
        ol = g.get("out_loss")
        if ol is not None:
            _require(ol, "out_loss", (1,), dev, torch.float64)
        if g["loss"] not in kinds:
            raise ValueError("loss must be 'l2' or 'poisson'")
        SG[k].scene, SG[k].loss_kind = si, kinds[g["loss"]]
        SG[k].ray_o, SG[k].ray_d, SG[k].stride = ro.data_ptr(), rd.data_ptr(), m
        SG[k].ray_offset, SG[k].n_rays = off, cnt
        SG[k].target, SG[k].out_offset = tgt.data_ptr(), oo
        SG[k].out_proj = None if op is None else op.data_ptr()
        SG[k].accum = g["accum"].data_ptr()
        SG[k].out_loss = None if ol is None else ol.data_ptr()
        SG[k].background = float(g.get("background", 0.0))
    ln = _launch(waves_per_group, 0, 0, dev, traversal, hit_list_cap)
    st = _stream(dev) if stream is None else ctypes.c_void_p(stream.cuda_stream)
    nb = 0 if scratch is None else scratch.numel() * scratch.element_size()
    L.check("gr_project_backward_batched",
            L.load().gr_project_backward_batched(SC, len(scenes), SG, len(segments), _ptr(scratch), nb,
                                                 ln.ref, st))


def backward_finish(scene: Scene, accum: torch.Tensor, grads: Optional[Dict] = None,
                    stream: Optional[torch.cuda.Stream] = None) -> Dict[str, torch.Tensor]:
    """Parameter gradients from a request's accumulators (gr_backward_finish)."""
    dev = scene.device
    n = scene.n
    _require(accum, "accum", (backward_scratch_bytes(n) // 4,), dev)
    if grads is None:
        grads = {"mean": torch.empty(3, n, device=dev), "scale": torch.empty(3, n, device=dev),
                 "quat": torch.empty(4, n, device=dev), "density": torch.empty(n, device=dev)}
    st = _stream(dev) if stream is None else ctypes.c_void_p(stream.cuda_stream)
    L.check("gr_backward_finish",
            L.load().gr_backward_finish(ctypes.byref(scene.c_struct), _ptr(accum), _ptr(grads["mean"]),
                                        _ptr(grads["scale"]), _ptr(grads["quat"]), _ptr(grads["density"]), st))
    return grads


def voxelize(scene: Scene, origin, spacing, dims, out: Optional[torch.Tensor] = None):
    """The scene's mixture density at the voxel centres origin + (ix, iy, iz) *
    spacing (gr_voxelize); returns a (nz, ny, nx) FP32 tensor."""
    return _voxelize(scene, origin, spacing, dims, out, None)


def voxelize_stats(scene: Scene, origin, spacing, dims, out: Optional[torch.Tensor] = None):
    """voxelize plus its work counters (gr_voxelize_stats): returns (volume,
    {"pairs": voxel-Gaussian pairs inside the cutoff, "evaluated": pairs
    evaluated})."""
    st = torch.zeros(2, dtype=torch.int64, device=scene.device)
    out = _voxelize(scene, origin, spacing, dims, out, st)
    a, b = (int(x) for x in st.cpu())
    return out, {"pairs": a, "evaluated": b}


def _voxelize(scene, origin, spacing, dims, out, stats):
    nx, ny, nz = (int(x) for x in dims)
    dev = scene.device
    if out is None:
        out = torch.empty(nz, ny, nx, device=dev)
    _require(out, "out", (nz, ny, nx), dev)
    g = L.GrGrid((ctypes.c_double * 3)(*[float(x) for x in origin]),
                 (ctypes.c_double * 3)(*[float(x) for x in spacing]), (ctypes.c_int64 * 3)(nx, ny, nz))
    lib = L.load()
    if stats is None:
        L.check("gr_voxelize", lib.gr_voxelize(ctypes.byref(scene.c_struct), ctypes.byref(g), _ptr(out),
                                               None, _stream(dev)))
    else:
        L.check("gr_voxelize_stats", lib.gr_voxelize_stats(ctypes.byref(scene.c_struct), ctypes.byref(g),
                                                           _ptr(out), _ptr(stats), None, _stream(dev)))
    return out


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam step in place on a contiguous FP32 device tensor (gr_adam_step);
    m and v are its moment tensors (zero before step 1)."""
    dev = param.device
    shape = tuple(param.shape)
    for t, nm in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _require(t, nm, shape, dev)
    hp = L.GrAdam(float(lr), float(beta1), float(beta2), float(eps), int(step))
    L.check("gr_adam_step", L.load().gr_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                                  ctypes.byref(hp), _stream(dev)))


def _tof_struct(n_bins: int, sigma: float, bin_width: float, center, atten, m: int, dev) -> L.GrTof:
    for t, nm in ((center, "center"), (atten, "atten")):
        if t is not None:
            _require(t, nm, (m,), dev)
    return L.GrTof(int(n_bins), float(sigma), float(bin_width), 0,
                   None if center is None else center.data_ptr(), None if atten is None else atten.data_ptr())


def project_tof(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor, n_bins: int, sigma: float = 0.0,
                bin_width: float = 0.0, center: Optional[torch.Tensor] = None,
                atten: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                waves_per_group: int = 0, xcd_remap: int = 0, persistent=0, traversal: int = 0) -> torch.Tensor:
    """Time-of-flight projection with attenuation (gr_project_tof): returns
    (max(1, n_bins), m), bin-major. n_bins = 0: atten times the projection."""
    m = int(rays_o.shape[1]) if rays_o.dim() == 2 else -1
    dev = scene.device
    _require(rays_o, "rays_o", (3, m), dev)
    _require(rays_d, "rays_d", (3, m), dev)
    nb = max(1, int(n_bins))
    if out is None:
        out = torch.empty(nb, m, dtype=torch.float32, device=dev)
    _require(out, "out", (nb, m), dev)
    tof = _tof_struct(n_bins, sigma, bin_width, center, atten, m, dev)
    ln = _launch(waves_per_group, xcd_remap, persistent, dev, traversal)
    L.check("gr_project_tof", L.load().gr_project_tof(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d), m,
                                                      ctypes.byref(tof), _ptr(out), ln.ref, _stream(dev)))
    return out


def project_tof_backward(scene: Scene, rays_o: torch.Tensor, rays_d: torch.Tensor, grad_out: torch.Tensor,
                         n_bins: int, sigma: float = 0.0, bin_width: float = 0.0,
                         center: Optional[torch.Tensor] = None, atten: Optional[torch.Tensor] = None,
                         scratch: Optional[torch.Tensor] = None, grads: Optional[Dict] = None,
                         waves_per_group: int = 0, xcd_remap: int = 0, persistent=0,
                         traversal: int = 0) -> Dict[str, torch.Tensor]:
    """Gradient of sum grad_out[b, r] I_b(r) of the TOF projection
    (gr_project_tof_backward) with respect to mean, scale, quat and density."""
    m = int(rays_o.shape[1]) if rays_o.dim() == 2 else -1
    dev = scene.device
    n = scene.n
    _require(rays_o, "rays_o", (3, m), dev)
    _require(rays_d, "rays_d", (3, m), dev)
    _require(grad_out, "grad_out", (max(1, int(n_bins)), m), dev)
    if grads is None:
        grads = {"mean": torch.empty(3, n, device=dev), "scale": torch.empty(3, n, device=dev),
                 "quat": torch.empty(4, n, device=dev), "density": torch.empty(n, device=dev)}
    if scratch is None:
        scratch = torch.empty(backward_scratch_bytes(n) // 4, dtype=torch.float32, device=dev)
    tof = _tof_struct(n_bins, sigma, bin_width, center, atten, m, dev)
    ln = _launch(waves_per_group, xcd_remap, persistent, dev, traversal)
    L.check("gr_project_tof_backward",
            L.load().gr_project_tof_backward(ctypes.byref(scene.c_struct), _ptr(rays_o), _ptr(rays_d), m,
                                             ctypes.byref(tof), _ptr(grad_out), _ptr(grads["mean"]),
                                             _ptr(grads["scale"]), _ptr(grads["quat"]), _ptr(grads["density"]),
                                             _ptr(scratch), scratch.numel() * scratch.element_size(), ln.ref,
                                             _stream(dev)))
    return grads


def tof_centers(rays_o: torch.Tensor, rays_d: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """TOF centre of each ray: its closest approach to the z axis in the
    transaxial plane (gr_tof_centers)."""
    m = int(rays_o.shape[1]) if rays_o.dim() == 2 else -1
    dev = rays_o.device
    _require(rays_o, "rays_o", (3, m), dev)
    _require(rays_d, "rays_d", (3, m), dev)
    if out is None:
        out = torch.empty(m, dtype=torch.float32, device=dev)
    _require(out, "out", (m,), dev)
    L.check("gr_tof_centers", L.load().gr_tof_centers(_ptr(rays_o), _ptr(rays_d), m, _ptr(out), _stream(dev)))
    return out


def loss_weights(kind: str, proj: torch.Tensor, target: torch.Tensor, background=0.0,
                 weight: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None):
    """Per-measurement weights dL/dI and the loss (gr_loss_weights): kind "l2"
    or "poisson"; background is a scalar or a tensor shaped like proj
    (expected randoms + scatter). Returns (weight, loss) with loss a (1,)
    float64 tensor the loss is added to."""
    dev = proj.device
    shape = tuple(proj.shape)
    _require(proj, "proj", shape, dev)
    _require(target, "target", shape, dev)
    bg_t = background if isinstance(background, torch.Tensor) else None
    if bg_t is not None:
        _require(bg_t, "background", shape, dev)
    if weight is None:
        weight = torch.empty(shape, dtype=torch.float32, device=dev)
    _require(weight, "weight", shape, dev)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
    _require(loss, "loss", (1,), dev, torch.float64)
    kinds = {"l2": L.GR_LOSS_L2, "poisson": L.GR_LOSS_POISSON}
    L.check("gr_loss_weights",
            L.load().gr_loss_weights(kinds[kind], _ptr(proj), _ptr(target), None if bg_t is None else _ptr(bg_t),
                                     0.0 if bg_t is not None else float(background), proj.numel(), _ptr(weight),
                                     _ptr(loss), _stream(dev)))
    return weight, loss


ADAM_GROUPS = ("mean", "scale", "quat", "density")


def adam_gaussians(theta: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                   natural: torch.Tensor, step: int, lr, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8) -> None:
    """One fused Adam step on an (11, n) scene (gr_adam_gaussians): rows mean
    (0-2), log-scale (3-5), quaternion (6-9), log-density (10) of theta; grad
    is dL/d natural; natural is rewritten with the updated parameters. lr is a
    float or a dict over mean/scale/quat/density."""
    dev = theta.device
    if theta.dim() != 2 or theta.shape[0] != 11:
        raise ValueError(f"theta must be (11, n), got {tuple(theta.shape)}")
    shape = tuple(theta.shape)
    for t, nm in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v"), (natural, "natural")):
        _require(t, nm, shape, dev)
    lrs = [float(lr[k]) for k in ADAM_GROUPS] if isinstance(lr, dict) else [float(lr)] * 4
    hp = L.GrGaussAdam((ctypes.c_float * 4)(*lrs), float(beta1), float(beta2), float(eps), 0, int(step))
    L.check("gr_adam_gaussians", L.load().gr_adam_gaussians(shape[1], _ptr(theta), _ptr(grad), _ptr(m), _ptr(v),
                                                            _ptr(natural), ctypes.byref(hp), _stream(dev)))


def _ct_struct(g: Dict) -> L.GrCtGeom:
    return L.GrCtGeom(int(g["cone"]), int(g["n_views"]), int(g["nu"]), int(g["nv"]),
                      float(g["angle0"]), float(g["angle_range"]), float(g.get("dso", 0.0)),
                      float(g.get("dsd", 0.0)), float(g["pitch_u"]), float(g["pitch_v"]),
                      float(g.get("offset_u", 0.0)), float(g.get("offset_v", 0.0)),
                      int(g.get("tile_u", 8)), int(g.get("tile_v", 8)))


def _pet_struct(g: Dict, planes: Optional[torch.Tensor]) -> L.GrPetGeom:
    return L.GrPetGeom(float(g["ring_radius"]), float(g["ring_pitch"]), int(g["n_crystals"]),
                       int(g["n_rings"]), int(g["n_radial"]), int(g["n_views"]),
                       int(g["max_ring_diff"]), int(g.get("arc_correct", 1)),
                       None if planes is None else planes.data_ptr(),
                       0 if planes is None else int(planes.shape[0]),
                       int(g.get("tile_radial", 8)), int(g.get("tile_axial", 8)), int(g.get("tile_views", 1)))


def ray_count(g: Dict, planes: Optional[torch.Tensor] = None) -> int:
    out = ctypes.c_int64()
    lib = L.load()
    if g["kind"] == "ct":
        L.check("gr_rays_count_ct", lib.gr_rays_count_ct(ctypes.byref(_ct_struct(g)), ctypes.byref(out)))
    else:
        L.check("gr_rays_count_pet",
                lib.gr_rays_count_pet(ctypes.byref(_pet_struct(g, planes)), ctypes.byref(out)))
    return int(out.value)


def make_rays(g: Dict, device="cuda", planes: Optional[torch.Tensor] = None,
              out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None
              ) -> Tuple[torch.Tensor, torch.Tensor]:
    """Rays of a CT (kind "ct") or PET (kind "pet") geometry, SoA (3, m) each."""
    device = torch.device(device)
    if device.type == "cuda" and device.index is None:
        device = torch.device("cuda", torch.cuda.current_device())
    if planes is not None:
        _require(planes, "planes", (int(planes.shape[0]), 2), device, torch.int32)
    m = ray_count(g, planes)
    if out is None:
        o = torch.empty(3, m, device=device)
        d = torch.empty(3, m, device=device)
    else:
        o, d = out
        _require(o, "ray_o", (3, m), device)
        _require(d, "ray_d", (3, m), device)
    lib = L.load()
    if g["kind"] == "ct":
        L.check("gr_make_rays_ct", lib.gr_make_rays_ct(ctypes.byref(_ct_struct(g)), _ptr(o), _ptr(d),
                                                       _stream(device)))
    else:
        L.check("gr_make_rays_pet_arccorr",
                lib.gr_make_rays_pet_arccorr(ctypes.byref(_pet_struct(g, planes)), _ptr(o), _ptr(d),
                                             _stream(device)))
    return o, d


class GaussianProjection(torch.autograd.Function):
    """I = GaussianProjection.apply(mean, scale, quat, density, rays_o, rays_d, kappa, leaf_size).

    The forward builds the acceleration structure and projects; only the
    scene (parameters and workspace) and the rays are saved. The backward
    re-traverses (hit lists are recomputed, not stored) through
    gr_project_backward. Gradients flow to mean, scale, quat and density;
    rays, kappa and leaf_size get none. Parameter activations (exp, softplus,
    ...) belong outside, in ordinary torch code."""

    @staticmethod
    def forward(ctx, mean, scale, quat, density, rays_o, rays_d, kappa=3.0, leaf_size=0):
        scene = Scene(mean.detach().contiguous(), scale.detach().contiguous(),
                      quat.detach().contiguous(), density.detach().contiguous(), kappa, leaf_size)
        ro = rays_o.detach().contiguous()
        rd = rays_d.detach().contiguous()
        out = project(scene, ro, rd)
        ctx.scene = scene
        ctx.save_for_backward(ro, rd)
        return out

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_out):
        ro, rd = ctx.saved_tensors
        g = project_backward(ctx.scene, ro, rd, grad_out.contiguous().float())
        ctx.scene = None
        return g["mean"], g["scale"], g["quat"], g["density"], None, None, None, None


def gaussian_projection(mean, scale, quat, density, rays_o, rays_d, kappa: float = 3.0,
                        leaf_size: int = 0) -> torch.Tensor:
    return GaussianProjection.apply(mean, scale, quat, density, rays_o, rays_d, kappa, leaf_size)
