"""Autotuner for the projector's build and launch parameters.

Searched knobs:
  leaf        Gaussians per LBVH leaf (build parameter)            16, 32, 64
  waves       waves (64-ray packets) per workgroup                  1, 2, 4
  remap       XCD-aware packet order (1) or plain dispatch order (2)
  persistent  one wave per packet (0) or persistent waves pulling packets (1)
  traversal   binary LBVH with per-ray slab tests (1) or the 64-wide hierarchy
              with beam tests (2)
  tile        packet shape of the ray generators: tile_u x tile_v for CT
              (8x8, 16x4, 4x16); tile_radial x tile_axial x tile_views
              for PET (8x8x1, 8x2x4, 4x4x4, 8x1x8)

Each candidate is timed with HIP events on the real scene and rays (or on a
contiguous slice of the views when ``max_rays`` is given), median of a few
repetitions, after one warm-up call. Results are cached in a JSON file
(``GR_TUNE_CACHE`` or ~/.cache/gaussray/tune.json) keyed by GPU architecture,
compute-unit count, geometry kind, operation and power-of-two buckets of the
Gaussian and ray counts, so later runs of similar workloads skip the search.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import statistics
from typing import Dict, Iterable, Optional

import torch

from . import api

# "tile": None = the geometry kind's default packet shape (DEFAULT_TILE)
DEFAULT = {"leaf": 64, "waves": 1, "remap": 1, "persistent": 0, "traversal": 2, "tile": None}
DEFAULT_TILE = {"ct": [8, 8], "pet": [8, 1, 8]}
SEARCH = {"leaf": [16, 32, 64], "waves": [1, 2, 4], "remap": [1, 2], "persistent": [0, 1],
          "traversal": [1, 2], "tile": None}
SEARCH_TILE = {"ct": [[8, 8], [16, 4], [4, 16]], "pet": [[8, 8, 1], [8, 2, 4], [4, 4, 4], [8, 1, 8]]}
# The fused forward -> loss -> backward pass with hit lists is always a
# persistent launch, so the grid-launch knobs (remap, persistent) do not apply.
SEARCH_FUSED = {"leaf": [32, 64], "waves": [1, 2], "remap": [1], "persistent": [0], "traversal": [1, 2],
                "tile": None}
# Timing noise between near-equal configurations: the default configuration is
# kept unless another one is faster by more than this fraction, so that
# repeated tuning runs settle on the same configuration.
KEEP_DEFAULT_WITHIN = 0.05


def cache_path() -> str:
    return os.environ.get("GR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gaussray", "tune.json"))


def _bucket(x: int) -> int:
    return int(math.floor(math.log2(max(1, x))))


def device_tag(device) -> str:
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "gpu").split(":")[0]
    return f"{arch}|cu{p.multi_processor_count}"


def cache_key(device, kind: str, op: str, n: int, m: int) -> str:
    tag = device if isinstance(device, str) else device_tag(device)
    return f"{tag}|{kind}|{op}|n2^{_bucket(n)}|m2^{_bucket(m)}"


def load_cache() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(key: str, cfg: Dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    c = load_cache()
    c[key] = cfg
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(device, kind: str, op: str, n: int, m: int) -> Dict:
    """Cached configuration for this workload bucket, else the defaults."""
    return dict(load_cache().get(cache_key(device, kind, op, n, m), DEFAULT))


def _time(fn, reps: int = 3) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def _pet_planes(g: Dict, count: int):
    """The first ``count`` ring pairs in the generators' default order (ring
    difference 0, +1, -1, +2, -2, ..., r1 ascending within a difference)."""
    out = []
    n, dmax = int(g["n_rings"]), int(g["max_ring_diff"])
    for dd in [0] + [s * d for d in range(1, dmax + 1) for s in (1, -1)]:
        for r1 in range(n):
            if 0 <= r1 + dd < n:
                out.append((r1, r1 + dd))
                if len(out) == count:
                    return out
    return out


def _slice_geom(geom: Dict, max_rays: Optional[int]):
    """A slice of the geometry holding about max_rays rays, and the PET ring
    pairs it uses (None: the geometry's own). CT keeps the views that fit. PET
    keeps every view, since the views' angular spacing is set by their count
    and view-blocked packets depend on it, and takes whole blocks of 8
    (the tallest axial tile searched) of the default ring pairs instead."""
    g = dict(geom)
    if not max_rays:
        return g, None
    if g["kind"] == "pet":
        per = int(g["n_radial"]) * int(g["n_views"])
        total = len(_pet_planes(g, 1 << 30))
        blk = max(t[1] for t in SEARCH_TILE["pet"])
        k = max(1, min(total, max_rays // max(1, per)))
        if k < total:
            k = min(total, max(blk, (k // blk) * blk))
        return g, (None if k == total else _pet_planes(g, k))
    per = api.ray_count(dict(g, n_views=1), None)
    g["n_views"] = max(1, min(int(g["n_views"]), max_rays // max(1, per)))
    return g, None


def _tile_keys(kind: str):
    return ("tile_u", "tile_v") if kind == "ct" else ("tile_radial", "tile_axial", "tile_views")


def _tile_fields(kind: str, tile) -> Dict:
    """Geometry fields of a packet shape (a PET shape of two numbers has one
    view per tile)."""
    t = [int(x) for x in tile] + [1] * (len(_tile_keys(kind)) - len(tile))
    return dict(zip(_tile_keys(kind), t))


def tune(params, geom: Dict, op: str = "fwd", kappa: float = 3.0, max_rays: Optional[int] = 2_000_000,
         search: Optional[Dict[str, Iterable]] = None, reps: int = 3, save: bool = True,
         log=None) -> Dict:
    """Search the knobs for a scene (mean, scale, quat, density tensors) and a
    geometry dict, for op "fwd" (gr_project) or "bwd" (fused L2 backward).
    Returns the best configuration with its time; stores it in the cache."""
    sp = dict(SEARCH)
    if search:
        sp.update({k: (None if v is None else list(v)) for k, v in search.items()})
    dev = params[0].device
    kind = geom["kind"]
    g, planes = _slice_geom(geom, max_rays)
    if planes is not None:
        planes = torch.tensor(planes, dtype=torch.int32, device=dev)
    results = []
    target = None
    for tile in (sp["tile"] or SEARCH_TILE[kind]):
        gt = dict(g, **_tile_fields(kind, tile))
        ro, rd = api.make_rays(gt, dev, planes=planes)
        m = ro.shape[1]
        out = torch.empty(m, device=dev)
        if op == "bwd" and (target is None or target.numel() != m):
            target = torch.zeros(m, device=dev)
        for leaf in sp["leaf"]:
            scene = api.Scene(*params, kappa=kappa, leaf_size=leaf)
            for waves, remap, pers, trav in itertools.product(sp["waves"], sp["remap"], sp["persistent"],
                                                              sp["traversal"]):
                scratch = None if op == "fwd" else torch.empty(
                    api.fused_scratch_bytes(scene.n, waves) // 4, device=dev)
                if pers and remap == 2:
                    continue  # the remap does not apply to persistent launches
                kw = dict(waves_per_group=waves, xcd_remap=remap, persistent=bool(pers), traversal=trav)
                if op == "fwd":
                    fn = lambda: api.project(scene, ro, rd, out=out, **kw)  # noqa: E731
                else:
                    fn = lambda: api.project_backward(scene, ro, rd, loss="l2", target=target,  # noqa: E731
                                                      scratch=scratch, **kw)
                t = _time(fn, reps)
                cfg = {"leaf": leaf, "waves": waves, "remap": remap, "persistent": int(pers),
                       "traversal": int(trav), "tile": [int(x) for x in tile], "ms": t, "rays_timed": m}
                results.append(cfg)
                if log:
                    log(cfg)
            if scene.status_flags() != 0:
                raise RuntimeError("device-side consistency check failed during tuning")
    best = min(results, key=lambda c: c["ms"])
    dtile = [int(x) for x in DEFAULT_TILE[kind]]
    for c in results:
        is_default = all(c[k] == DEFAULT[k] for k in ("leaf", "waves", "traversal")) and c["tile"] == dtile \
            and (op != "fwd" or (c["remap"] == DEFAULT["remap"] and c["persistent"] == DEFAULT["persistent"]))
        if is_default and c["ms"] <= best["ms"] * (1.0 + KEEP_DEFAULT_WITHIN):
            best = c
            break
    if save:
        n = int(params[3].shape[0])
        store(cache_key(dev, kind, op, n, api.ray_count(geom)), best)
    return best


def launch_kwargs(cfg: Dict) -> Dict:
    """Keyword arguments of api.project / project_backward for a configuration."""
    return {"waves_per_group": int(cfg.get("waves", 1)), "xcd_remap": int(cfg.get("remap", 1)),
            "persistent": bool(cfg.get("persistent", 0)), "traversal": int(cfg.get("traversal", 2))}


def apply_tile(geom: Dict, cfg: Dict) -> Dict:
    kind = geom["kind"]
    t = cfg.get("tile") or DEFAULT_TILE[kind]
    return dict(geom, **_tile_fields(kind, t))
