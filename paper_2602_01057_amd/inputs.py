"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random scenes and holds the named workload presets (sizes and
scanner parameters). It contains none of the projection method's arithmetic: no
rotation matrices, no covariances, no ray geometry, no line integrals. Both the
HIP path and the FP64 oracle receive the arrays it returns as plain inputs.

Scene recipe (drawn in FP64 with numpy's PCG64 ``default_rng(seed)``, in this
order, then cast to FP32):
  1. means: uniform in a ball (or a z-aligned cylinder) by rejection sampling
     from its bounding box, in batches;
  2. scales: per axis, independently log-uniform in [s_lo, s_hi];
  3. quaternions (w, x, y, z): a 4-D standard normal draw divided by its norm,
     i.e. uniform on the 3-sphere;
  4. densities: uniform in [0, 1).

The Gaussian parameterisation (mean, scale, rotation, peak density) is the one
of Sec. 3.1 (Eq. 2 and the factorisation of the covariance into rotation and
scale); the densities are peak values because the normalisation is absorbed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Scene:
    """SoA FP32 Gaussian parameters: mean/scale are (3, n), quat is (4, n) as
    (w, x, y, z), density is (n,)."""

    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    density: np.ndarray

    @property
    def n(self) -> int:
        return int(self.density.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx].copy(), self.scale[:, idx].copy(),
                     self.quat[:, idx].copy(), self.density[idx].copy())


def _sample_points(rng, n: int, region: str, radius: float, half_len: float) -> np.ndarray:
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(1024, int(1.5 * (n - out.shape[0])) + 16)
        if region == "ball":
            c = rng.uniform(-radius, radius, size=(m, 3))
            keep = (c * c).sum(axis=1) <= radius * radius
        elif region == "cylinder":
            c = np.empty((m, 3))
            c[:, 0:2] = rng.uniform(-radius, radius, size=(m, 2))
            c[:, 2] = rng.uniform(-half_len, half_len, size=m)
            keep = (c[:, 0:2] ** 2).sum(axis=1) <= radius * radius
        else:
            raise ValueError(f"unknown region {region!r}")
        out = np.concatenate([out, c[keep]], axis=0)
    return out[:n]


def sample_scene(n: int, seed: int, *, region: str = "ball", radius: float = 100.0,
                 length: float = 0.0, scale_range: Tuple[float, float] = (1.5, 12.0),
                 density_range: Tuple[float, float] = (0.0, 1.0)) -> Scene:
    """Draw ``n`` Gaussians with the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    means = _sample_points(rng, n, region, radius, 0.5 * length)
    lo, hi = scale_range
    scales = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n, 3)))
    q = rng.standard_normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    dens = rng.uniform(density_range[0], density_range[1], size=n)
    return Scene(np.ascontiguousarray(means.T, dtype=np.float32),
                 np.ascontiguousarray(scales.T, dtype=np.float32),
                 np.ascontiguousarray(q.T, dtype=np.float32),
                 np.ascontiguousarray(dens, dtype=np.float32))


def sample_unit_weights(n: int, seed: int) -> np.ndarray:
    """Seeded per-ray loss weights (dL/dI) in [-1, 1), FP32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=n).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads. Numbers are the scanner and scene sizes of the benchmark
# configurations; geometry fields use the names of the C geometry structs.
# ---------------------------------------------------------------------------

CT_PARALLEL_SMALL: Dict = dict(
    name="parallel-beam CT, 512 Gaussians, 32 views x 64x64 at 4 mm",
    scene=dict(n=512, seed=0, region="ball", radius=100.0, scale_range=(1.5, 12.0)),
    geom=dict(kind="ct", cone=0, n_views=32, nu=64, nv=64, angle0=0.0, angle_range=math.pi,
              dso=0.0, dsd=0.0, pitch_u=4.0, pitch_v=4.0, offset_u=0.0, offset_v=0.0,
              tile_u=8, tile_v=8),
)

CT_CONE_50K: Dict = dict(
    name="cone-beam CT, 50k Gaussians, 50 views x 256x256 at 1.6 mm",
    scene=dict(n=50_000, seed=0, region="ball", radius=100.0, scale_range=(0.8, 6.0)),
    target_seed=1,
    geom=dict(kind="ct", cone=1, n_views=50, nu=256, nv=256, angle0=0.0, angle_range=2 * math.pi,
              dso=1000.0, dsd=1500.0, pitch_u=1.6, pitch_v=1.6, offset_u=0.0, offset_v=0.0,
              tile_u=8, tile_v=8),
)

PET_200K: Dict = dict(
    name="cylindrical PET, 200k Gaussians, 344 radial x 252 angles x 752 planes",
    scene=dict(n=200_000, seed=0, region="cylinder", radius=300.0, length=250.0,
               scale_range=(1.0, 8.0)),
    target_seed=1,
    geom=dict(kind="pet", ring_radius=400.0, ring_pitch=4.0, n_crystals=504, n_rings=32,
              n_radial=344, n_views=252, max_ring_diff=15, arc_correct=1,
              tile_radial=8, tile_axial=1, tile_views=8),
)

CT_CONE_500K: Dict = dict(
    name="cone-beam CT, 500k Gaussians, 360 views x 512x512 at 0.8 mm",
    scene=dict(n=500_000, seed=0, region="ball", radius=100.0, scale_range=(0.5, 4.0)),
    geom=dict(kind="ct", cone=1, n_views=360, nu=512, nv=512, angle0=0.0, angle_range=2 * math.pi,
              dso=1000.0, dsd=1500.0, pitch_u=0.8, pitch_v=0.8, offset_u=0.0, offset_v=0.0,
              tile_u=8, tile_v=8),
)

PRESETS = {
    "ct_parallel_512": CT_PARALLEL_SMALL,
    "ct_cone_50k": CT_CONE_50K,
    "pet_200k": PET_200K,
    "ct_cone_500k": CT_CONE_500K,
}


def preset_scene(preset: Dict, seed: Optional[int] = None, n: Optional[int] = None) -> Scene:
    kw = dict(preset["scene"])
    if seed is not None:
        kw["seed"] = seed
    if n is not None:
        kw["n"] = n
    n_ = kw.pop("n")
    seed_ = kw.pop("seed")
    return sample_scene(n_, seed_, **kw)

