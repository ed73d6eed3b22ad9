"""Reconstruction loop around the projector (Fig. 1): optimise the Gaussians so
that their projections match measured projections, with Adam (Sec. 4.1), then
voxelise them and compare volumes with 3D PSNR and 3D SSIM (the CT metrics of
the paper's evaluation).

Every step on the device runs in libgr: the fused forward -> loss -> backward
pass (gr_project_backward), the acceleration-structure rebuild after each
update (gr_build_accel), the Adam step (gr_adam_gaussians) and the voxelisation
(gr_voxelize). Scales and densities are optimised through their logarithms
so that they stay positive; the fused Adam step (gr_adam_gaussians) applies
the chain rule of that reparametrisation and writes the parameters the next
projection reads. Densify-and-prune (the R2-Gaussian rules
the paper reuses) is not part of this loop.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import torch

from . import api


def psnr3d(x: torch.Tensor, ref: torch.Tensor, data_range: Optional[float] = None) -> float:
    """10 log10(R^2 / MSE) with R the reference's value range (max - min)."""
    x = x.double()
    ref = ref.double()
    r = float(ref.max() - ref.min()) if data_range is None else float(data_range)
    mse = float(((x - ref) ** 2).mean())
    return math.inf if mse == 0.0 else 10.0 * math.log10(r * r / mse)


def _gauss_window(size: int, sigma: float, device) -> torch.Tensor:
    t = torch.arange(size, dtype=torch.float64, device=device) - (size - 1) / 2.0
    g = torch.exp(-0.5 * (t / sigma) ** 2)
    g = g / g.sum()
    return g


def ssim3d(x: torch.Tensor, ref: torch.Tensor, data_range: Optional[float] = None, win: int = 7,
           sigma: float = 1.5) -> float:
    """Mean structural similarity over 3D Gaussian windows (Wang et al. 2004,
    with the separable window of size win and width sigma, K1 = 0.01, K2 =
    0.03, L the reference's value range), over the valid (unpadded) region."""
    x = x.double()[None, None]
    ref = ref.double()[None, None]
    r = float(ref.max() - ref.min()) if data_range is None else float(data_range)
    c1 = (0.01 * r) ** 2
    c2 = (0.03 * r) ** 2
    g = _gauss_window(win, sigma, x.device)

    def blur(v):
        v = torch.nn.functional.conv3d(v, g.view(1, 1, -1, 1, 1))
        v = torch.nn.functional.conv3d(v, g.view(1, 1, 1, -1, 1))
        return torch.nn.functional.conv3d(v, g.view(1, 1, 1, 1, -1))

    mx, my = blur(x), blur(ref)
    sxx = blur(x * x) - mx * mx
    syy = blur(ref * ref) - my * my
    sxy = blur(x * ref) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(s.mean())


class Reconstruction:
    """Gaussian parameters under optimisation, as (11, n) device arrays: theta
    (rows mean 0-2, log-scale 3-5, quaternion 6-9, log-density 10), its Adam
    moments, the gradient, and `natural`, the parameters the projector reads
    (a scene whose four arrays are row views of it)."""

    def __init__(self, mean: torch.Tensor, scale: torch.Tensor, quat: torch.Tensor, density: torch.Tensor,
                 kappa: float = 3.0, leaf_size: int = 0, rebuild_every: int = 8):
        n = int(density.shape[0])
        dev = density.device
        self.natural = torch.empty(11, n, device=dev)
        self.natural[0:3] = mean
        self.natural[3:6] = scale
        self.natural[6:10] = quat
        self.natural[10] = density
        self.theta = self.natural.clone()
        self.theta[3:6] = scale.log()
        self.theta[10] = density.log()
        self.grad = torch.empty_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step_count = 0
        self.kappa = kappa
        self.leaf_size = leaf_size
        self.scene = None
        self.scratch = None
        self.rebuild_every = max(1, int(rebuild_every))
        self.since_build = 0

    def params(self):
        x = self.natural
        return x[0:3], x[3:6], x[6:10], x[10]

    def build(self) -> api.Scene:
        """Brings the acceleration structure up to date with the current
        parameters: a full build every `rebuild_every` calls, a refit (same
        order and tree, new boxes) in between. The scene reads `natural` in
        place, so it stays bound across steps."""
        if self.scene is None:
            self.scene = api.Scene(*self.params(), kappa=self.kappa, leaf_size=self.leaf_size)
            self.since_build = 0
        elif self.since_build + 1 >= self.rebuild_every:
            self.scene.build()
            self.since_build = 0
        else:
            self.scene.refit()
            self.since_build += 1
        return self.scene

    def step(self, rays_o: torch.Tensor, rays_d: torch.Tensor, target: torch.Tensor, lr: Dict[str, float],
             loss: str = "l2", background: float = 0.0) -> float:
        """One iteration: rebuild or refit, fused forward -> loss -> backward,
        fused Adam.
        lr maps mean, log_scale, quat, log_density (or scale, density) to
        learning rates."""
        scene = self.build()
        n = self.theta.shape[1]
        if self.scratch is None:
            self.scratch = torch.empty((api.fused_scratch_bytes(n) + 3) // 4, device=self.theta.device)
        out_loss = torch.zeros(1, dtype=torch.float64, device=rays_o.device)
        g = self.grad
        api.project_backward(scene, rays_o, rays_d, loss=loss, target=target, background=background,
                             out_loss=out_loss, scratch=self.scratch,
                             grads={"mean": g[0:3], "scale": g[3:6], "quat": g[6:10], "density": g[10]})
        self.step_count += 1
        lrs = {k[4:] if k.startswith("log_") else k: float(x) for k, x in lr.items()}
        api.adam_gaussians(self.theta, self.grad, self.m, self.v, self.natural, self.step_count, lrs)
        return float(out_loss.item())

    def voxelize(self, origin, spacing, dims) -> torch.Tensor:
        return api.voxelize(self.build(), origin, spacing, dims)


def reconstruct(target_scene: api.Scene, init: Reconstruction, rays_o: torch.Tensor, rays_d: torch.Tensor,
                iters: int, lr: Dict[str, float], loss: str = "l2") -> List[float]:
    """Fits init to the projections of target_scene along the given rays;
    returns the loss after every iteration."""
    target = api.project(target_scene, rays_o, rays_d)
    return [init.step(rays_o, rays_d, target, lr, loss=loss) for _ in range(iters)]
