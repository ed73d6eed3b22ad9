"""MI355X (gfx950) ray / 3D-Gaussian line-integral projector.

The compute path is the HIP library libgr (csrc/, C ABI in include/gr.h);
``api`` is its torch binding, ``tune`` the launch autotuner, ``serve`` the
continuous-batching request server, ``inputs`` the seeded synthetic inputs.
Importing the package does not import torch; the binding loads on first use.
"""
from __future__ import annotations

import importlib

__all__ = ["Scene", "project", "project_stats", "project_batched", "project_backward", "make_rays", "ray_count",
           "GaussianProjection", "gaussian_projection", "accel_bytes", "backward_scratch_bytes",
           "fused_scratch_bytes", "voxelize", "voxelize_stats", "adam_step", "adam_gaussians",
           "project_tof", "project_tof_backward", "tof_centers", "loss_weights",
           "project_backward_batched", "backward_accum_zero", "backward_finish", "project_backward_static",
           "load_library"]


def load_library():
    """Load libgr.so, raising if it is not built."""
    from . import _lib
    return _lib.load()


def __getattr__(name):
    if name in __all__:
        api = importlib.import_module(".api", __name__)
        return getattr(api, name)
    raise AttributeError(name)
