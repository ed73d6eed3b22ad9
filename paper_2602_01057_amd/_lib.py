"""ctypes view of the libgr C ABI (include/gr.h). Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# GR_LIB_PATH selects another build of the same library (the host-sanitized
# copy used by the ABI tests); there is no implementation other than libgr.
LIB_PATH = os.environ.get("GR_LIB_PATH") or os.path.join(_PKG, "libgr.so")

GR_OK = 0
GR_E_ARG = -1
GR_E_WORKSPACE = -2
GR_E_HIP = -3
GR_E_UNSUPPORTED = -4
GR_E_STATE = -5
GR_LOSS_NONE, GR_LOSS_L2, GR_LOSS_POISSON = 0, 1, 2
GR_MAX_SEGMENTS = 32
GR_STATIC_SCRATCH_BYTES = 128 << 20
GR_MAX_SCENES = 8


class GrScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("density", ctypes.c_void_p), ("kappa", ctypes.c_float),
                ("leaf_size", ctypes.c_int32), ("accel", ctypes.c_void_p),
                ("accel_bytes", ctypes.c_size_t)]


class GrLaunch(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("persistent_groups", ctypes.c_int32), ("traversal", ctypes.c_int32),
                ("work_counter", ctypes.c_void_p), ("hit_list_cap", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class GrSegment(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ray_o", ctypes.c_void_p), ("ray_d", ctypes.c_void_p), ("stride", ctypes.c_int64),
                ("ray_offset", ctypes.c_int64), ("n_rays", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("out_offset", ctypes.c_int64)]


class GrLoss(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("background", ctypes.c_float),
                ("target", ctypes.c_void_p), ("out_proj", ctypes.c_void_p),
                ("out_loss", ctypes.c_void_p)]


class GrBwdSegment(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("loss_kind", ctypes.c_int32),
                ("ray_o", ctypes.c_void_p), ("ray_d", ctypes.c_void_p), ("stride", ctypes.c_int64),
                ("ray_offset", ctypes.c_int64), ("n_rays", ctypes.c_int64),
                ("target", ctypes.c_void_p), ("out_proj", ctypes.c_void_p), ("out_offset", ctypes.c_int64),
                ("accum", ctypes.c_void_p), ("out_loss", ctypes.c_void_p), ("background", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class GrCtGeom(ctypes.Structure):
    _fields_ = [("cone", ctypes.c_int32), ("n_views", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("angle0", ctypes.c_double),
                ("angle_range", ctypes.c_double), ("dso", ctypes.c_double),
                ("dsd", ctypes.c_double), ("pitch_u", ctypes.c_double),
                ("pitch_v", ctypes.c_double), ("offset_u", ctypes.c_double),
                ("offset_v", ctypes.c_double), ("tile_u", ctypes.c_int32),
                ("tile_v", ctypes.c_int32)]


class GrPetGeom(ctypes.Structure):
    _fields_ = [("ring_radius", ctypes.c_double), ("ring_pitch", ctypes.c_double),
                ("n_crystals", ctypes.c_int32), ("n_rings", ctypes.c_int32),
                ("n_radial", ctypes.c_int32), ("n_views", ctypes.c_int32),
                ("max_ring_diff", ctypes.c_int32), ("arc_correct", ctypes.c_int32),
                ("planes", ctypes.c_void_p), ("n_planes", ctypes.c_int32),
                ("tile_radial", ctypes.c_int32), ("tile_axial", ctypes.c_int32),
                ("tile_views", ctypes.c_int32)]


class GrGrid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("dims", ctypes.c_int64 * 3)]


class GrAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int64)]


class GrTof(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("sigma", ctypes.c_float), ("bin_width", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("center", ctypes.c_void_p), ("atten", ctypes.c_void_p)]


GR_TOF_MAX_BINS = 32


class GrGaussAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 4), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("reserved", ctypes.c_int32), ("step", ctypes.c_int64)]


# name -> (restype, argtypes); every exported symbol of gr.h
_P = ctypes.POINTER
_VP = ctypes.c_void_p
SIGNATURES = {
    "gr_voxelize": (ctypes.c_int32, [_P(GrScene), _P(GrGrid), _VP, _VP, _VP]),
    "gr_voxelize_stats": (ctypes.c_int32, [_P(GrScene), _P(GrGrid), _VP, _VP, _VP, _VP]),
    "gr_adam_step": (ctypes.c_int32, [_VP, _VP, _VP, _VP, ctypes.c_int64, _P(GrAdam), _VP]),
    "gr_adam_gaussians": (ctypes.c_int32, [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _P(GrGaussAdam), _VP]),
    "gr_project_tof": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _P(GrTof), _VP, _P(GrLaunch),
                                        _VP]),
    "gr_project_tof_backward": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _P(GrTof), _VP, _VP, _VP,
                                                 _VP, _VP, _VP, ctypes.c_size_t, _P(GrLaunch), _VP]),
    "gr_tof_centers": (ctypes.c_int32, [_VP, _VP, ctypes.c_int64, _VP, _VP]),
    "gr_loss_weights": (ctypes.c_int32, [ctypes.c_int32, _VP, _VP, _VP, ctypes.c_float, ctypes.c_int64, _VP, _VP,
                                         _VP]),
    "gr_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "gr_abi_version": (ctypes.c_int32, []),
    "gr_accel_bytes": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_size_t)]),
    "gr_build_accel": (ctypes.c_int32, [_P(GrScene), _VP]),
    "gr_refit_accel": (ctypes.c_int32, [_P(GrScene), _VP]),
    "gr_scene_invalid_count": (ctypes.c_int32, [_P(GrScene), _P(ctypes.c_int64), _VP]),
    "gr_scene_status": (ctypes.c_int32, [_P(GrScene), _P(ctypes.c_int32), _VP]),
    "gr_project": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _VP, _P(GrLaunch), _VP]),
    "gr_project_stats": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _VP, _VP,
                                          _P(GrLaunch), _VP]),
    "gr_project_batched": (ctypes.c_int32, [_P(GrScene), ctypes.c_int32, _P(GrSegment),
                                            ctypes.c_int32, _P(GrLaunch), _VP]),
    "gr_backward_scratch_bytes": (ctypes.c_int32, [ctypes.c_int64, _P(ctypes.c_size_t)]),
    "gr_fused_scratch_bytes": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_void_p, _P(ctypes.c_size_t)]),
    "gr_project_backward": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _VP,
                                             _P(GrLoss), _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                             _P(GrLaunch), _VP]),
    "gr_project_backward_static": (ctypes.c_int32, [_P(GrScene), _VP, _VP, ctypes.c_int64, _VP, _P(GrLoss),
                                                    _VP, _VP, _VP, _VP, _P(GrLaunch), _VP]),
    "gr_backward_accum_zero": (ctypes.c_int32, [ctypes.c_int64, _VP, _VP]),
    "gr_project_backward_batched": (ctypes.c_int32, [_P(GrScene), ctypes.c_int32, _P(GrBwdSegment),
                                                     ctypes.c_int32, _VP, ctypes.c_size_t, _P(GrLaunch), _VP]),
    "gr_backward_finish": (ctypes.c_int32, [_P(GrScene), _VP, _VP, _VP, _VP, _VP, _VP]),
    "gr_rays_count_ct": (ctypes.c_int32, [_P(GrCtGeom), _P(ctypes.c_int64)]),
    "gr_rays_count_pet": (ctypes.c_int32, [_P(GrPetGeom), _P(ctypes.c_int64)]),
    "gr_make_rays_ct": (ctypes.c_int32, [_P(GrCtGeom), _VP, _VP, _VP]),
    "gr_make_rays_pet_arccorr": (ctypes.c_int32, [_P(GrPetGeom), _VP, _VP, _VP]),
}

_lib = None


class GrError(RuntimeError):
    def __init__(self, fn: str, code: int, text: str):
        super().__init__(f"{fn} failed: {text} ({code})")
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgr.so (built in-tree by build_lib.py). Raises if it is absent:
    there is no other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgr is not built ({path} missing); run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch bundles its own HIP runtime; it must be loaded first so that libgr
    # binds to the same runtime instance instead of bringing in a second one
    # (pointers and streams from one runtime are invalid in the other)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, code: int) -> None:
    if code != GR_OK:
        text = load().gr_status_str(code).decode()
        raise GrError(fn, code, text)
