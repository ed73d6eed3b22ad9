"""FP64 CPU oracle for the ray / 3D-Gaussian line-integral projector.

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import this package. The HIP library
never calls it, and the two share no code: the oracle is plain C (gr_oracle.c,
brute force over every ray and every Gaussian in double precision) plus the
numpy ray geometry in geometry.py.

What each function follows in the paper (Radioactive 3D Gaussian Ray Tracing):
  project    -- Eq. 7 (A, B, C), Eq. 11 (single closed form), Eq. 12 (sum);
                the kappa cutoff reads the unstated "negligible" rule of
                Sec. 4.1 as D <= kappa^2.
  grad       -- derivative of Eq. 11 (the paper calls the projection
                differentiable but derives no gradient; see gr_oracle.c).
  pair_values-- Eq. 11 for one Gaussian, for finite differences.
  voxelize   -- the mixture density at voxel centres (Fig. 1: the reconstruction
                is the voxelised Gaussians; Eq. 2 field, same kappa cutoff).
  adam       -- one Adam step (the optimiser of Sec. 4.1); adam_gaussians the
                step on a scene's eleven parameter rows.
  project_tof, grad_tof
             -- time-of-flight bins and attenuation, the projector extensions
                the paper names as future work (Sec. 5): the TOF kernel's
                quadratic added to the Gaussian's keeps Eq. 11's closed form.
  loss_weights
             -- L2 and Poisson losses and their weights dL/dI.
  geometry   -- ray set-up from scanner geometry (Fig. 1, Fig. 2, Sec. 3), and
                the TOF centres of PET lines.
Pins that tie these to the mathematics rather than to themselves live in
tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

from . import geometry  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "gr_oracle.c")
    if (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_project.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, _D, _D, _D, _D, _D, _D, _I64, ctypes.c_int]
    lib.orc_project.restype = ctypes.c_int
    lib.orc_pair_values.argtypes = [_D, ctypes.c_int64, _D, _D, _D, _D]
    lib.orc_pair_values.restype = ctypes.c_int
    lib.orc_grad.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int64, _D, _D, _D, _I64, ctypes.c_int64, _D, _D, _D,
                             ctypes.c_int]
    lib.orc_grad.restype = ctypes.c_int
    lib.orc_precision.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _D]
    lib.orc_precision.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_voxelize.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                 _D, _D, _I64, _D, _D, _D, _D, _I64, ctypes.c_int]
    lib.orc_voxelize.restype = ctypes.c_int
    lib.orc_adam.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int64]
    lib.orc_adam.restype = None
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_project_tof.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int64, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    _D, _D, _D, _D, _D, _D, ctypes.c_int]
    lib.orc_project_tof.restype = ctypes.c_int
    lib.orc_grad_tof.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int64, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 _D, _D, _D, _I64, ctypes.c_int64, _D, _D, _D, ctypes.c_int]
    lib.orc_grad_tof.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a, shape=None) -> np.ndarray:
    """Exact cast to a C-contiguous float64 array (FP32 inputs are exact in FP64)."""
    out = np.ascontiguousarray(np.asarray(a), dtype=np.float64)
    if shape is not None:
        out = out.reshape(shape)
    return out


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_D if a.dtype == np.float64 else _I64)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _scene_arrays(scene):
    n = int(np.asarray(scene.density).shape[0])
    return (n, _f64(scene.mean, (3, n)), _f64(scene.scale, (3, n)), _f64(scene.quat, (4, n)),
            _f64(scene.density, (n,)))


def project(scene, ray_o, ray_d, kappa: float = 3.0, tau: float = 1e-5, nthreads: int = 0
            ) -> Dict[str, np.ndarray]:
    """Brute-force FP64 projection of every ray through every Gaussian.

    ``scene`` has SoA arrays mean (3,n), scale (3,n), quat (4,n) as (w,x,y,z),
    density (n,). Rays are SoA (3, m). Returns a dict with I_kappa, I_inf,
    I_in, I_hi (float64 (m,)) and hits (int64 (m,)); see gr_oracle.c.
    """
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    ro = _f64(ray_o)
    m = ro.size // 3
    ro = ro.reshape(3, m)
    rd = _f64(ray_d, (3, m))
    out = {k: np.empty(m, dtype=np.float64) for k in ("I_kappa", "I_inf", "I_in", "I_hi")}
    hits = np.empty(m, dtype=np.int64)
    rc = lib.orc_project(n, _p(mean), _p(scale), _p(quat), _p(dens), float(kappa), float(tau),
                         m, _p(ro), _p(rd), _p(out["I_kappa"]), _p(out["I_inf"]), _p(out["I_in"]),
                         _p(out["I_hi"]), hits.ctypes.data_as(_I64), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle projection failed")
    out["hits"] = hits
    return out


def voxelize(scene, origin, spacing, dims, kappa: float = 3.0, tau: float = 1e-5, nthreads: int = 0
             ) -> Dict[str, np.ndarray]:
    """Brute-force FP64 voxelisation of the Gaussian mixture (Fig. 1; Eq. 2):
    V at voxel centres origin + (ix, iy, iz) * spacing, as arrays of shape
    (nz, ny, nx): V (kappa cutoff), V_inf, V_in, V_hi; see gr_oracle.c. Also
    "pairs_in" / "pairs_hi": the (voxel, Gaussian) pairs with D within
    kappa^2 (1 -+ tau)."""
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    nx, ny, nz = (int(x) for x in dims)
    o = _f64(origin, (3,))
    sp = _f64(spacing, (3,))
    dm = np.array([nx, ny, nz], dtype=np.int64)
    out = {k: np.empty((nz, ny, nx), dtype=np.float64) for k in ("V", "V_inf", "V_in", "V_hi")}
    counts = np.zeros(2, dtype=np.int64)
    rc = lib.orc_voxelize(n, _p(mean), _p(scale), _p(quat), _p(dens), float(kappa), float(tau), _p(o),
                          _p(sp), dm.ctypes.data_as(_I64), _p(out["V"]), _p(out["V_inf"]),
                          _p(out["V_in"]), _p(out["V_hi"]), counts.ctypes.data_as(_I64), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle voxelisation failed")
    out["pairs_in"], out["pairs_hi"] = int(counts[0]), int(counts[1])
    return out


def adam(p, g, m, v, lr: float, b1: float, b2: float, eps: float, step: int) -> None:
    """One Adam step in FP64, in place on float64 arrays p, m, v (Sec. 4.1)."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (p, g, m, v)]
    for a, b in zip(arrs, (p, g, m, v)):
        if a is not b:
            raise ValueError("adam updates contiguous float64 arrays in place")
    lib.orc_adam(p.size, _p(p), _p(g), _p(m), _p(v), float(lr), float(b1), float(b2), float(eps), int(step))


_GROUP_ROWS = ((0, 3), (3, 6), (6, 10), (10, 11))  # mean, scale, quaternion, density
_LOG_GROUPS = (1, 3)


def adam_gaussians(theta, grad, m, v, natural, lr, b1: float, b2: float, eps: float, step: int) -> None:
    """One Adam step on the (11, n) parameters of a scene, in FP64, in place.

    Rows: mean (0-2), log-scale (3-5), quaternion (6-9), log-density (10) of
    theta; grad is dL/d(natural parameter) and natural holds the parameters
    the projector used (scale and density positive). The step is the chain
    rule of the log reparametrisation (dL/dlog x = x dL/dx, from x = exp(t)),
    then Adam per group with lr[group] (Sec. 4.1), then natural rewritten from
    the updated theta."""
    for a in (theta, grad, m, v, natural):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.ndim == 2 and a.shape[0] == 11
                and a.flags.c_contiguous):
            raise ValueError("adam_gaussians updates contiguous (11, n) float64 arrays in place")
    for gi, (r0, r1) in enumerate(_GROUP_ROWS):
        t = theta[r0:r1].reshape(-1)  # views: adam updates them in place
        mm = m[r0:r1].reshape(-1)
        vv = v[r0:r1].reshape(-1)
        g = grad[r0:r1].reshape(-1)
        if gi in _LOG_GROUPS:
            g = g * natural[r0:r1].reshape(-1)
        adam(t, np.ascontiguousarray(g), mm, vv, lr[gi], b1, b2, eps, step)
        natural[r0:r1] = np.exp(theta[r0:r1]) if gi in _LOG_GROUPS else theta[r0:r1]


def project_tof(scene, ray_o, ray_d, n_bins: int, sigma: float = 0.0, bin_width: float = 0.0,
                center=None, atten=None, kappa: float = 3.0, tau: float = 1e-5, nthreads: int = 0
                ) -> Dict[str, np.ndarray]:
    """Time-of-flight PET projection with attenuation in FP64 (see
    orc_project_tof): arrays of shape (max(1, n_bins), m) for I_kappa, I_in,
    I_hi and I_inf. n_bins = 0: attenuation only."""
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    ro = _f64(ray_o)
    m = ro.size // 3
    ro = ro.reshape(3, m)
    rd = _f64(ray_d, (3, m))
    c = None if center is None else _f64(center, (m,))
    a = None if atten is None else _f64(atten, (m,))
    nb = max(1, int(n_bins))
    out = {k: np.empty((nb, m)) for k in ("I_kappa", "I_in", "I_hi", "I_inf")}
    rc = lib.orc_project_tof(n, _p(mean), _p(scale), _p(quat), _p(dens), float(kappa), float(tau), m,
                             _p(ro), _p(rd), int(n_bins), float(sigma), float(bin_width), _p(c), _p(a),
                             _p(out["I_kappa"]), _p(out["I_in"]), _p(out["I_hi"]), _p(out["I_inf"]),
                             int(nthreads))
    if rc == -2:
        raise ValueError("bad TOF parameters")
    if rc != 0:
        raise MemoryError("oracle TOF projection failed")
    return out


def grad_tof(scene, ray_o, ray_d, w, n_bins: int, sigma: float = 0.0, bin_width: float = 0.0,
             center=None, atten=None, sel=None, kappa: float = 3.0, tau: float = 1e-5,
             nthreads: int = 0) -> Dict[str, np.ndarray]:
    """Analytic gradient of L = sum w[b, r] I_b(r) of the TOF projection
    (orc_grad_tof); w has shape (max(1, n_bins), m). Same keys as grad()."""
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    ro = _f64(ray_o)
    m = ro.size // 3
    ro = ro.reshape(3, m)
    rd = _f64(ray_d, (3, m))
    nb = max(1, int(n_bins))
    ww = _f64(w, (nb, m))
    c = None if center is None else _f64(center, (m,))
    a = None if atten is None else _f64(atten, (m,))
    sl = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    k = n if sl is None else sl.size
    g = np.empty((k, 11))
    gabs = np.empty((k, 11))
    gband = np.empty((k, 11))
    rc = lib.orc_grad_tof(n, _p(mean), _p(scale), _p(quat), _p(dens), float(kappa), float(tau), m,
                          _p(ro), _p(rd), int(n_bins), float(sigma), float(bin_width), _p(c), _p(a), _p(ww),
                          None if sl is None else sl.ctypes.data_as(_I64), k, _p(g), _p(gabs), _p(gband),
                          int(nthreads))
    if rc == -2:
        raise ValueError("bad TOF parameters")
    if rc != 0:
        raise MemoryError("oracle TOF gradient failed")
    return _grad_dict(g, gabs, gband)


def loss_weights(kind: str, I, y, background=0.0):
    """Loss and per-measurement weight dL/dI in FP64: "l2" L = sum (I - y)^2 / 2,
    w = I - y; "poisson" L = sum (Ib - y log Ib), w = 1 - y / Ib with Ib = I +
    background (a scalar or an array: randoms and scatter as expected counts)."""
    I = np.asarray(I, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if kind == "l2":
        e = I - y
        return 0.5 * float((e * e).sum()), e
    if kind == "poisson":
        Ib = I + np.asarray(background, dtype=np.float64)
        return float((Ib - y * np.log(Ib)).sum()), 1.0 - y / Ib
    raise ValueError(kind)


def pair_values(theta, ray_o, ray_d):
    """T and D of one Gaussian (theta = mu(3), s(3), q(4) raw, rho) on each
    ray, without the cutoff."""
    lib = _load()
    th = _f64(theta, (11,))
    ro = _f64(ray_o)
    m = ro.size // 3
    ro = ro.reshape(3, m)
    rd = _f64(ray_d, (3, m))
    T = np.empty(m)
    D = np.empty(m)
    if lib.orc_pair_values(_p(th), m, _p(ro), _p(rd), _p(T), _p(D)) != 0:
        raise ValueError("invalid Gaussian parameters")
    return T, D


def grad(scene, ray_o, ray_d, w, sel=None, kappa: float = 3.0, tau: float = 1e-5,
         nthreads: int = 0) -> Dict[str, np.ndarray]:
    """Analytic gradient of L = sum_r w_r I_kappa(r) w.r.t. the raw parameters
    of the Gaussians in ``sel`` (default all). Returns dict with keys mean
    (k,3), scale (k,3), quat (k,4), density (k,), the same for the absolute
    per-pair sums (``abs_*``) and for boundary-band pairs (``band_*``)."""
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    ro = _f64(ray_o)
    m = ro.size // 3
    ro = ro.reshape(3, m)
    rd = _f64(ray_d, (3, m))
    wv = _f64(w, (m,))
    if sel is None:
        seli = None
        k = n
    else:
        seli = np.ascontiguousarray(np.asarray(sel), dtype=np.int64)
        k = seli.size
    g = np.zeros((k, 11))
    ga = np.zeros((k, 11))
    gb = np.zeros((k, 11))
    rc = lib.orc_grad(n, _p(mean), _p(scale), _p(quat), _p(dens), float(kappa), float(tau), m,
                      _p(ro), _p(rd), _p(wv), None if seli is None else seli.ctypes.data_as(_I64),
                      k, _p(g), _p(ga), _p(gb), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle gradient failed")
    return _grad_dict(g, ga, gb)


def _grad_dict(g, ga, gb):
    def split(a, pre):
        return {pre + "mean": a[:, 0:3], pre + "scale": a[:, 3:6], pre + "quat": a[:, 6:10],
                pre + "density": a[:, 10]}

    out = split(g, "")
    out.update(split(ga, "abs_"))
    out.update(split(gb, "band_"))
    out["flat"] = g
    out["flat_abs"] = ga
    out["flat_band"] = gb
    return out


def precision(scene):
    """Row-major P = Sigma^-1 and R per Gaussian, each (n, 3, 3)."""
    lib = _load()
    n, mean, scale, quat, dens = _scene_arrays(scene)
    P = np.empty((n, 3, 3))
    R = np.empty((n, 3, 3))
    lib.orc_precision(n, _p(mean), _p(scale), _p(quat), _p(dens), _p(P), _p(R))
    return P, R


def fd_linear(theta, ray_o, ray_d, w, include, rel_step: float = 1e-6) -> np.ndarray:
    """Central finite differences of L = sum_r w_r T_r(theta) over the rays in
    the frozen inclusion set ``include`` (bool mask), for one Gaussian with
    raw parameters theta (11,). Only the selected Gaussian's own terms enter,
    so no large total is differenced."""
    th = _f64(theta, (11,))
    w = _f64(w)
    inc = np.asarray(include, dtype=bool)
    ro = _f64(ray_o)[:, inc]
    rd = _f64(ray_d)[:, inc]
    wi = w[inc]
    out = np.zeros(11)
    for k in range(11):
        h = rel_step * max(1.0, abs(th[k]))
        tp = th.copy()
        tm = th.copy()
        tp[k] += h
        tm[k] -= h
        Tp, _ = pair_values(tp, ro, rd)
        Tm, _ = pair_values(tm, ro, rd)
        out[k] = float(np.dot(wi, Tp - Tm)) / (2.0 * h)
    return out
