"""FP64 ray geometry of the oracle: cone-/parallel-beam CT rays and PET lines
of response, in the packet (tile-major) order the library documents.

TEST INFRASTRUCTURE ONLY: it defines the expected rays for checking the HIP
ray generators and supplies rays to the oracle. It shares no code with the
HIP library.

The paper sets each ray's origin and direction from the scanner geometry
(Fig. 1) and places PET lines of response at their true positions on the
cylindrical detector instead of resampling the sinogram (Sec. 3, Inherent
limitations; Fig. 2; Sec. 6). Readings used where the paper gives no formula:

CT (rotation axis z). View v has angle th = angle0 + v * (angle_range / n_views).
Source direction e_s = (cos th, sin th, 0), detector axes e_u = (-sin th,
cos th, 0) and e_v = (0, 0, 1); pixel (i, j) sits at
u = (i - (nu-1)/2) pitch_u + offset_u, w = (j - (nv-1)/2) pitch_v + offset_v.
  parallel beam: d = -e_s, o = u e_u + w e_v;
  cone beam: source S = dso e_s, pixel P = -(dsd - dso) e_s + u e_u + w e_v,
             d = (P - S)/|P - S|, o = S - (S.d) d.
PET (ring radius Rr, N crystals per ring, ring z = (r - (n_rings-1)/2) pitch).
Radial index k = kk - n_radial//2. The line normal angle is
psi = pi v / n_views + (k odd) pi / N, and the end points sit at angles
psi +- (pi/2 - pi k / N) on rings r1 and r2, which are crystal centres when
n_views = N/2 (arc-corrected: the chord distance is Rr sin(pi k / N), the true
non-uniform spacing). The non-arc model moves the same line in-plane along its
normal to the uniform distance k pi Rr / N. d = (B - A)/|B - A| and
o = A - (A.d) d, the foot of the perpendicular from the isocentre.

Ordering: rays are grouped view by view; inside a view the (i, j) grid, or the
(radial, plane) grid for PET, is cut into tiles of tu x tv and enumerated tile
row by tile row, tile by tile, and row-major inside a tile; edge tiles are
partial. ``tiled_index`` states the closed form. PET may group views in blocks
of tile_views: each tile then lists its cells for every view of the block,
view by view (``untile_views``).
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Tuple

import numpy as np


def tiled_index(i, j, nu, nv, tu, tv):
    """Position of grid cell (i, j) (i fastest) inside one view's ray block."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    ti, tj = i // tu, j // tv
    h_t = np.minimum(tv, nv - tj * tv)
    w_t = np.minimum(tu, nu - ti * tu)
    return tj * tv * nu + ti * tu * h_t + (j - tj * tv) * w_t + (i - ti * tu)


def untile(idx, nu, nv, tu, tv):
    """Inverse of ``tiled_index`` for positions inside one view's block."""
    idx = np.asarray(idx, dtype=np.int64)
    tj = idx // (tv * nu)
    rem = idx - tj * tv * nu
    h_t = np.minimum(tv, nv - tj * tv)
    ti = rem // (tu * h_t)
    rem2 = rem - ti * tu * h_t
    w_t = np.minimum(tu, nu - ti * tu)
    return ti * tu + rem2 % w_t, tj * tv + rem2 // w_t


def untile_views(idx, n_views, nu, nv, tu, tv, kv):
    """Inverse of the view-blocked tiled order: views in blocks of kv (the
    last block may be shorter, V views); inside a block the (i, j) grid is
    tiled as in ``untile`` and each tile lists its cells for every view of the
    block, view by view. A shorter last block whose V divides kv uses tiles
    kv / V times taller, so that they hold as many rays as the others.
    Returns (view, i, j). kv = 1 is the per-view order."""
    idx = np.asarray(idx, dtype=np.int64)
    per = nu * nv
    b = idx // (kv * per)
    V = np.minimum(kv, n_views - b * kv)
    tv = np.where((V < kv) & (kv % V == 0), tv * (kv // V), tv)
    pos = idx - b * kv * per
    tj = pos // (V * tv * nu)
    rem = pos - tj * V * tv * nu
    h_t = np.minimum(tv, nv - tj * tv)
    ti = rem // (V * tu * h_t)
    rem2 = rem - ti * V * tu * h_t
    w_t = np.minimum(tu, nu - ti * tu)
    k = rem2 // (w_t * h_t)
    rem3 = rem2 - k * w_t * h_t
    return b * kv + k, ti * tu + rem3 % w_t, tj * tv + rem3 // w_t


def ct_count(g: Dict) -> int:
    return int(g["n_views"]) * int(g["nu"]) * int(g["nv"])


def ct_rays64(g: Dict, index: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """FP64 (3, m) origins and directions of the CT rays at positions ``index``
    (default: all) of the ray order."""
    nu, nv, nview = int(g["nu"]), int(g["nv"]), int(g["n_views"])
    tu, tv = int(g["tile_u"]), int(g["tile_v"])
    per = nu * nv
    if index is None:
        index = np.arange(nview * per, dtype=np.int64)
    index = np.asarray(index, dtype=np.int64)
    v = index // per
    i, j = untile(index - v * per, nu, nv, tu, tv)
    th = g["angle0"] + v * (g["angle_range"] / nview)
    c, s = np.cos(th), np.sin(th)
    es = np.stack([c, s, np.zeros_like(c)])
    eu = np.stack([-s, c, np.zeros_like(c)])
    ev = np.stack([np.zeros_like(c), np.zeros_like(c), np.ones_like(c)])
    u = (i - (nu - 1) / 2.0) * g["pitch_u"] + g["offset_u"]
    w = (j - (nv - 1) / 2.0) * g["pitch_v"] + g["offset_v"]
    if int(g["cone"]) == 0:
        d = -es
        o = u * eu + w * ev
    else:
        S = g["dso"] * es
        P = -(g["dsd"] - g["dso"]) * es + u * eu + w * ev
        d = P - S
        d = d / np.sqrt((d * d).sum(axis=0))
        o = S - (S * d).sum(axis=0) * d
    return o, d


def pet_default_planes(n_rings: int, max_ring_diff: int) -> np.ndarray:
    """Ring pairs (r1, r2), |r1 - r2| <= max_ring_diff, grouped by ring
    difference 0, +1, -1, +2, -2, ... and by r1 inside a group."""
    out = []
    for a in range(0, max_ring_diff + 1):
        for diff in ((0,) if a == 0 else (a, -a)):
            for r1 in range(n_rings):
                r2 = r1 + diff
                if 0 <= r2 < n_rings:
                    out.append((r1, r2))
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def pet_planes(g: Dict) -> np.ndarray:
    if g.get("planes") is not None:
        return np.asarray(g["planes"], dtype=np.int64).reshape(-1, 2)
    return pet_default_planes(int(g["n_rings"]), int(g["max_ring_diff"]))


def pet_count(g: Dict) -> int:
    return int(g["n_views"]) * int(g["n_radial"]) * pet_planes(g).shape[0]


def pet_rays64(g: Dict, index: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    o, d, _ = _pet_lines(g, index)
    return o, d


def pet_tof_centers64(g: Dict, index: Optional[np.ndarray] = None) -> np.ndarray:
    """Ray parameter of each line's TOF centre: the midpoint of its two end
    points (crystal centres when arc-corrected, the moved end points of the
    straightened model), t = ((A + B)/2 - o) . d."""
    return _pet_lines(g, index)[2]


def _pet_lines(g: Dict, index: Optional[np.ndarray] = None):
    planes = pet_planes(g)
    npl = planes.shape[0]
    nrad, nview = int(g["n_radial"]), int(g["n_views"])
    N = int(g["n_crystals"])
    Rr = float(g["ring_radius"])
    per = nrad * npl
    if index is None:
        index = np.arange(nview * per, dtype=np.int64)
    index = np.asarray(index, dtype=np.int64)
    kv = max(1, int(g.get("tile_views", 1)))
    v, kk, p = untile_views(index, nview, nrad, npl, int(g["tile_radial"]), int(g["tile_axial"]), kv)
    k = kk - nrad // 2
    r1, r2 = planes[p, 0], planes[p, 1]
    z1 = (r1 - (int(g["n_rings"]) - 1) / 2.0) * g["ring_pitch"]
    z2 = (r2 - (int(g["n_rings"]) - 1) / 2.0) * g["ring_pitch"]
    psi = math.pi * v / nview + (k & 1) * (math.pi / N)
    gam = math.pi / 2.0 - math.pi * k / N
    aA, aB = psi + gam, psi - gam
    A = np.stack([Rr * np.cos(aA), Rr * np.sin(aA), z1])
    B = np.stack([Rr * np.cos(aB), Rr * np.sin(aB), z2])
    if int(g.get("arc_correct", 1)) == 0:
        shift = k * (math.pi * Rr / N) - Rr * np.sin(math.pi * k / N)
        nrm = np.stack([np.cos(psi), np.sin(psi), np.zeros_like(psi)])
        A = A + shift * nrm
        B = B + shift * nrm
    d = B - A
    d = d / np.sqrt((d * d).sum(axis=0))
    o = A - (A * d).sum(axis=0) * d
    tc = ((0.5 * (A + B) - o) * d).sum(axis=0)
    return o, d, tc


def rays64(g: Dict, index=None):
    return ct_rays64(g, index) if g["kind"] == "ct" else pet_rays64(g, index)


def rays32(g: Dict, index=None):
    """The rays rounded to FP32, SoA (3, m) float32 each."""
    o, d = rays64(g, index)
    return (np.ascontiguousarray(o, dtype=np.float32),
            np.ascontiguousarray(d, dtype=np.float32))


def count(g: Dict) -> int:
    return ct_count(g) if g["kind"] == "ct" else pet_count(g)
