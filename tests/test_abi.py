"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/gr.h declares, its structs match the ctypes binding, and argument
errors come back as status codes before any GPU work is enqueued."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2602_01057_amd import _lib as L
from paper_2602_01057_amd.inputs import CT_CONE_50K, PET_200K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gr.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libgr.so is not built: run __graft_entry__.build()")
    return L.load()


def header_functions():
    text = open(HEADER).read()
    return re.findall(r"^\s*(?:gr_status|const char \s*\*|int32_t)\s*(gr_[a-z_]+)\(", text, re.M)


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) == 29
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"{n} missing from the ctypes binding"
    assert lib.gr_abi_version() == 1


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(gr_scene), sizeof(gr_launch), sizeof(gr_segment),
         sizeof(gr_loss), sizeof(gr_ct_geom), sizeof(gr_pet_geom));
  printf("%zu %zu %zu %zu\\n", offsetof(gr_scene, kappa), offsetof(gr_scene, accel_bytes),
         offsetof(gr_ct_geom, tile_u), offsetof(gr_pet_geom, planes));
  printf("%zu %zu %zu %zu\\n", sizeof(gr_grid), offsetof(gr_grid, dims), sizeof(gr_adam),
         offsetof(gr_adam, step));
  printf("%zu %zu %zu\\n", sizeof(gr_gauss_adam), offsetof(gr_gauss_adam, eps), offsetof(gr_gauss_adam, step));
  printf("%zu %zu %zu %d\\n", sizeof(gr_tof), offsetof(gr_tof, center), offsetof(gr_tof, atten), GR_TOF_MAX_BINS);
  printf("%zu %zu\\n", offsetof(gr_launch, precision), offsetof(gr_launch, reserved));
  printf("%zu %zu %zu %zu\\n", sizeof(gr_bwd_segment), offsetof(gr_bwd_segment, target),
         offsetof(gr_bwd_segment, accum), offsetof(gr_bwd_segment, background));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    sizes = [ctypes.sizeof(c) for c in (L.GrScene, L.GrLaunch, L.GrSegment, L.GrLoss, L.GrCtGeom,
                                        L.GrPetGeom)]
    offs = [L.GrScene.kappa.offset, L.GrScene.accel_bytes.offset, L.GrCtGeom.tile_u.offset,
            L.GrPetGeom.planes.offset]
    vol = [ctypes.sizeof(L.GrGrid), L.GrGrid.dims.offset, ctypes.sizeof(L.GrAdam), L.GrAdam.step.offset,
           ctypes.sizeof(L.GrGaussAdam), L.GrGaussAdam.eps.offset, L.GrGaussAdam.step.offset,
           ctypes.sizeof(L.GrTof), L.GrTof.center.offset, L.GrTof.atten.offset, L.GR_TOF_MAX_BINS]
    bseg = [L.GrLaunch.precision.offset, L.GrLaunch.reserved.offset,
            ctypes.sizeof(L.GrBwdSegment), L.GrBwdSegment.target.offset, L.GrBwdSegment.accum.offset,
            L.GrBwdSegment.background.offset]
    assert [int(x) for x in out] == sizes + offs + vol + bseg


def test_size_queries_and_argument_errors(lib):
    b = ctypes.c_size_t()
    assert lib.gr_accel_bytes(1000, 0, ctypes.byref(b)) == L.GR_OK and b.value > 64 * 1000
    b16 = b.value
    assert lib.gr_accel_bytes(1000, 64, ctypes.byref(b)) == L.GR_OK and b.value == b16  # default leaf
    assert lib.gr_accel_bytes(0, 0, ctypes.byref(b)) == L.GR_OK and b.value > 0
    assert lib.gr_accel_bytes(-1, 0, ctypes.byref(b)) == L.GR_E_ARG
    assert lib.gr_accel_bytes(10, 65, ctypes.byref(b)) == L.GR_E_ARG
    assert lib.gr_accel_bytes(1 << 29, 16, ctypes.byref(b)) == L.GR_E_UNSUPPORTED
    assert lib.gr_accel_bytes(10, 0, None) == L.GR_E_ARG
    assert lib.gr_backward_scratch_bytes(100, ctypes.byref(b)) == L.GR_OK and b.value >= 4000
    acc = b.value
    # fused scratch: accumulators, a 256-byte counter slot, then 4- and 8-byte
    # hit-list entries for persistent_groups x waves_per_group waves
    opt = L.GrLaunch()
    opt.waves_per_group, opt.persistent_groups, opt.hit_list_cap = 2, 10, 64
    assert lib.gr_fused_scratch_bytes(100, ctypes.byref(opt), ctypes.byref(b)) == L.GR_OK
    assert b.value == acc + 256 + 20 * 64 * 4 + 20 * 64 * 8
    opt.hit_list_cap = -1
    assert lib.gr_fused_scratch_bytes(100, ctypes.byref(opt), ctypes.byref(b)) == L.GR_OK and b.value == acc
    for bad in (1, 63, (1 << 20) + 1, -2):
        opt.hit_list_cap = bad
        assert lib.gr_fused_scratch_bytes(100, ctypes.byref(opt), ctypes.byref(b)) == L.GR_E_ARG
    # scene checks happen before anything touches the GPU
    fake = 1 << 20  # never dereferenced: the checks reject these calls first
    sc = L.GrScene(10, fake, fake, fake, fake, 3.0, 0, fake, 16)
    assert lib.gr_build_accel(ctypes.byref(sc), None) == L.GR_E_WORKSPACE
    sc.kappa = 0.0
    assert lib.gr_build_accel(ctypes.byref(sc), None) == L.GR_E_ARG
    sc.kappa = float("nan")
    assert lib.gr_build_accel(ctypes.byref(sc), None) == L.GR_E_ARG
    sc.kappa = 3.0
    sc.mean = None
    assert lib.gr_build_accel(ctypes.byref(sc), None) == L.GR_E_ARG
    assert lib.gr_build_accel(None, None) == L.GR_E_ARG
    sc.mean = fake
    sc.accel = fake + 4  # misaligned
    sc.accel_bytes = 1 << 30
    assert lib.gr_build_accel(ctypes.byref(sc), None) == L.GR_E_ARG
    sc.accel = fake
    assert lib.gr_project(ctypes.byref(sc), fake, fake, -1, fake, None, None) == L.GR_E_ARG
    assert lib.gr_project(ctypes.byref(sc), None, fake, 5, fake, None, None) == L.GR_E_ARG
    bad = L.GrLaunch(17, 0)
    assert lib.gr_project(ctypes.byref(sc), fake, fake, 5, fake, ctypes.byref(bad), None) == L.GR_E_ARG
    bad = L.GrLaunch()
    bad.precision = 2   # only 0 (FP64) and 1 (compact FP32)
    assert lib.gr_project(ctypes.byref(sc), fake, fake, 5, fake, ctypes.byref(bad), None) == L.GR_E_ARG
    # backward: neither grad_out nor loss, and a too-small scratch
    gm = fake
    assert lib.gr_project_backward(ctypes.byref(sc), fake, fake, 5, None, None, gm, gm, gm, gm, fake,
                                   1 << 20, None, None) == L.GR_E_ARG
    assert lib.gr_project_backward(ctypes.byref(sc), fake, fake, 5, fake, None, gm, gm, gm, gm, fake,
                                   4, None, None) == L.GR_E_WORKSPACE
    # voxelisation: missing grid, bad spacing, negative dims, no output
    grid = L.GrGrid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (4, 4, 4))
    assert lib.gr_voxelize(ctypes.byref(sc), None, fake, None, None) == L.GR_E_ARG
    assert lib.gr_voxelize(ctypes.byref(sc), ctypes.byref(grid), None, None, None) == L.GR_E_ARG
    grid.spacing[1] = 0.0
    assert lib.gr_voxelize(ctypes.byref(sc), ctypes.byref(grid), fake, None, None) == L.GR_E_ARG
    grid.spacing[1], grid.dims[2] = 1.0, -1
    assert lib.gr_voxelize(ctypes.byref(sc), ctypes.byref(grid), fake, None, None) == L.GR_E_ARG
    grid.dims[0], grid.dims[1], grid.dims[2] = 1 << 20, 1 << 20, 1 << 20
    assert lib.gr_voxelize(ctypes.byref(sc), ctypes.byref(grid), fake, None, None) == L.GR_E_UNSUPPORTED
    # Adam: step 0, beta out of range, missing buffers
    hp = L.GrAdam(0.01, 0.9, 0.999, 1e-8, 0)
    assert lib.gr_adam_step(fake, fake, fake, fake, 10, ctypes.byref(hp), None) == L.GR_E_ARG
    hp.step, hp.beta1 = 1, 1.0
    assert lib.gr_adam_step(fake, fake, fake, fake, 10, ctypes.byref(hp), None) == L.GR_E_ARG
    hp.beta1 = 0.9
    assert lib.gr_adam_step(None, fake, fake, fake, 10, ctypes.byref(hp), None) == L.GR_E_ARG
    assert lib.gr_adam_step(fake, fake, fake, fake, 10, None, None) == L.GR_E_ARG
    assert lib.gr_adam_step(None, None, None, None, 0, ctypes.byref(hp), None) == L.GR_OK
    # fused scene Adam: a bad learning rate in one group, overlapping arrays,
    # misalignment, too many Gaussians
    ga = L.GrGaussAdam((ctypes.c_float * 4)(0.1, 0.02, 0.01, 0.03), 0.9, 0.999, 1e-8, 0, 1)
    arrs = [fake + k * 11 * 4 * 100 for k in range(5)]
    ga.lr[2] = float("nan")
    assert lib.gr_adam_gaussians(100, *arrs, ctypes.byref(ga), None) == L.GR_E_ARG
    ga.lr[2] = 0.01
    assert lib.gr_adam_gaussians(100, arrs[0], arrs[1], arrs[2], arrs[3], arrs[2] + 4, ctypes.byref(ga),
                                 None) == L.GR_E_ARG
    assert lib.gr_adam_gaussians(100, arrs[0] + 2, *arrs[1:], ctypes.byref(ga), None) == L.GR_E_ARG
    assert lib.gr_adam_gaussians(1 << 29, *arrs, ctypes.byref(ga), None) == L.GR_E_UNSUPPORTED
    assert lib.gr_adam_gaussians(0, None, None, None, None, None, ctypes.byref(ga), None) == L.GR_OK
    ga.step = 0
    assert lib.gr_adam_gaussians(100, *arrs, ctypes.byref(ga), None) == L.GR_E_ARG
    # TOF: bad bin counts and kernel widths, too many waves, missing buffers
    tof = L.GrTof(7, 20.0, 15.0, 0, None, None)
    assert lib.gr_project_tof(ctypes.byref(sc), fake, fake, 5, None, fake, None, None) == L.GR_E_ARG
    for nb, sg, bw, code in ((-1, 20.0, 15.0, L.GR_E_ARG), (33, 20.0, 15.0, L.GR_E_UNSUPPORTED),
                             (7, 0.0, 15.0, L.GR_E_ARG), (7, 20.0, -1.0, L.GR_E_ARG),
                             (7, float("inf"), 15.0, L.GR_E_ARG), (7, 1e-13, 15.0, L.GR_E_ARG),
                             (7, 2e19, 15.0, L.GR_E_ARG)):
        t = L.GrTof(nb, sg, bw, 0, None, None)
        assert lib.gr_project_tof(ctypes.byref(sc), fake, fake, 5, ctypes.byref(t), fake, None, None) == code
    assert lib.gr_project_tof(ctypes.byref(sc), fake, fake, 5, ctypes.byref(tof), None, None, None) == L.GR_E_ARG
    w8 = L.GrLaunch(8, 0)
    assert lib.gr_project_tof(ctypes.byref(sc), fake, fake, 5, ctypes.byref(tof), fake, ctypes.byref(w8),
                              None) == L.GR_E_ARG
    assert lib.gr_project_tof_backward(ctypes.byref(sc), fake, fake, 5, ctypes.byref(tof), None, gm, gm, gm, gm,
                                       fake, 1 << 20, None, None) == L.GR_E_ARG
    assert lib.gr_project_tof_backward(ctypes.byref(sc), fake, fake, 5, ctypes.byref(tof), fake, gm, gm, gm, gm,
                                       fake, 4, None, None) == L.GR_E_WORKSPACE
    assert lib.gr_tof_centers(None, fake, 5, fake, None) == L.GR_E_ARG
    assert lib.gr_tof_centers(None, None, 0, None, None) == L.GR_OK
    # loss weights: unknown kind, Poisson without any background, misaligned loss
    assert lib.gr_loss_weights(7, fake, fake, None, 1.0, 5, fake, None, None) == L.GR_E_ARG
    assert lib.gr_loss_weights(L.GR_LOSS_POISSON, fake, fake, None, 0.0, 5, fake, None, None) == L.GR_E_ARG
    assert lib.gr_loss_weights(L.GR_LOSS_L2, fake, fake, None, 0.0, 5, fake, fake + 4, None) == L.GR_E_ARG
    assert lib.gr_loss_weights(L.GR_LOSS_L2, None, None, None, 0.0, 0, None, None, None) == L.GR_OK
    # voxelisation counters must be an aligned pointer
    grid.dims[0] = grid.dims[1] = grid.dims[2] = 4
    assert lib.gr_voxelize_stats(ctypes.byref(sc), ctypes.byref(grid), fake, None, None, None) == L.GR_E_ARG
    assert lib.gr_voxelize_stats(ctypes.byref(sc), ctypes.byref(grid), fake, fake + 4, None, None) == L.GR_E_ARG
    # batched: too many segments, bad scene index
    SC = (L.GrScene * 1)(sc)
    SG = (L.GrSegment * 40)()
    assert lib.gr_project_batched(SC, 1, SG, 40, None, None) == L.GR_E_UNSUPPORTED
    SG[0].scene = 3
    SG[0].n_rays = 5
    SG[0].stride = 5
    assert lib.gr_project_batched(SC, 1, SG, 1, None, None) == L.GR_E_ARG   # bad scene index
    SG[0].scene = 0
    assert lib.gr_project_batched(SC, 1, SG, 1, None, None) == L.GR_E_ARG   # null ray arrays
    SG[0].ray_o = SG[0].ray_d = SG[0].out = fake
    SG[0].ray_offset = 1
    assert lib.gr_project_batched(SC, 1, SG, 1, None, None) == L.GR_E_ARG   # past the array end
    # batched fused backward: segment count, scene index, loss kind, Poisson
    # background, missing targets, misaligned accumulators, short scratch
    BS = (L.GrBwdSegment * 40)()
    assert lib.gr_project_backward_batched(SC, 1, BS, 40, None, 0, None, None) == L.GR_E_UNSUPPORTED
    b = BS[0]
    b.scene, b.loss_kind, b.n_rays, b.stride = 0, L.GR_LOSS_L2, 64, 64
    b.ray_o = b.ray_d = fake
    b.accum = fake
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, None, 0, None, None) == L.GR_E_ARG  # no target
    b.target = fake
    b.scene = 1
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, None, 0, None, None) == L.GR_E_ARG  # scene index
    b.scene = 0
    b.loss_kind = 7
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, None, 0, None, None) == L.GR_E_ARG  # loss kind
    b.loss_kind = L.GR_LOSS_POISSON
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, None, 0, None, None) == L.GR_E_ARG  # background 0
    b.loss_kind = L.GR_LOSS_L2
    b.accum = fake + 4
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, None, 0, None, None) == L.GR_E_ARG  # misaligned
    b.accum = fake
    assert lib.gr_project_backward_batched(SC, 1, BS, 1, fake, 256, None, None) == L.GR_E_WORKSPACE
    assert lib.gr_backward_accum_zero(-1, fake, None) == L.GR_E_ARG
    assert lib.gr_backward_accum_zero(5, fake + 4, None) == L.GR_E_ARG
    assert lib.gr_backward_finish(ctypes.byref(sc), None, fake, fake, fake, fake, None) == L.GR_E_ARG
    # the static-scratch backward refuses scenes whose sums do not fit its array
    big = L.GrScene(sc.n, sc.mean, sc.scale, sc.quat, sc.density, 3.0, 0, sc.accel, 1 << 40)
    big.n = (L.GR_STATIC_SCRATCH_BYTES // 40) + 1
    assert lib.gr_project_backward_static(ctypes.byref(big), fake, fake, 64, fake, None, fake, fake, fake, fake,
                                          None, None) == L.GR_E_UNSUPPORTED
    assert lib.gr_status_str(L.GR_E_WORKSPACE) == b"workspace or scratch buffer too small"
    assert lib.gr_status_str(12345) == b"unknown status"


def test_ray_counts_match_oracle_geometry(lib):
    from oracle import geometry as G
    from paper_2602_01057_amd.api import _ct_struct, _pet_struct
    n = ctypes.c_int64()
    g = CT_CONE_50K["geom"]
    assert lib.gr_rays_count_ct(ctypes.byref(_ct_struct(g)), ctypes.byref(n)) == L.GR_OK
    assert n.value == G.count(g) == 3_276_800
    p = PET_200K["geom"]
    assert lib.gr_rays_count_pet(ctypes.byref(_pet_struct(p, None)), ctypes.byref(n)) == L.GR_OK
    assert n.value == G.count(p) == 65_189_376
    for mrd in (0, 3, 40):
        pp = dict(p, max_ring_diff=mrd, n_rings=5)
        assert lib.gr_rays_count_pet(ctypes.byref(_pet_struct(pp, None)), ctypes.byref(n)) == L.GR_OK
        assert n.value == G.count(pp)
    bad = dict(p, n_radial=600)  # |k| pi / N would pass pi / 2
    assert lib.gr_rays_count_pet(ctypes.byref(_pet_struct(bad, None)), ctypes.byref(n)) == L.GR_E_ARG
    cone_bad = dict(g, dsd=500.0)
    assert lib.gr_rays_count_ct(ctypes.byref(_ct_struct(cone_bad)), ctypes.byref(n)) == L.GR_E_ARG
