"""3D PSNR and 3D SSIM (the paper's CT metrics) on the CPU: identity, the
closed form of PSNR for a known error, symmetry and bounds of SSIM."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_psnr_closed_form_and_identity():
    from paper_2602_01057_amd.recon import psnr3d
    ref = torch.zeros(10, 10, 10, dtype=torch.float64)
    ref[0, 0, 0] = 2.0  # range 2
    x = ref + 0.1
    assert abs(psnr3d(x, ref) - 10 * math.log10(4.0 / 0.01)) <= 1e-12
    assert psnr3d(ref, ref) == math.inf


def test_ssim_identity_symmetry_bounds():
    from paper_2602_01057_amd.recon import ssim3d
    rng = np.random.default_rng(0)
    a = torch.from_numpy(rng.uniform(0, 1, (16, 16, 16)))
    b = a + torch.from_numpy(rng.normal(0, 0.1, (16, 16, 16)))
    assert abs(ssim3d(a, a) - 1.0) <= 1e-12
    s = ssim3d(b, a, data_range=1.0)
    assert abs(s - ssim3d(a, b, data_range=1.0)) <= 1e-12
    assert 0.0 < s < 1.0
    c = a + torch.from_numpy(rng.normal(0, 0.3, (16, 16, 16)))
    assert ssim3d(c, a, data_range=1.0) < s  # more noise, less similar
