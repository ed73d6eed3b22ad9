"""Pins of the oracle's voxelisation (Fig. 1: the reconstruction is the
optimised Gaussians voxelised; the field is Eq. 2's mixture) and of its Adam
step (the optimiser of Sec. 4.1) to mathematics and to an independent library:
the peak and principal-axis values of one Gaussian, its mass (spectrally exact
Riemann sums), the kappa-truncated mass (chi-square with 3 degrees of freedom),
agreement with the separately pinned line integral along grid lines, and
torch.optim.Adam."""
import math

import numpy as np
import pytest

import oracle
from paper_2602_01057_amd.inputs import Scene


def one(mu, s, q, rho):
    return Scene(np.asarray(mu, np.float64).reshape(3, 1), np.asarray(s, np.float64).reshape(3, 1),
                 np.asarray(q, np.float64).reshape(4, 1), np.asarray([rho], np.float64))


def rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


Q = (0.8, -0.3, 0.4, 0.33)
S = (1.1, 1.7, 2.4)
MU = (0.3, -0.7, 1.9)


def test_peak_and_principal_axes():
    g = one(MU, S, Q, 2.5)
    v = oracle.voxelize(g, MU, (1, 1, 1), (1, 1, 1))["V_inf"]
    assert v.shape == (1, 1, 1) and abs(v[0, 0, 0] - 2.5) <= 1e-14
    R = rot(Q)
    for k in range(3):
        for sign in (1, -1):
            x = np.asarray(MU) + sign * S[k] * R[:, k]
            v = oracle.voxelize(g, x, (1, 1, 1), (1, 1, 1))["V_inf"][0, 0, 0]
            assert abs(v - 2.5 * math.exp(-0.5)) <= 1e-12
            # 3 sigma along an axis is exactly on the kappa = 3 boundary
            x3 = np.asarray(MU) + sign * 2.9999 * S[k] * R[:, k]
            assert oracle.voxelize(g, x3, (1, 1, 1), (1, 1, 1), kappa=3.0)["V"][0, 0, 0] > 0
            x3 = np.asarray(MU) + sign * 3.0001 * S[k] * R[:, k]
            assert oracle.voxelize(g, x3, (1, 1, 1), (1, 1, 1), kappa=3.0)["V"][0, 0, 0] == 0


def test_mass_untruncated_and_truncated():
    g = one(MU, S, Q, 1.3)
    h = 0.5
    n = 96
    origin = np.asarray(MU) - h * (n // 2) + 0.123  # voxel centres off the mean
    r = oracle.voxelize(g, origin, (h, h, h), (n, n, n))
    mass = 1.3 * (2 * math.pi) ** 1.5 * S[0] * S[1] * S[2]
    assert abs(r["V_inf"].sum() * h ** 3 - mass) <= 1e-9 * mass
    # inside the kappa-ellipsoid: P(chi2_3 <= kappa^2) of the mass; the sum is
    # a Riemann sum of a function with a jump of ~1% of the peak at the boundary
    kap = 3.0
    frac = math.erf(kap / math.sqrt(2)) - math.sqrt(2 / math.pi) * kap * math.exp(-kap * kap / 2)
    h2 = 0.25
    n2 = 112
    origin2 = np.asarray(MU) - h2 * (n2 // 2) + 0.0371
    r2 = oracle.voxelize(g, origin2, (h2, h2, h2), (n2, n2, n2), kappa=kap)
    assert abs(r2["V"].sum() * h2 ** 3 - frac * mass) <= 2e-3 * frac * mass


def test_grid_lines_integrate_to_the_projection():
    """Sum of V_inf along a grid line times the spacing equals the line integral
    of the mixture (Eq. 12 without cutoff) along that line."""
    rng = np.random.default_rng(3)
    n = 5
    sc = Scene(rng.uniform(-3, 3, (3, n)), rng.uniform(0.8, 2.0, (3, n)), rng.normal(size=(4, n)),
               rng.uniform(0.5, 2.0, n))
    h = 0.2
    for axis in range(3):
        x0 = np.array([0.37, -0.41, 0.53])
        x0[axis] = -30.0
        dims = [1, 1, 1]
        dims[axis] = 301
        sp = [1.0, 1.0, 1.0]
        sp[axis] = h
        line = oracle.voxelize(sc, x0, sp, dims)["V_inf"].ravel()
        d = np.zeros((3, 1))
        d[axis, 0] = 1.0
        ref = oracle.project(sc, x0.reshape(3, 1), d)["I_inf"][0]
        assert abs(line.sum() * h - ref) <= 1e-10 * ref


def test_order_and_density_linearity():
    rng = np.random.default_rng(4)
    n = 7
    sc = Scene(rng.uniform(-2, 2, (3, n)), rng.uniform(0.5, 1.5, (3, n)), rng.normal(size=(4, n)),
               rng.uniform(0.5, 2.0, n))
    perm = rng.permutation(n)
    sp = Scene(sc.mean[:, perm], sc.scale[:, perm], sc.quat[:, perm], sc.density[perm])
    a = oracle.voxelize(sc, (-4, -4, -4), (0.5, 0.5, 0.5), (17, 17, 17))["V"]
    b = oracle.voxelize(sp, (-4, -4, -4), (0.5, 0.5, 0.5), (17, 17, 17))["V"]
    assert np.allclose(a, b, rtol=1e-13, atol=0)
    s2 = Scene(sc.mean, sc.scale, sc.quat, 3.0 * sc.density)
    c = oracle.voxelize(s2, (-4, -4, -4), (0.5, 0.5, 0.5), (17, 17, 17))["V"]
    assert np.allclose(c, 3.0 * a, rtol=1e-13, atol=0)


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 8):
        g = rng.normal(size=50) * (1 + step)
        oracle.adam(p, g, m, v, 0.01, 0.9, 0.999, 1e-8, step)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_gaussians_matches_autograd_and_torch_optim():
    """The fused step on an (11, n) scene against torch: the log rows get their
    gradient from autograd through x = exp(t), the update from torch.optim.Adam
    with one parameter group per row group and its own learning rate."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    n = 40
    nat = np.concatenate([rng.normal(0, 20, (3, n)), rng.uniform(0.5, 6, (3, n)), rng.normal(size=(4, n)),
                          rng.uniform(0.05, 1, (1, n))])
    theta = nat.copy()
    theta[3:6] = np.log(nat[3:6])
    theta[10] = np.log(nat[10])
    m = np.zeros((11, n))
    v = np.zeros((11, n))
    lr = (0.1, 0.02, 0.01, 0.03)
    rows = ((0, 3), (3, 6), (6, 10), (10, 11))
    tp = [torch.tensor(theta[a:b].copy(), dtype=torch.float64, requires_grad=True) for a, b in rows]
    opt = torch.optim.Adam([{"params": [t], "lr": l} for t, l in zip(tp, lr)], betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 7):
        G = rng.normal(size=(11, n)) * 10 ** rng.uniform(-2, 1, (11, n))  # dL/d natural
        oracle.adam_gaussians(theta, G, m, v, nat, lr, 0.9, 0.999, 1e-8, step)
        opt.zero_grad()
        xs = [tp[0], tp[1].exp(), tp[2], tp[3].exp()]
        L = sum((x * torch.tensor(G[a:b])).sum() for x, (a, b) in zip(xs, rows))
        L.backward()
        opt.step()
        ref = np.concatenate([t.detach().numpy() for t in tp])
        assert np.allclose(theta, ref, rtol=1e-12, atol=1e-14)
        nat_ref = ref.copy()
        nat_ref[3:6] = np.exp(ref[3:6])
        nat_ref[10] = np.exp(ref[10])
        assert np.allclose(nat, nat_ref, rtol=1e-13, atol=0)
    # a sign or group slip would move the parameters differently: check the
    # first step's direction on a fresh state, row by row
    th = np.zeros((11, 3))
    nat1 = np.ones((11, 3))
    G = np.tile(np.array([1.0, -1.0, 2.0]), (11, 1))
    oracle.adam_gaussians(th, G, np.zeros((11, 3)), np.zeros((11, 3)), nat1, lr, 0.9, 0.999, 1e-8, 1)
    for gi, (a, b) in enumerate(rows):
        assert np.allclose(th[a:b], -lr[gi] * np.sign(G[a:b]), rtol=1e-6)


def test_voxel_pair_counts_fill_the_cutoff_ellipsoid():
    """The pairs inside the cutoff of one Gaussian on a fine grid number about
    the ellipsoid's volume (4/3 pi kappa^3 s1 s2 s3) over the voxel volume."""
    sc = Scene(np.zeros((3, 1), np.float32), np.array([[1.0], [1.5], [0.75]], np.float32),
               np.array([[0.9], [0.3], [-0.2], [0.25]], np.float32), np.ones(1, np.float32))
    h = 0.25
    k = 80
    r = oracle.voxelize(sc, (-k * h / 2,) * 3, (h,) * 3, (k + 1,) * 3)
    vol = 4.0 / 3.0 * np.pi * 27.0 * 1.0 * 1.5 * 0.75
    assert abs(r["pairs_in"] * h ** 3 / vol - 1.0) < 0.01
    assert r["pairs_in"] <= r["pairs_hi"] <= r["pairs_in"] + 50
    assert r["pairs_hi"] == int((r["V_hi"] > 0).sum())
