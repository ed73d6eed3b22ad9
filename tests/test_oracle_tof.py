"""Pins of the oracle's time-of-flight / attenuation projection and gradient
(the projector extensions the paper names as future work, Sec. 5).

Each check compares against an independent quantity: quadrature of the
Gaussian times the TOF kernel along the line with an independently built
covariance inverse, the sum over bins against the plain projection (the bins
of a kernel narrower than their spacing times two tile the line), the limit of
a vanishing kernel width (the density sampled at the bin centre), finite
differences of the forward, the gradient through (A, B, C) against the
envelope-theorem gradient without TOF, and the geometry of the TOF centres.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_2602_01057_amd.inputs import PET_200K, sample_scene
from test_oracle_pins import one, rand_gauss, sigma_inv_independent

SQRT2PI = math.sqrt(2.0 * math.pi)


def _tof_quadrature(mu, s, q, rho, o, d, tau_b, sigma, width):
    """Trapezoid rule for rho Int G(o + t d) h(t) dt with the TOF kernel
    h(t) = width / (sqrt(2 pi) sigma) exp(-(t - tau_b)^2 / (2 sigma^2))."""
    Pi = sigma_inv_independent(s, q)
    dl = o - mu
    a = d @ Pi @ d
    tc = -(d @ Pi @ dl) / a
    half = 12.0 / math.sqrt(a)
    h = min(0.05 / math.sqrt(a), sigma / 20.0)
    lo, hi = min(tc - half, tau_b - 12 * sigma), max(tc + half, tau_b + 12 * sigma)
    t = np.arange(lo, hi + h, h)
    x = o[:, None] + t[None, :] * d[:, None] - mu[:, None]
    f = np.exp(-0.5 * np.einsum("in,ij,jn->n", x, Pi, x))
    f *= width / (SQRT2PI * sigma) * np.exp(-0.5 * ((t - tau_b) / sigma) ** 2)
    return rho * (f.sum() - 0.5 * (f[0] + f[-1])) * h


def test_tof_bin_matches_quadrature():
    rng = np.random.default_rng(41)
    for _ in range(25):
        mu, s, q, rho = rand_gauss(rng)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        foot = mu + rng.standard_normal(3) * s.max()
        o = foot + rng.uniform(-50, 50) * d
        sigma = rng.uniform(2.0, 40.0)
        width = rng.uniform(0.5, 2.0) * sigma
        nb = 7
        c = rng.uniform(-30, 30)
        r = oracle.project_tof(one(mu, s, q, rho), o.reshape(3, 1), d.reshape(3, 1), nb, sigma, width,
                               center=[c], kappa=math.inf)
        for b in range(nb):
            tb = c + (b - (nb - 1) / 2) * width
            ref = _tof_quadrature(mu, s, q, rho, o, d, tb, sigma, width)
            assert abs(r["I_kappa"][b, 0] - ref) <= 1e-9 * abs(ref) + 1e-300, (b, r["I_kappa"][b, 0], ref)


def test_tof_bins_sum_to_plain_projection_and_attenuation_scales():
    """Bins of spacing <= 2 sigma that cover the line's mass sum to the plain
    projection (Poisson summation: the relative error is below
    2 exp(-2 pi^2 sigma^2 / width^2)), and attenuation scales every bin."""
    sc = sample_scene(40, seed=42, radius=30.0, scale_range=(1.0, 6.0)).subset(np.arange(40))
    rng = np.random.default_rng(43)
    m = 60
    d = rng.standard_normal((3, m))
    d /= np.linalg.norm(d, axis=0)
    o = rng.uniform(-20, 20, (3, m))
    o -= (o * d).sum(axis=0) * d  # foot points: the line's mass sits within |t| < 60
    sigma, width = 20.0, 15.0
    nb = 2 * int((60 + 10 * sigma) / width) + 1
    atten = rng.uniform(0.1, 1.0, m)
    plain = oracle.project(sc, o, d)
    tof = oracle.project_tof(sc, o, d, nb, sigma, width, center=np.zeros(m), atten=atten)
    s = tof["I_kappa"].sum(axis=0)
    assert np.allclose(s, atten * plain["I_kappa"], rtol=1e-9, atol=1e-300)
    att = oracle.project_tof(sc, o, d, 0, atten=atten)
    assert att["I_kappa"].shape == (1, m)
    assert np.allclose(att["I_kappa"][0], atten * plain["I_kappa"], rtol=1e-14, atol=0)
    assert np.array_equal(oracle.project_tof(sc, o, d, 0)["I_kappa"][0], plain["I_kappa"])
    # shifting the centre by one bin width shifts the outputs by one bin
    sh = oracle.project_tof(sc, o, d, nb, sigma, width, center=np.full(m, width), atten=atten)
    assert np.allclose(sh["I_kappa"][:-1], tof["I_kappa"][1:], rtol=1e-10, atol=1e-300)


def test_narrow_kernel_samples_the_density_at_the_bin_centre():
    """As sigma -> 0 the kernel tends to width * delta(t - tau_b): the bin
    reads width * rho G(o + tau_b d), the density on the line at its centre."""
    rng = np.random.default_rng(44)
    for _ in range(20):
        mu, s, q, rho = rand_gauss(rng)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        o = mu + rng.standard_normal(3) * 0.5 * s.min()
        o -= (o - mu) @ d * d
        nb, width, sigma = 5, 0.7 * s.min(), 1e-4
        r = oracle.project_tof(one(mu, s, q, rho), o.reshape(3, 1), d.reshape(3, 1), nb, sigma, width,
                               kappa=math.inf)
        Pi = sigma_inv_independent(s, q)
        for b in range(nb):
            x = o + (b - (nb - 1) / 2) * width * d - mu
            ref = width * rho * math.exp(-0.5 * x @ Pi @ x)
            assert abs(r["I_kappa"][b, 0] - ref) <= 1e-6 * ref, (b, r["I_kappa"][b, 0], ref)


def _loss_tof(th, o, d, w, nb, sigma, width, center, atten):
    sc = one(th[0:3], th[3:6], th[6:10], th[10])
    return float((w * oracle.project_tof(sc, o, d, nb, sigma, width, center, atten,
                                         kappa=math.inf)["I_kappa"]).sum())


def test_tof_gradient_matches_finite_differences():
    rng = np.random.default_rng(45)
    for trial in range(6):
        mu, s, q, rho = rand_gauss(rng)
        th = np.concatenate([mu, s, q, [rho]])
        m = 12
        d = rng.standard_normal((3, m))
        d /= np.linalg.norm(d, axis=0)
        o = mu[:, None] + rng.standard_normal((3, m)) * s.max() + rng.uniform(-40, 40, m) * d
        nb = 0 if trial == 0 else 5
        sigma, width = rng.uniform(3, 30), rng.uniform(2, 20)
        center = rng.uniform(-20, 20, m)
        atten = rng.uniform(0.2, 1.0, m)
        w = rng.uniform(-1, 1, (max(1, nb), m))
        g = oracle.grad_tof(one(mu, s, q, rho), o, d, w, nb, sigma, width, center, atten, kappa=math.inf)
        fd = np.zeros(11)
        for k in range(11):
            h = 1e-6 * max(1.0, abs(th[k]))
            tp, tm = th.copy(), th.copy()
            tp[k] += h
            tm[k] -= h
            fd[k] = (_loss_tof(tp, o, d, w, nb, sigma, width, center, atten)
                     - _loss_tof(tm, o, d, w, nb, sigma, width, center, atten)) / (2 * h)
        an = g["flat"][0]
        for sl in (slice(0, 3), slice(3, 6), slice(6, 10), slice(10, 11)):
            ref = np.linalg.norm(fd[sl])
            assert np.linalg.norm(an[sl] - fd[sl]) <= 2e-6 * ref + 1e-9 * np.linalg.norm(
                g["flat_abs"][0][sl]) + 1e-14, (trial, sl, an[sl], fd[sl])


def test_gradient_through_abc_matches_envelope_gradient():
    """Without a TOF kernel the gradient through the partials in A, B, C must
    equal the oracle's envelope-theorem gradient (two derivations), and the
    attenuation enters as a factor on the weights."""
    sc = sample_scene(25, seed=46, radius=25.0, scale_range=(1.0, 6.0))
    rng = np.random.default_rng(47)
    m = 400
    d = rng.standard_normal((3, m))
    d /= np.linalg.norm(d, axis=0)
    o = rng.uniform(-25, 25, (3, m))
    w = rng.uniform(-1, 1, m)
    atten = rng.uniform(0.1, 1.0, m)
    a = oracle.grad_tof(sc, o, d, w[None], 0, atten=atten)
    b = oracle.grad(sc, o, d, atten * w)
    scale = np.abs(b["flat_abs"]).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(a["flat"] - b["flat"]) <= 1e-10 * scale)
    assert np.allclose(a["flat_band"], b["flat_band"], rtol=1e-10, atol=1e-300)


def test_pet_tof_centres_are_the_closest_approach_to_the_axis():
    """The TOF centre (midpoint of the line's end points) is where the line
    passes closest to the scanner axis in the transaxial plane, and for an
    arc-corrected line it is equidistant from its two crystals."""
    for arc in (1, 0):
        g = dict(PET_200K["geom"], arc_correct=arc)
        idx = np.random.default_rng(48).integers(0, G.count(g), 4000)
        o, d = G.pet_rays64(g, idx)
        tc = G.pet_tof_centers64(g, idx)
        x = o + tc * d
        assert np.all(np.abs(x[0] * d[0] + x[1] * d[1]) <= 1e-9)
        assert np.abs(tc).max() > 1.0  # oblique lines have off-foot centres
        if arc:
            # both crystals sit on the ring: points at equal |t - tc| reach radius R together
            R = g["ring_radius"]
            a2 = d[0] ** 2 + d[1] ** 2
            r2c = x[0] ** 2 + x[1] ** 2
            half = np.sqrt((R * R - r2c) / a2)
            for sgn in (-1, 1):
                e = x + sgn * half * d
                assert np.allclose(np.hypot(e[0], e[1]), R, rtol=1e-12)


def test_loss_weights_are_the_loss_derivatives():
    rng = np.random.default_rng(49)
    I = rng.uniform(0.1, 5.0, 50)
    y = rng.poisson(3.0, 50).astype(np.float64)
    bg = rng.uniform(0.01, 0.2, 50)
    for kind, b in (("l2", 0.0), ("poisson", bg), ("poisson", 0.05)):
        L, w = oracle.loss_weights(kind, I, y, b)
        h = 1e-6
        for k in range(0, 50, 7):
            e = np.zeros(50)
            e[k] = h
            fd = (oracle.loss_weights(kind, I + e, y, b)[0] - oracle.loss_weights(kind, I - e, y, b)[0]) / (2 * h)
            assert abs(fd - w[k]) <= 1e-6 * max(1.0, abs(w[k]))


def test_loss_values_match_the_likelihoods():
    """The loss values themselves, pinned to scipy's distributions rather than
    to the oracle's own formulas: the L2 loss is the negative Gaussian
    log-likelihood of unit variance less its constant (n/2) log(2 pi), and the
    Poisson loss the negative Poisson log-likelihood of the counts y with mean
    I + b, less the data-only term sum log y! (PET counts are Poisson
    distributed, Sec. 2.1)."""
    from scipy import special, stats
    rng = np.random.default_rng(50)
    n = 200
    I = rng.uniform(0.0, 8.0, n)
    I[:5] = 0.0                      # rays with nothing in reach
    y = rng.poisson(4.0, n).astype(np.float64)
    y[5:10] = 0.0                    # empty bins
    L2, _ = oracle.loss_weights("l2", I, y)
    ref = -stats.norm.logpdf(y, loc=I, scale=1.0).sum() - 0.5 * n * np.log(2.0 * np.pi)
    assert abs(L2 - ref) <= 1e-12 * max(1.0, abs(ref))
    for b in (0.05, rng.uniform(0.01, 0.3, n)):
        Lp, _ = oracle.loss_weights("poisson", I, y, b)
        ref = -stats.poisson.logpmf(y, I + b).sum() - special.gammaln(y + 1.0).sum()
        assert abs(Lp - ref) <= 1e-11 * max(1.0, abs(ref))
    # a planted slip is caught: the Poisson loss without the background
    Lp0, _ = oracle.loss_weights("poisson", I, y, 0.05)
    wrong = -stats.poisson.logpmf(y, I + 0.1).sum() - special.gammaln(y + 1.0).sum()
    assert abs(Lp0 - wrong) > 1e-3
