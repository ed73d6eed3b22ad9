"""Comparison rules between the HIP path and the FP64 oracle.

Forward: a pair counts iff D <= kappa^2. Pairs whose D lies within a
relative tau = 1e-5 of kappa^2 may flip between FP32 and FP64, so the oracle
returns the sums over D <= kappa^2 (1 - tau) (I_in) and D <= kappa^2 (1 + tau)
(I_hi), and a ray passes when its GPU value lies in
[I_in (1 - tol), I_hi (1 + tol)] with tol = 1e-5 (all densities are >= 0, so
every term is >= 0). A ray with no pair in reach (I_hi = 0) must be exactly 0.

Gradient: per Gaussian and per parameter group (mean, scale, quat, density),
||g_gpu - g_ref|| <= 1e-4 ||g_ref|| + 2e-6 ||sum |per-pair terms| || + ||band terms||,
where the second term is the FP32 summation scale of sums of mixed-sign terms
(10^2 - 10^3 FP32 partial sums per Gaussian and group, whose rounding adds up
like a random walk: sqrt(n) x 6e-8 = 0.6e-6 - 1.9e-6 of the sum of magnitudes)
and the third covers the pairs on the kappa boundary.
"""
from __future__ import annotations

import numpy as np

FWD_TOL = 1e-5
GRAD_REL = 1e-4
GRAD_ABS_SCALE = 2e-6


def forward_report(I_gpu, ref, tol: float = FWD_TOL):
    I = np.asarray(I_gpu, dtype=np.float64)
    lo = ref["I_in"] * (1.0 - tol)
    hi = ref["I_hi"] * (1.0 + tol)
    ok = (I >= lo) & (I <= hi)
    zero = ref["I_hi"] == 0
    ok &= ~zero | (I == 0)
    denom = np.where(ref["I_in"] > 0, ref["I_in"], np.where(ref["I_hi"] > 0, ref["I_hi"], 1.0))
    dist = np.maximum(np.maximum(ref["I_in"] - I, I - ref["I_hi"]), 0.0)
    rel = dist / denom
    return ok, rel


def assert_forward(I_gpu, ref, tol: float = FWD_TOL, what: str = ""):
    ok, rel = forward_report(I_gpu, ref, tol)
    if not ok.all():
        bad = np.nonzero(~ok)[0][:10]
        raise AssertionError(f"{what}: {int((~ok).sum())} of {ok.size} rays outside tolerance; "
                             f"max rel {rel.max():.3e}; first bad {bad.tolist()} "
                             f"gpu {np.asarray(I_gpu)[bad].tolist()} ref {ref['I_kappa'][bad].tolist()}")
    return float(rel.max()) if rel.size else 0.0


GROUPS = {"mean": slice(0, 3), "scale": slice(3, 6), "quat": slice(6, 10), "density": slice(10, 11)}


def gpu_grad_rows(grads, idx):
    """(k, 11) float64 rows mean, scale, quat, density for Gaussians idx."""
    idx = np.asarray(idx)
    m = grads["mean"].detach().cpu().double().numpy()[:, idx].T
    s = grads["scale"].detach().cpu().double().numpy()[:, idx].T
    q = grads["quat"].detach().cpu().double().numpy()[:, idx].T
    d = grads["density"].detach().cpu().double().numpy()[idx][:, None]
    return np.concatenate([m, s, q, d], axis=1)


def assert_grad(g_gpu_rows, ref, what: str = ""):
    worst = 0.0
    for name, sl in GROUPS.items():
        got = g_gpu_rows[:, sl]
        want = ref["flat"][:, sl]
        err = np.linalg.norm(got - want, axis=1)
        tol = (GRAD_REL * np.linalg.norm(want, axis=1)
               + GRAD_ABS_SCALE * np.linalg.norm(ref["flat_abs"][:, sl], axis=1)
               + np.linalg.norm(ref["flat_band"][:, sl], axis=1))
        bad = err > tol
        if bad.any():
            i = int(np.nonzero(bad)[0][0])
            raise AssertionError(f"{what} {name}: {int(bad.sum())} Gaussians out of tolerance; first "
                                 f"#{i}: err {err[i]:.3e} tol {tol[i]:.3e} got {got[i]} want {want[i]}")
        nz = np.linalg.norm(want, axis=1) > 0
        if nz.any():
            worst = max(worst, float((err[nz] / np.linalg.norm(want, axis=1)[nz]).max()))
    return worst


def grad_abs_term_report(g_gpu_rows, ref):
    """How many (Gaussian, group) gradients pass the bar only thanks to its
    absolute FP32-summation term: err > 1e-4 ||g_ref|| + band, yet within the
    full tolerance. Returns (that count, the number of non-zero reference
    gradients, the largest err / (GRAD_ABS_SCALE sum |per-pair terms|) among them)."""
    n_abs, n_nz, worst = 0, 0, 0.0
    for sl in GROUPS.values():
        got = g_gpu_rows[:, sl]
        want = ref["flat"][:, sl]
        err = np.linalg.norm(got - want, axis=1)
        rel_part = GRAD_REL * np.linalg.norm(want, axis=1) + np.linalg.norm(ref["flat_band"][:, sl], axis=1)
        abs_part = GRAD_ABS_SCALE * np.linalg.norm(ref["flat_abs"][:, sl], axis=1)
        nz = np.linalg.norm(want, axis=1) > 0
        need = nz & (err > rel_part) & (err <= rel_part + abs_part)
        n_abs += int(need.sum())
        n_nz += int(nz.sum())
        if need.any():
            worst = max(worst, float(((err - rel_part)[need] / abs_part[need]).max()))
    return n_abs, n_nz, worst
