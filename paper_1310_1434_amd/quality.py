"""Image-quality measures for comparing reconstructions of the quality
phantoms: contrast-to-noise ratio of disc targets and full width at half
maximum of bar profiles (the two measures of the paper's Results section).

These run on the host, on finished images; they are evaluation, not part of
the reconstruction path.  Images are [j][i] arrays with pixel centres at
((i - (n-1)/2) pixel, (j - (n-1)/2) pixel).

Readings where the paper gives no definition:

* CNR = |mu_t - mu_b| / sqrt(sigma_t^2 + sigma_b^2) over the pixel centres of
  the target disc and the background annulus, sigma the population standard
  deviation (the Results section states the formula, not the estimator).
* FWHM of a bar: the profile across the group is sampled bilinearly every
  0.1 mm; the bar's peak is the maximum within one bar width of its nominal
  centre, its base the mean of the minima within two bar widths on either side
  (the neighbouring gaps, or the background past the group's ends); the width
  is taken where the profile crosses halfway between base and peak, with
  linear interpolation between samples.  A bar whose profile does not fall
  below the half level on both sides within two widths is unresolved (NaN).
"""
from __future__ import annotations

import math

import numpy as np


def cnr(img: np.ndarray, target: np.ndarray, background: np.ndarray) -> float:
    t = np.asarray(img, np.float64)[target]
    b = np.asarray(img, np.float64)[background]
    return float(abs(t.mean() - b.mean()) / math.sqrt(t.var() + b.var()))


def sample_bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray, pixel: float) -> np.ndarray:
    """Bilinear interpolation of the image at points (x, y) in mm (inside the image)."""
    n = img.shape[0]
    fi = np.asarray(x, np.float64) / pixel + 0.5 * (n - 1)
    fj = np.asarray(y, np.float64) / pixel + 0.5 * (n - 1)
    i0 = np.clip(np.floor(fi).astype(int), 0, n - 2)
    j0 = np.clip(np.floor(fj).astype(int), 0, n - 2)
    a, b = fi - i0, fj - j0
    im = np.asarray(img, np.float64)
    return ((1 - a) * (1 - b) * im[j0, i0] + a * (1 - b) * im[j0, i0 + 1] +
            (1 - a) * b * im[j0 + 1, i0] + a * b * im[j0 + 1, i0 + 1])


def _crossing(s: np.ndarray, f: np.ndarray, k_from: int, k_to: int, level: float) -> float:
    """First point from index k_from towards k_to where f falls below level
    (linear interpolation), or NaN if it never does."""
    step = 1 if k_to > k_from else -1
    for k in range(k_from + step, k_to + step, step):
        if f[k] < level:
            kp = k - step
            t = (f[kp] - level) / (f[kp] - f[k])
            return float(s[kp] + t * (s[k] - s[kp]))
    return float("nan")


def peak_fwhm(s: np.ndarray, f: np.ndarray, centre: float, width: float) -> float:
    """FWHM of the peak of profile f(s) nearest `centre` (see the module docstring)."""
    s = np.asarray(s, np.float64)
    f = np.asarray(f, np.float64)
    near = np.abs(s - centre) <= width
    kp = int(np.flatnonzero(near)[np.argmax(f[near])])
    left = (s >= centre - 2 * width) & (s <= centre)
    right = (s >= centre) & (s <= centre + 2 * width)
    base = 0.5 * (f[left].min() + f[right].min())
    half = base + 0.5 * (f[kp] - base)
    k_lo = int(np.flatnonzero(left)[0])
    k_hi = int(np.flatnonzero(right)[-1])
    sl = _crossing(s, f, kp, k_lo, half)
    sr = _crossing(s, f, kp, k_hi, half)
    return sr - sl


def bar_fwhm(img: np.ndarray, group, pixel: float, step: float = 0.1) -> dict:
    """FWHM of every bar of a bar group (synth.quality.BarGroup) and their mean."""
    from synth.quality import bar_profile_line

    x, y, s = bar_profile_line(group, step=step)
    f = sample_bilinear(img, x, y, pixel)
    per = [peak_fwhm(s, f, c, group.width) for c in group.centres()]
    ok = [w for w in per if np.isfinite(w)]
    return {"lp_per_cm": group.lp_per_cm, "bar_mm": group.width, "fwhm_mm": float(np.mean(ok)) if ok else float("nan"),
            "resolved": len(ok) == len(per), "per_bar_mm": per}


def target_cnrs(img: np.ndarray, phantom, pixel: float) -> list:
    from synth.quality import target_rois

    out = []
    for t in phantom.targets:
        tm, bm = target_rois(t, img.shape[0], pixel)
        out.append({"radius_mm": t.radius, "contrast": t.contrast, "cnr": cnr(img, tm, bm)})
    return out


__all__ = ["cnr", "sample_bilinear", "peak_fwhm", "bar_fwhm", "target_cnrs"]


# ---------------------------------------------------------------------------- the three arms
def power_start(n: int, seed: int = 0) -> np.ndarray:
    """Seeded start vector of the power iteration, [n, n] float32."""
    return np.random.default_rng(seed).uniform(size=(n, n)).astype(np.float32)


def top_eigenvalue(plan, filter: int, iters: int = 30, seed: int = 0) -> float:
    """Largest eigenvalue of the normal operator (A'^T A for filter 1, A^T A for
    filter 0): `iters` power-iteration steps on the GPU library from
    power_start(n, seed); the estimate is |M x| / |x| at the last step."""
    import torch

    x = torch.from_numpy(power_start(plan.n, seed)[None]).to(plan.device)
    lam = 0.0
    for _ in range(iters):
        y = plan.normal_apply(x, 0.0, filter)
        lam = float(torch.linalg.vector_norm(y.double()) / torch.linalg.vector_norm(x.double()))
        x = y / torch.linalg.vector_norm(y)
    return lam


def run_arms(plan, y, lam: float, mu: float, n_outer: int, n_cg: int, ir_scale: float) -> dict:
    """FBP, IR and AIR reconstructions of sinograms y [B, V, D] (device tensor).

    FBP is the filtered adjoint A'^T Y.  AIR is the split-Bregman solve with
    A'^T; IR the same solve with A^T, its lambda and mu multiplied by ir_scale
    (the ratio of the two normal operators' largest eigenvalues), so that both
    weigh the prior against data terms of the same curvature; the shrinkage
    threshold lambda / (2 mu) is the same for both."""
    fbp = plan.filtered_backproject(y, filter=1)
    air_x, _ = plan.solve(y, lam, mu, n_outer, n_cg, filter=1)
    ir_x, _ = plan.solve(y, lam * ir_scale, mu * ir_scale, n_outer, n_cg, filter=0)
    return {"FBP": fbp, "IR": ir_x, "AIR": air_x}


__all__ += ["power_start", "top_eigenvalue", "run_arms"]
