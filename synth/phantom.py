"""Seeded ellipse phantoms, their exact line integrals, and Poisson noise.

A phantom is a background disk of attenuation 0.02 / mm plus random ellipses
whose values add to whatever lies beneath them.  Random draws, per ellipse and
in this order, from ``numpy.random.default_rng(seed)``:

    r = R_c * sqrt(U), phi = 2 pi U          (centre, uniform over a disk of radius R_c)
    a = s * U[3, 25], b = s * U[3, 25]       (semi-axes, mm)
    alpha = U[0, pi)                         (orientation)
    value = U[-0.01, 0.02]                   (additive attenuation, 1 / mm)

with s = R_disk / 60 and R_c = 45 s.  After the phantom, the same generator
draws the Poisson counts, so a seed fixes the whole case.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .configs import Geometry, Workload, subsample_views

MU_DISK = 0.02


@dataclasses.dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    a: float
    b: float
    alpha: float
    value: float


def draw_phantom(rng: np.random.Generator, w: Workload) -> list[Ellipse]:
    s = w.scale
    r_c = 45.0 * s
    out = [Ellipse(0.0, 0.0, w.disk_radius, w.disk_radius, 0.0, MU_DISK)]
    for _ in range(w.n_ellipses):
        r = r_c * np.sqrt(rng.uniform())
        phi = 2.0 * np.pi * rng.uniform()
        a = s * rng.uniform(3.0, 25.0)
        b = s * rng.uniform(3.0, 25.0)
        alpha = rng.uniform(0.0, np.pi)
        val = rng.uniform(-0.01, 0.02)
        out.append(Ellipse(float(r * np.cos(phi)), float(r * np.sin(phi)), float(a), float(b),
                           float(alpha), float(val)))
    return out


def rasterize(ellipses: list[Ellipse], n: int, pixel: float) -> np.ndarray:
    """Sample the phantom at pixel centres (a centre on the boundary counts as inside)."""
    c = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pixel
    x = c[None, :]
    y = c[:, None]
    img = np.zeros((n, n), dtype=np.float64)
    for e in ellipses:
        ca, sa = np.cos(e.alpha), np.sin(e.alpha)
        dx = x - e.cx
        dy = y - e.cy
        xr = dx * ca + dy * sa
        yr = -dx * sa + dy * ca
        img += e.value * ((xr / e.a) ** 2 + (yr / e.b) ** 2 <= 1.0)
    return img


def line_integrals(ellipses: list[Ellipse], geom: Geometry) -> np.ndarray:
    """Exact line integrals (mm * 1/mm) of the continuous phantom, [n_views, n_bins]."""
    p0, d = geom.rays()
    px, py = p0[..., 0], p0[..., 1]
    dx, dy = d[..., 0], d[..., 1]
    dnorm = np.hypot(dx, dy)
    out = np.zeros(px.shape, dtype=np.float64)
    for e in ellipses:
        ca, sa = np.cos(e.alpha), np.sin(e.alpha)
        qx, qy = px - e.cx, py - e.cy
        # rotate into the ellipse frame and scale to the unit circle
        ux = (qx * ca + qy * sa) / e.a
        uy = (-qx * sa + qy * ca) / e.b
        vx = (dx * ca + dy * sa) / e.a
        vy = (-dx * sa + dy * ca) / e.b
        aa = vx * vx + vy * vy
        bb = ux * vx + uy * vy
        cc = ux * ux + uy * uy - 1.0
        disc = bb * bb - aa * cc
        chord = np.where(disc > 0.0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / aa, 0.0) * dnorm
        out += e.value * chord
    return out


def noisy_sinogram(rng: np.random.Generator, p: np.ndarray, i0: float) -> np.ndarray:
    """Y = -ln(max(Poisson(I0 exp(-p)), 1) / I0); zero counts are clamped to one."""
    counts = rng.poisson(i0 * np.exp(-p)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    return -np.log(counts / i0)


def make_case(w: Workload, seed: int, noise: bool = True) -> dict:
    """One seeded reconstruction case.

    Returns a dict with ``x_true`` [n, n], ``y`` [n_views, n_bins] (noisy, or the
    exact line integrals when ``noise`` is False), ``y_clean`` and the view tables
    ``cos``/``sin``.  A subsampled geometry takes its rows from the full scan's
    noisy sinogram, so 25% data is the same measurement, equally undersampled.
    """
    rng = np.random.default_rng(seed)
    ell = draw_phantom(rng, w)
    g = w.geom
    full = dataclasses.replace(g, n_views=g.n_views_full, view_step=1, n_views_full=g.n_views_full)
    p_full = line_integrals(ell, full)
    y_full = noisy_sinogram(rng, p_full, w.i0) if noise else p_full
    sl = slice(0, g.n_views_full, g.view_step)
    return {
        "x_true": rasterize(ell, g.n, g.pixel),
        "y": np.ascontiguousarray(y_full[sl][: g.n_views]),
        "y_clean": np.ascontiguousarray(p_full[sl][: g.n_views]),
        "cos": g.view_cos,
        "sin": g.view_sin,
        "ellipses": ell,
    }


def batch_cases(w: Workload, seeds, noise: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Stack ``make_case`` over seeds: (x_true [B, n, n], y [B, V, D])."""
    xs, ys = [], []
    for s in seeds:
        c = make_case(w, int(s), noise)
        xs.append(c["x_true"])
        ys.append(c["y"])
    return np.stack(xs), np.stack(ys)


__all__ = ["Ellipse", "draw_phantom", "rasterize", "line_integrals", "noisy_sinogram",
           "make_case", "batch_cases", "subsample_views"]
