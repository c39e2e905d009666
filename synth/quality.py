"""Image-quality phantoms for the FBP / IR / AIR comparison, with their
measurement regions.

Two slices stand in for the physical image-quality phantom of the paper's
Materials section (which is not available): a *resolution* slice with groups
of high-contrast bars at several line-pair frequencies, measured by the full
width at half maximum of the bar profiles, and a *contrast* slice with
low-contrast disc targets, measured by the contrast-to-noise ratio between a
disc region inside each target and an annulus of background around it.  Both
sit in a water-like disc of attenuation 0.02 / mm.  Shapes are ellipses and
rotated rectangles with exact line integrals, so the sinogram is the
continuous phantom's, not a discrete projector's.

The geometry follows the paper's scan as far as it is stated: a 350 x 350
image of 1 mm pixels and 528 detector bins, with 800 views per rotation (100%
data) or every 4th of them (25% data).  The fan-beam distances and the bin
pitch are not stated; source-to-isocentre 850 mm, source-to-detector 1450 mm
and a 1.1 mm pitch (the detector then spans the whole 150 mm phantom disc, the
field of view being the inscribed circle of the image) stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .configs import Geometry, subsample_views
from .phantom import Ellipse, line_integrals as ellipse_line_integrals, noisy_sinogram, rasterize as rasterize_ellipses

MU_WATER = 0.02
DISC_RADIUS = 150.0


def paper_geometry(step: int = 1) -> Geometry:
    """350^2 x 1 mm, 528 bins, 800 views over 2 pi (step 4: the 200-view subset)."""
    g = Geometry("fan", n=350, pixel=1.0, n_views=800, n_bins=528, bin=1.1, sod=850.0, sdd=1450.0)
    return subsample_views(g, step) if step > 1 else g


@dataclasses.dataclass(frozen=True)
class Rect:
    """Rectangle of half-sizes (hx, hy) about (cx, cy), rotated by alpha."""
    cx: float
    cy: float
    hx: float
    hy: float
    alpha: float
    value: float


def rect_line_integrals(rects: list[Rect], geom: Geometry) -> np.ndarray:
    """Exact line integrals of rectangles along every ray, [n_views, n_bins].

    In the rectangle's frame a ray p + t d is inside while |x| <= hx and
    |y| <= hy: the intersection of two parameter slabs (empty if the ray runs
    parallel to a slab it lies outside of)."""
    p0, d = geom.rays()
    px, py = p0[..., 0], p0[..., 1]
    dx, dy = d[..., 0], d[..., 1]
    dnorm = np.hypot(dx, dy)
    out = np.zeros(px.shape, dtype=np.float64)
    for r in rects:
        ca, sa = math.cos(r.alpha), math.sin(r.alpha)
        qx, qy = px - r.cx, py - r.cy
        ux, uy = qx * ca + qy * sa, -qx * sa + qy * ca
        vx, vy = dx * ca + dy * sa, -dx * sa + dy * ca
        t_lo = np.full(px.shape, -np.inf)
        t_hi = np.full(px.shape, np.inf)
        for u, v, h in ((ux, vx, r.hx), (uy, vy, r.hy)):
            moving = np.abs(v) > 1e-300
            with np.errstate(divide="ignore", invalid="ignore"):
                a = np.where(moving, (-h - u) / v, -np.inf)
                b = np.where(moving, (h - u) / v, np.inf)
            lo, hi = np.minimum(a, b), np.maximum(a, b)
            outside = ~moving & (np.abs(u) > h)
            lo = np.where(outside, np.inf, lo)
            hi = np.where(outside, -np.inf, hi)
            t_lo = np.maximum(t_lo, lo)
            t_hi = np.minimum(t_hi, hi)
        out += r.value * np.maximum(t_hi - t_lo, 0.0) * dnorm
    return out


def rasterize_rects(rects: list[Rect], n: int, pixel: float) -> np.ndarray:
    c = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pixel
    x, y = c[None, :], c[:, None]
    img = np.zeros((n, n), dtype=np.float64)
    for r in rects:
        ca, sa = math.cos(r.alpha), math.sin(r.alpha)
        xr = (x - r.cx) * ca + (y - r.cy) * sa
        yr = -(x - r.cx) * sa + (y - r.cy) * ca
        img += r.value * ((np.abs(xr) <= r.hx) & (np.abs(yr) <= r.hy))
    return img


@dataclasses.dataclass(frozen=True)
class BarGroup:
    """Four bars of width w = 10 / (2 lp) mm (gaps of w), long axis along the
    direction (-sin phi, cos phi); the profile runs across them along (cos phi, sin phi)."""
    lp_per_cm: float
    cx: float
    cy: float
    phi: float
    length: float = 14.0
    bars: int = 4

    @property
    def width(self) -> float:
        return 10.0 / (2.0 * self.lp_per_cm)

    def centres(self) -> np.ndarray:
        """Offsets of the bar centres along the profile direction (mm)."""
        return (np.arange(self.bars) - 0.5 * (self.bars - 1)) * 2.0 * self.width


@dataclasses.dataclass(frozen=True)
class Target:
    cx: float
    cy: float
    radius: float
    contrast: float          # added attenuation, 1 / mm


@dataclasses.dataclass(frozen=True)
class QualityPhantom:
    name: str
    ellipses: tuple
    rects: tuple
    bar_groups: tuple = ()
    targets: tuple = ()

    def image(self, n: int, pixel: float) -> np.ndarray:
        return rasterize_ellipses(list(self.ellipses), n, pixel) + rasterize_rects(list(self.rects), n, pixel)

    def line_integrals(self, geom: Geometry) -> np.ndarray:
        p = ellipse_line_integrals(list(self.ellipses), geom)
        if self.rects:
            p = p + rect_line_integrals(list(self.rects), geom)
        return p


def resolution_phantom(bar_value: float = 0.02, lps=(2.0, 3.0, 4.0, 5.0), ring: float = 70.0,
                       disc: float = DISC_RADIUS, length: float = 14.0) -> QualityPhantom:
    """Water disc with one bar group per frequency on a ring (each group's
    profile direction tangent to the ring, the bars across it)."""
    groups, rects = [], []
    for k, lp in enumerate(lps):
        ang = 2.0 * math.pi * k / len(lps) + math.pi / 8
        cx, cy = ring * math.cos(ang), ring * math.sin(ang)
        phi = ang + math.pi / 2              # profile along the tangent
        gr = BarGroup(lp, cx, cy, phi, length=length)
        groups.append(gr)
        for off in gr.centres():
            rects.append(Rect(cx + off * math.cos(phi), cy + off * math.sin(phi), gr.width / 2, gr.length / 2,
                              phi, bar_value))
    water = Ellipse(0.0, 0.0, disc, disc, 0.0, MU_WATER)
    return QualityPhantom("resolution", (water,), tuple(rects), bar_groups=tuple(groups))


def contrast_phantom(contrasts=(0.0005, 0.001, 0.002, 0.004), radii=(12.0, 8.0), ring: float = 80.0,
                     disc: float = DISC_RADIUS) -> QualityPhantom:
    """Water disc with disc targets of the given added attenuation (2.5% to 20%
    of water) and radii, evenly spaced on a ring."""
    targets = []
    items = [(c, r) for r in radii for c in contrasts]
    for k, (c, r) in enumerate(items):
        ang = 2.0 * math.pi * k / len(items)
        targets.append(Target(ring * math.cos(ang), ring * math.sin(ang), r, c))
    ell = [Ellipse(0.0, 0.0, disc, disc, 0.0, MU_WATER)]
    ell += [Ellipse(t.cx, t.cy, t.radius, t.radius, 0.0, t.contrast) for t in targets]
    return QualityPhantom("contrast", tuple(ell), (), targets=tuple(targets))


def make_quality_case(ph: QualityPhantom, geom: Geometry, i0: float, seed: int) -> dict:
    """Noisy sinogram of a quality phantom.  The 25% geometry takes every 4th
    row of the full scan's noisy sinogram (the same measurement)."""
    full = dataclasses.replace(geom, n_views=geom.n_views_full, view_step=1, n_views_full=geom.n_views_full)
    p_full = ph.line_integrals(full)
    rng = np.random.default_rng(seed)
    y_full = noisy_sinogram(rng, p_full, i0)
    sl = slice(0, geom.n_views_full, geom.view_step)
    return {"x_true": ph.image(geom.n, geom.pixel), "y": np.ascontiguousarray(y_full[sl][: geom.n_views])}


def target_rois(t: Target, n: int, pixel: float, inner: float = 0.6, ann=(1.5, 2.2)):
    """Boolean masks (pixel centres): the disc of radius inner * r inside the
    target, and the background annulus between ann[0] * r and ann[1] * r."""
    c = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pixel
    rr = np.hypot(c[None, :] - t.cx, c[:, None] - t.cy)
    return rr <= inner * t.radius, (rr >= ann[0] * t.radius) & (rr <= ann[1] * t.radius)


def bar_profile_line(gr: BarGroup, step: float = 0.1, margin: float = 2.0):
    """Points (x, y) and offsets s of a line across a bar group's centre,
    covering the group plus `margin` bar widths on both sides."""
    half = 0.5 * (gr.bars * 2 - 1) * gr.width + margin * gr.width
    s = np.arange(-half, half + 0.5 * step, step)
    return gr.cx + s * math.cos(gr.phi), gr.cy + s * math.sin(gr.phi), s


__all__ = ["paper_geometry", "Rect", "rect_line_integrals", "rasterize_rects", "BarGroup", "Target",
           "QualityPhantom", "resolution_phantom", "contrast_phantom", "make_quality_case", "target_rois",
           "bar_profile_line", "MU_WATER"]
