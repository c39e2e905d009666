"""Scan geometries and workloads for the synthetic AIR experiments.

Conventions (shared by every consumer of these inputs):

* Image: ``n x n`` square pixels of side ``pixel`` (mm), centred on the
  isocentre; pixel (i, j) has centre ((i - (n-1)/2) * pixel, (j - (n-1)/2) * pixel),
  i the column (x), j the row (y).  Arrays are stored ``[j][i]``.
* Detector bin k has centre coordinate ``u_k = (k - (n_bins-1)/2) * bin`` (mm)
  along the detector axis.
* Parallel beam, view angle theta: detector axis e = (cos, sin), ray through
  u_k * e with direction (-sin, cos).  Angles theta_v = pi * v / V on [0, pi).
* Fan beam with a flat detector, source angle beta: source s = sod * (cos, sin),
  detector axis w = (-sin, cos) on the plane at distance ``sdd`` from the source;
  the ray for bin k runs from s towards s - sdd * (cos, sin) + u_k * w.
  Angles beta_v = 2 pi v / V on [0, 2 pi).
* "25% data" keeps every 4th view of the full scan (equal undersampling, as in
  the paper's Materials section): the same rows of the same noisy sinogram.

The view cosine/sine tables are computed here once (numpy, float64) and handed
to both the oracle and the GPU library, so neither side's libm enters them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    beam: str                 # "parallel" or "fan"
    n: int                    # image is n x n pixels
    pixel: float              # pixel side (mm)
    n_views: int              # number of views in this geometry
    n_bins: int               # detector bins per view
    bin: float                # detector pitch (mm)
    sod: float = 0.0          # source to isocentre (fan only, mm)
    sdd: float = 0.0          # source to detector (fan only, mm)
    view_step: int = 1        # stride into the full view set (4 for 25% data)
    n_views_full: int = 0     # views of the full scan this one is drawn from

    def __post_init__(self):
        if self.beam not in ("parallel", "fan"):
            raise ValueError(f"unknown beam {self.beam!r}")
        if self.n_views_full == 0:
            object.__setattr__(self, "n_views_full", self.n_views * self.view_step)

    @property
    def angles(self) -> np.ndarray:
        """View angles (radians, float64) of the views this geometry keeps."""
        full = self.n_views_full
        period = math.pi if self.beam == "parallel" else 2.0 * math.pi
        v = np.arange(0, full, self.view_step, dtype=np.float64)[: self.n_views]
        return period * v / full

    @property
    def view_cos(self) -> np.ndarray:
        return np.ascontiguousarray(np.cos(self.angles))

    @property
    def view_sin(self) -> np.ndarray:
        return np.ascontiguousarray(np.sin(self.angles))

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_bins

    def rays(self) -> tuple[np.ndarray, np.ndarray]:
        """Ray origin and direction, each [n_views, n_bins, 2] float64.

        Origins lie on the ray (bin point for parallel beam, the source for fan
        beam); directions are not normalised.
        """
        c = self.view_cos[:, None]
        s = self.view_sin[:, None]
        u = (np.arange(self.n_bins, dtype=np.float64) - 0.5 * (self.n_bins - 1)) * self.bin
        u = u[None, :]
        if self.beam == "parallel":
            p0 = np.stack(np.broadcast_arrays(u * c, u * s), axis=-1)
            d = np.stack(np.broadcast_arrays(-s + 0 * u, c + 0 * u), axis=-1)
        else:
            p0 = np.stack(np.broadcast_arrays(self.sod * c + 0 * u, self.sod * s + 0 * u), axis=-1)
            d = np.stack(np.broadcast_arrays(-self.sdd * c - u * s, -self.sdd * s + u * c), axis=-1)
        return np.ascontiguousarray(p0), np.ascontiguousarray(d)


def subsample_views(g: Geometry, step: int) -> Geometry:
    """Keep every ``step``-th view of ``g`` (e.g. step=4 gives 25% data)."""
    if g.n_views % step:
        raise ValueError("view count must be divisible by the step")
    return dataclasses.replace(g, n_views=g.n_views // step, view_step=g.view_step * step,
                               n_views_full=g.n_views_full)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    geom: Geometry
    disk_radius: float        # background disk (mm), attenuation 0.02 / mm
    n_ellipses: int
    i0: float                 # incident photon count per ray
    lam: float = 0.005        # framelet weight (lambda)
    mu: float = 1.0           # Bregman penalty (mu)
    n_outer: int = 10
    n_cg: int = 5
    batch: int = 1

    @property
    def scale(self) -> float:
        """Size scale of the random ellipses relative to the 60 mm reference disk."""
        return self.disk_radius / 60.0


def _c1() -> Workload:
    g = Geometry("parallel", n=128, pixel=1.0, n_views=180, n_bins=185, bin=1.0)
    return Workload("c1_parallel_128", g, disk_radius=60.0, n_ellipses=8, i0=1e5,
                    n_outer=10, n_cg=5)


def _c2() -> Workload:
    g = Geometry("fan", n=512, pixel=0.78, n_views=720, n_bins=736, bin=1.2, sod=850.0, sdd=1450.0)
    return Workload("c2_fan_512_720", g, disk_radius=190.0, n_ellipses=20, i0=2e4,
                    n_outer=50, n_cg=5)


def _c3() -> Workload:
    w = _c1()
    return dataclasses.replace(w, name="c3_parallel_128_b64", batch=64)


def _c5() -> Workload:
    g = Geometry("fan", n=1024, pixel=0.39, n_views=2304, n_bins=1536, bin=0.6, sod=850.0, sdd=1450.0)
    return Workload("c5_fan_1024_2304", g, disk_radius=190.0, n_ellipses=40, i0=5e4,
                    n_outer=50, n_cg=5, batch=16)


def serving_geometry(n: int, n_views: int, step: int = 1) -> Geometry:
    """Fan-beam geometry of the serving mix: pixel 0.78 mm, 1.2 mm bins,
    n_bins = 1.4375 * n (736 at n = 512), over 2 pi."""
    g = Geometry("fan", n=n, pixel=0.78, n_views=n_views, n_bins=(n * 23) // 16, bin=1.2,
                 sod=850.0, sdd=1450.0)
    return subsample_views(g, step) if step > 1 else g


CONFIGS = {"c1": _c1, "c2": _c2, "c3": _c3, "c5": _c5}


def workload(name: str, **overrides) -> Workload:
    """Named workload, optionally with fields replaced (e.g. n_outer=2)."""
    if name == "c2_25":
        w = _c2()
        w = dataclasses.replace(w, name="c2_fan_512_180", geom=subsample_views(w.geom, 4))
    else:
        w = CONFIGS[name]()
    return dataclasses.replace(w, **overrides) if overrides else w
