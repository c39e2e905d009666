"""Seeded synthetic inputs for the AIR reconstruction path.

This package draws phantoms, computes their exact (continuous) line
integrals for a given scan geometry, adds Poisson noise and provides the
per-view cosine/sine tables.  It is shared by the FP64 oracle and the GPU
library as their common source of inputs; it contains none of the
reconstruction arithmetic (no discrete projector, filter, framelet or
solver).  The paper's experimental scan (a physical image-quality phantom
on a megavoltage CT) is not available, so these phantoms stand in for it.
"""
from .configs import Geometry, Workload, CONFIGS, workload, subsample_views
from .phantom import Ellipse, draw_phantom, rasterize, line_integrals, noisy_sinogram, make_case

__all__ = [
    "Geometry", "Workload", "CONFIGS", "workload", "subsample_views",
    "Ellipse", "draw_phantom", "rasterize", "line_integrals", "noisy_sinogram", "make_case",
]
