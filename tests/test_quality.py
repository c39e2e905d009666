"""CPU checks of the image-quality phantoms and measures (CNR, FWHM).

Pins: exact rectangle chords against closed forms and brute-force ray
marching; FWHM of sampled Gaussians against 2 sqrt(2 ln 2) sigma; FWHM of an
ideal bar pattern against the bar width; CNR of constructed samples against
its formula; ROI areas against pi r^2."""
import math

import numpy as np
import pytest

from paper_1310_1434_amd import quality as Q
from synth import quality as SQ
from synth.configs import Geometry


def test_rect_chords_axis_aligned_closed_form():
    # parallel beam, view 0: rays run along +y at x = u_k; an axis-aligned
    # rectangle gives chord 2 hy for |u_k - cx| < hx and 0 outside
    g = Geometry("parallel", n=32, pixel=1.0, n_views=1, n_bins=41, bin=0.5)
    r = SQ.Rect(1.3, -2.0, 3.0, 4.5, 0.0, 0.7)
    p = SQ.rect_line_integrals([r], g)[0]
    u = (np.arange(41) - 20) * 0.5
    want = np.where(np.abs(u - 1.3) < 3.0, 0.7 * 9.0, 0.0)
    assert np.allclose(p, want, atol=1e-12)


def test_rect_chords_rotated_brute_force():
    g = Geometry("fan", n=64, pixel=1.0, n_views=7, n_bins=50, bin=1.5, sod=100.0, sdd=180.0)
    r = SQ.Rect(3.0, -2.0, 5.0, 2.5, 0.7, 1.0)
    p = SQ.rect_line_integrals([r], g)
    p0, d = g.rays()
    t = np.linspace(0.0, 1.2, 100001)
    dt = t[1] - t[0]
    x = p0[..., 0:1] + t * d[..., 0:1]
    y = p0[..., 1:2] + t * d[..., 1:2]
    ca, sa = math.cos(r.alpha), math.sin(r.alpha)
    xr = (x - r.cx) * ca + (y - r.cy) * sa
    yr = -(x - r.cx) * sa + (y - r.cy) * ca
    bf = ((np.abs(xr) <= r.hx) & (np.abs(yr) <= r.hy)).sum(-1) * dt * np.hypot(d[..., 0], d[..., 1])
    step = dt * np.hypot(d[..., 0], d[..., 1]).max()
    assert np.abs(bf - p).max() <= 2.5 * step
    assert p.max() > 9.0


def test_gaussian_fwhm():
    s = np.arange(-20.0, 20.0, 0.01)
    for sigma in (0.8, 1.5, 3.0):
        f = 0.3 + np.exp(-s ** 2 / (2 * sigma ** 2))
        w = Q.peak_fwhm(s, f, 0.0, 3.5 * sigma)
        assert abs(w - 2.0 * math.sqrt(2.0 * math.log(2.0)) * sigma) < 2e-3 * sigma


def test_ideal_bar_pattern_fwhm_equals_bar_width():
    pixel = 0.05
    ph = SQ.resolution_phantom(lps=(2.0, 4.0), ring=4.0, disc=18.0, length=3.0)
    img = ph.image(800, pixel)
    for gr in ph.bar_groups:
        r = Q.bar_fwhm(img, gr, pixel, step=0.01)
        assert r["resolved"]
        assert abs(r["fwhm_mm"] - gr.width) < 1.5 * pixel, (gr.lp_per_cm, r)


def test_shallow_modulation_is_resolved_and_a_ramp_is_not():
    s = np.arange(-10.0, 10.0, 0.005)
    f = 1.0 + 0.05 * np.cos(2 * np.pi * s / 2.0)      # period 2 w, w = 1: FWHM = w whatever the depth
    assert Q.peak_fwhm(s, f, 0.0, 1.0) == pytest.approx(1.0, abs=1e-3)
    assert np.isnan(Q.peak_fwhm(s, 0.1 * s, 0.0, 1.0))  # no peak: never falls below half on the right


def test_cnr_constructed():
    img = np.zeros((4, 8))
    t = np.zeros_like(img, bool)
    b = np.zeros_like(img, bool)
    t[:2] = True
    b[2:] = True
    img[:2] = np.where(np.arange(8) % 2, 0.025, 0.021)       # mean 0.023, std 0.002
    img[2:] = np.where(np.arange(8) % 2, 0.0205, 0.0195)     # mean 0.020, std 0.0005
    assert Q.cnr(img, t, b) == pytest.approx(0.003 / math.sqrt(0.002 ** 2 + 0.0005 ** 2), rel=1e-12)


def test_target_roi_areas():
    t = SQ.Target(10.0, -5.0, 8.0, 0.001)
    tm, bm = SQ.target_rois(t, 320, 0.25)
    assert tm.sum() * 0.25 ** 2 == pytest.approx(math.pi * (0.6 * 8.0) ** 2, rel=0.02)
    assert bm.sum() * 0.25 ** 2 == pytest.approx(math.pi * ((2.2 * 8.0) ** 2 - (1.5 * 8.0) ** 2), rel=0.02)
    assert not (tm & bm).any()


def test_quality_case_subset_is_the_same_measurement():
    g = Geometry("fan", n=48, pixel=1.0, n_views=40, n_bins=80, bin=1.1, sod=200.0, sdd=350.0)
    g25 = SQ.subsample_views(g, 4)
    ph = SQ.contrast_phantom(radii=(4.0,), ring=12.0, disc=20.0)
    full = SQ.make_quality_case(ph, g, 1e4, 3)
    sub = SQ.make_quality_case(ph, g25, 1e4, 3)
    assert np.array_equal(sub["y"], full["y"][::4])
    assert np.array_equal(full["y"], SQ.make_quality_case(ph, g, 1e4, 3)["y"])


def test_paper_geometry_covers_the_phantom_disc():
    g = SQ.paper_geometry()
    assert (g.n, g.pixel, g.n_bins, g.n_views) == (350, 1.0, 528, 800)
    assert SQ.paper_geometry(4).n_views == 200
    half = 0.5 * g.n_bins * g.bin
    need = g.sdd * SQ.DISC_RADIUS / math.sqrt(g.sod ** 2 - SQ.DISC_RADIUS ** 2)
    assert half > need
