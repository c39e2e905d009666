"""Pins for the FP64 oracle: each test ties one part of it to something
other than itself -- a closed form, an invariant the paper relies on, a
library routine, or brute force on a tiny case.

Paper references: Methods, Eqs. (1)-(5) and the split Bregman L2 step;
Materials for the tensor framelet and FBP as the analytic method.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.signal

import synth
from synth.configs import Geometry


def geom_custom(beam, n, pixel, angles, n_bins, bin, sod=0.0, sdd=0.0):
    """A synth.Geometry-like object with explicit view angles or (cos, sin) pairs."""

    class G:
        pass

    g = G()
    g.beam, g.n, g.pixel, g.n_bins, g.bin, g.sod, g.sdd = beam, n, pixel, n_bins, bin, sod, sdd
    if isinstance(angles, tuple):
        g.view_cos, g.view_sin = np.asarray(angles[0], float), np.asarray(angles[1], float)
    else:
        g.view_cos, g.view_sin = np.cos(angles), np.sin(angles)
    g.n_views = len(g.view_cos)
    return g


# ----------------------------------------------------------------------------- A: closed forms

def test_axis_aligned_rays_give_column_and_row_sums(orc):
    """Rays along the pixel grid through pixel centres: A x = pixel * line sums exactly."""
    n, pix = 9, 1.5
    g = orc.Geom(geom_custom("parallel", n, pix, ([1.0, 0.0], [0.0, 1.0]), n, pix))
    x = np.random.default_rng(1).standard_normal((n, n))
    y = orc.project(g, x)
    # view 0 (theta = 0): vertical rays at x = u_k -> column sums
    np.testing.assert_allclose(y[0], pix * x.sum(axis=0), rtol=0, atol=1e-12)
    # view 1 (theta = pi/2): horizontal rays at y = u_k -> row sums
    np.testing.assert_allclose(y[1], pix * x.sum(axis=1), rtol=0, atol=1e-12)


def test_diagonal_rays_give_scaled_diagonal_sums(orc):
    """45-degree rays through pixel centres (bin pitch pixel/sqrt2): A x = sqrt2 * pixel * anti-diagonal sums."""
    n, pix = 8, 1.0
    c = math.sqrt(0.5)
    g = orc.Geom(geom_custom("parallel", n, pix, ([c], [c]), 2 * n - 1, pix * c))
    x = np.random.default_rng(2).standard_normal((n, n))
    y = orc.project(g, x)[0]
    jj, ii = np.mgrid[0:n, 0:n]
    sums = np.array([x[(ii + jj) == k].sum() for k in range(2 * n - 1)])
    np.testing.assert_allclose(y, math.sqrt(2.0) * pix * sums, rtol=0, atol=1e-12)


def _gaussian_line_integral(p0, d, cx, cy, sigma):
    """Closed-form line integral of exp(-|r - c|^2 / sigma^2) along p0 + t d."""
    dn = np.hypot(d[..., 0], d[..., 1])
    cross = ((cx - p0[..., 0]) * d[..., 1] - (cy - p0[..., 1]) * d[..., 0]) / dn
    return sigma * math.sqrt(math.pi) * np.exp(-(cross ** 2) / sigma ** 2)


def _gaussian_image(n, pix, cx, cy, sigma):
    c = (np.arange(n) - 0.5 * (n - 1)) * pix
    return np.exp(-((c[None, :] - cx) ** 2 + (c[:, None] - cy) ** 2) / sigma ** 2)


@pytest.mark.parametrize("beam", ["parallel", "fan"])
def test_off_centre_gaussian_matches_analytic_projection(orc, beam):
    """An off-centre Gaussian blob pins rotation direction, bin orientation, centring
    and path-length scaling; the Joseph (linear-interpolation) error is O(pixel^2)."""
    cx, cy, sigma = 21.0, -13.0, 9.0
    errs = []
    for n, pix in [(48, 2.0), (96, 1.0), (192, 0.5)]:
        if beam == "parallel":
            geo = Geometry("parallel", n=n, pixel=pix, n_views=36, n_bins=121, bin=1.0)
        else:
            geo = Geometry("fan", n=n, pixel=pix, n_views=36, n_bins=121, bin=1.6, sod=300.0, sdd=520.0)
        p0, d = geo.rays()
        ref = _gaussian_line_integral(p0, d, cx, cy, sigma)
        y = orc.project(orc.Geom(geo), _gaussian_image(n, pix, cx, cy, sigma))
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.mark.parametrize("beam", ["parallel", "fan"])
def test_ellipse_chords_converge(orc, beam):
    """Projections of a pixel-sampled ellipse phantom approach the exact chord
    lengths (synth.line_integrals), with an error that shrinks under refinement."""
    ell = [synth.Ellipse(0.0, 0.0, 40.0, 40.0, 0.0, 0.02),
           synth.Ellipse(14.0, -9.0, 15.0, 7.0, 0.6, 0.01),
           synth.Ellipse(-20.0, 18.0, 6.0, 11.0, 2.1, -0.008)]
    errs = []
    for n, pix in [(64, 1.5), (128, 0.75), (256, 0.375)]:
        if beam == "parallel":
            geo = Geometry("parallel", n=n, pixel=pix, n_views=30, n_bins=101, bin=1.0)
        else:
            geo = Geometry("fan", n=n, pixel=pix, n_views=30, n_bins=101, bin=1.5, sod=300.0, sdd=520.0)
        ref = synth.line_integrals(ell, geo)
        y = orc.project(orc.Geom(geo), synth.rasterize(ell, n, pix))
        errs.append(np.abs(y - ref).sum() / np.abs(ref).sum())
    assert errs[-1] < 5e-3
    assert errs[0] > 1.6 * errs[1] > 2.56 * errs[2], errs


# ----------------------------------------------------------------------------- tables

def test_tables_match_intercept_range_by_brute_force(orc):
    """The index tables list exactly the driving indices whose sampled rows
    can be non-zero: checked against single-pixel projections."""
    geo = Geometry("fan", n=12, pixel=1.0, n_views=7, n_bins=19, bin=1.0, sod=30.0, sdd=50.0)
    g = orc.Geom(geo)
    axis, lo, hi = orc.tables(g)
    n = geo.n
    hit = np.zeros((geo.n_views, geo.n_bins, n), bool)   # [ray, driving index]
    for j in range(n):
        for i in range(n):
            e = np.zeros((n, n)); e[j, i] = 1.0
            y = orc.project(g, e)
            for v in range(geo.n_views):
                for k in range(geo.n_bins):
                    if y[v, k] != 0.0:
                        hit[v, k, i if axis[v, k] == 0 else j] = True
    for v in range(geo.n_views):
        for k in range(geo.n_bins):
            idx = np.flatnonzero(hit[v, k])
            if idx.size:
                assert lo[v, k] <= idx.min() and idx.max() <= hi[v, k]
                assert hi[v, k] - lo[v, k] - (idx.max() - idx.min()) <= 2
            else:
                assert hi[v, k] - lo[v, k] <= 1


def test_table_axis_rule(orc):
    """x-driven iff |d_x| >= |d_y| (ties go to x)."""
    c = math.sqrt(0.5)
    g = orc.Geom(geom_custom("parallel", 8, 1.0, ([1.0, 0.0, c], [0.0, 1.0, c]), 5, 1.0))
    axis, lo, hi = orc.tables(g)
    assert (axis[0] == 1).all()      # theta = 0: d = (0, 1), y-driven
    assert (axis[1] == 0).all()      # theta = pi/2: d = (-1, 0), x-driven
    assert (axis[2] == 0).all()      # 45 degrees: tie -> x-driven


# ----------------------------------------------------------------------------- A^T

@pytest.mark.parametrize("name", ["c1", "c2_small"])
def test_adjoint_dot_product(orc, name):
    """<A x, y> = <x, A^T y> to 1e-12 (compensated sums)."""
    if name == "c1":
        geo = synth.workload("c1").geom
    else:
        geo = Geometry("fan", n=96, pixel=2.0, n_views=90, n_bins=140, bin=2.4, sod=400.0, sdd=700.0)
    g = orc.Geom(geo)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((geo.n, geo.n))
    y = rng.standard_normal((geo.n_views, geo.n_bins))
    lhs = math.fsum((orc.project(g, x) * y).ravel())
    rhs = math.fsum((x * orc.backproject(g, y)).ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dense_adjoint_is_transpose(orc):
    """Dense A from unit images equals the transpose of dense A^T from unit rays."""
    geo = Geometry("fan", n=16, pixel=1.0, n_views=12, n_bins=23, bin=1.0, sod=40.0, sdd=70.0)
    g = orc.Geom(geo)
    n, nr = geo.n, geo.n_rays
    A = np.stack([orc.project(g, e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)
    At = np.stack([orc.backproject(g, e.reshape(geo.n_views, geo.n_bins)).ravel() for e in np.eye(nr)], axis=1)
    assert np.array_equal(A.T, At)
    assert (A >= 0).all() and A.any()


# ----------------------------------------------------------------------------- C

def test_ramp_taps_have_ramp_frequency_response(orc):
    """The Ram-Lak taps are the Fourier coefficients of |w| / (2 pi) on [-pi, pi]."""
    m = 20001
    r = orc.ramp_taps(m)
    w = np.linspace(0.0, math.pi, 64)
    k = np.arange(1, m)
    resp = r[0] + 2.0 * (r[1:][None, :] * np.cos(np.outer(w, k))).sum(axis=1)
    np.testing.assert_allclose(resp, w / (2 * math.pi), atol=2e-5)


def test_ramp_is_linear_convolution(orc):
    """C y equals kappa times a library FFT linear convolution with the taps,
    kappa = pi / (n_views * pixel^2)."""
    geo = synth.workload("c1").geom
    g = orc.Geom(geo)
    y = np.random.default_rng(4).standard_normal((geo.n_views, geo.n_bins))
    r = orc.ramp_taps(geo.n_bins)
    full = np.concatenate([r[:0:-1], r])                 # taps for offsets -(D-1)..(D-1)
    conv = scipy.signal.fftconvolve(y, full[None, :], mode="full", axes=1)
    ref = conv[:, geo.n_bins - 1: 2 * geo.n_bins - 1]
    kappa = math.pi / (geo.n_views * geo.pixel ** 2)
    np.testing.assert_allclose(orc.ramp(g, y), kappa * ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("nb", [47, 185])
def test_ramp_matrix_symmetric_positive_definite(orc, nb):
    """C = P^T P with P = C^(1/2) requires C symmetric and positive (semi)definite (Eqs. (2)-(3))."""
    g = orc.Geom(geom_custom("parallel", 4, 1.0, np.array([0.0]), nb, 1.0))
    R = np.stack([orc.ramp(g, e[None, :])[0] for e in np.eye(nb)], axis=1)
    assert np.array_equal(R, R.T)
    ev = np.linalg.eigvalsh(R)
    assert ev.min() > 0.0


def test_fbp_normalisation_on_a_disk(orc):
    """A^T C of the exact parallel-beam sinogram of a 0.02/mm disk reconstructs
    0.02/mm inside the disk (filtered backprojection, within 0.5%)."""
    geo = Geometry("parallel", n=128, pixel=1.0, n_views=360, n_bins=185, bin=1.0)
    disk = [synth.Ellipse(0.0, 0.0, 50.0, 50.0, 0.0, 0.02)]
    x = orc.filtered_backproject(orc.Geom(geo), synth.line_integrals(disk, geo), 1)
    c = np.arange(128) - 63.5
    r = np.hypot(c[None, :], c[:, None])
    inner = x[r < 40]
    assert abs(inner.mean() - 0.02) < 1e-4
    assert inner.std() < 2e-4


@pytest.mark.parametrize("kind,resp", [
    ("shepp-logan", lambda w: np.abs(np.sin(w / 2.0)) / math.pi),
    ("hann", lambda w: w / (2 * math.pi) * 0.5 * (1.0 + np.cos(w))),
    ("ram-lak", lambda w: w / (2 * math.pi)),
])
def test_ramp_windows_have_their_frequency_responses(orc, kind, resp):
    """The apodised windows' taps are the Fourier coefficients of their closed-form
    responses: Shepp-Logan |sin(w/2)| / pi, Hann |w| / (2 pi) (1 + cos w) / 2."""
    m = 20001
    r = orc.ramp_taps_kind(orc.RAMP_WINDOWS[kind], m)
    w = np.linspace(0.0, math.pi, 64)
    k = np.arange(1, m)
    got = r[0] + 2.0 * (r[1:][None, :] * np.cos(np.outer(w, k))).sum(axis=1)
    np.testing.assert_allclose(got, resp(w), atol=3e-5)


@pytest.mark.parametrize("kind", ["shepp-logan", "hann"])
@pytest.mark.parametrize("nb", [47, 185])
def test_apodised_ramp_matrices_are_positive_definite(orc, kind, nb):
    """Truncations of a non-negative response give symmetric positive definite C (Eq. (2))."""
    g = orc.Geom(geom_custom("parallel", 4, 1.0, np.array([0.0]), nb, 1.0), ramp=orc.RAMP_WINDOWS[kind])
    R = np.stack([orc.ramp(g, e[None, :])[0] for e in np.eye(nb)], axis=1)
    assert np.array_equal(R, R.T)
    assert np.linalg.eigvalsh(R).min() > 0.0


def test_cosine_weighted_ramp_is_symmetric_congruence(orc):
    """Symmetric cosine weighting gives C_w = D^(1/2) C D^(1/2) with
    D = diag(sdd / sqrt(sdd^2 + u_k^2)): checked column by column against the
    unweighted C, so a one-sided or squared weight fails."""
    geo = geom_custom("fan", 8, 1.0, np.array([0.3]), 41, 2.5, sod=60.0, sdd=100.0)
    g0, gw = orc.Geom(geo, ramp=2), orc.Geom(geo, ramp=2 | orc.RAMP_COSINE)
    C = np.stack([orc.ramp(g0, e[None, :])[0] for e in np.eye(41)], axis=1)
    Cw = np.stack([orc.ramp(gw, e[None, :])[0] for e in np.eye(41)], axis=1)
    u = (np.arange(41) - 20) * 2.5
    d = np.sqrt(100.0 / np.sqrt(100.0 ** 2 + u ** 2))
    np.testing.assert_allclose(Cw, d[:, None] * C * d[None, :], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(orc.ramp_weights(gw), d ** 2, rtol=1e-15)
    assert np.all(orc.ramp_weights(orc.Geom(geo)) == 1.0)
    assert np.linalg.eigvalsh(Cw).min() > 0.0


@pytest.mark.parametrize("ramp", [0, 1, 2, 16, 18])
def test_fan_beam_fbp_scale_of_a_disk(orc, ramp):
    """A^T C of an exact fan-beam disk sinogram reconstructs the disk's 0.02/mm
    interior to within 3% for every window, with or without the weighting (all
    windows share the ramp's low-frequency response, which sets the scale)."""
    geo = Geometry("fan", n=128, pixel=1.0, n_views=360, n_bins=256, bin=1.0, sod=200.0, sdd=350.0)
    disk = [synth.Ellipse(0.0, 0.0, 50.0, 50.0, 0.0, 0.02)]
    x = orc.filtered_backproject(orc.Geom(geo, ramp=ramp), synth.line_integrals(disk, geo), 1)
    c = np.arange(128) - 63.5
    inner = x[np.hypot(c[None, :], c[:, None]) < 40]
    assert abs(inner.mean() / 0.02 - 1.0) < 0.03
    assert inner.std() < 0.03 * 0.02

# ----------------------------------------------------------------------------- W

def test_framelet_perfect_reconstruction(orc):
    """W^T W = I (unitary extension principle of the piecewise-linear filters)."""
    x = np.random.default_rng(5).standard_normal((24, 24))
    z = orc.framelet(x)
    np.testing.assert_allclose(orc.framelet_adjoint(z), x, atol=1e-14)
    # W is an isometry, and W^T really is its adjoint
    assert abs(np.vdot(z, z) - np.vdot(x, x)) < 1e-12 * np.vdot(x, x)
    zz = np.random.default_rng(6).standard_normal((9, 24, 24))
    assert abs(np.vdot(orc.framelet(x), zz) - np.vdot(x, orc.framelet_adjoint(zz))) < 1e-12


def test_framelet_bands_on_polynomials(orc):
    """Orientation and normalisation of the bands (band = 3 m_y + m_x, correlation form):
    constants live in band 0 only; a ramp in x gives -sqrt2/2 in band 1 and nothing in
    band 2 or 3; x^2 gives -1/2 in band 2; a ramp in y gives -sqrt2/2 in band 3."""
    n = 16
    jj, ii = np.mgrid[0:n, 0:n].astype(float)
    z = orc.framelet(np.full((n, n), 3.0))
    np.testing.assert_allclose(z[0], 3.0, atol=1e-14)
    np.testing.assert_allclose(z[1:], 0.0, atol=1e-14)
    inner = (slice(2, n - 2), slice(2, n - 2))
    z = orc.framelet(ii)
    np.testing.assert_allclose(z[1][inner], -math.sqrt(2) / 2, atol=1e-13)
    np.testing.assert_allclose(z[2][inner], 0.0, atol=1e-13)
    np.testing.assert_allclose(z[3][inner], 0.0, atol=1e-13)
    np.testing.assert_allclose(z[0][inner], ii[inner], atol=1e-13)
    z = orc.framelet(ii ** 2)
    np.testing.assert_allclose(z[2][inner], -0.5, atol=1e-12)
    z = orc.framelet(jj)
    np.testing.assert_allclose(z[3][inner], -math.sqrt(2) / 2, atol=1e-13)
    np.testing.assert_allclose(z[1][inner], 0.0, atol=1e-13)


def test_shrink_values(orc):
    n = 2
    v = np.zeros((9, n, n))
    v[0] = [[5.0, -5.0], [0.1, -0.1]]
    v[4] = [[0.3, -0.3], [0.1, -0.25]]
    d = orc.shrink(v, 0.25)
    np.testing.assert_array_equal(d[0], v[0])                       # LL passes through
    np.testing.assert_allclose(d[4], [[0.05, -0.05], [0.0, 0.0]], atol=1e-16)


# ----------------------------------------------------------------------------- CG / Eq. (5) / split Bregman

def _small_problem(orc, n=24, views=40, bins=35, seed=7):
    geo = Geometry("parallel", n=n, pixel=1.0, n_views=views, n_bins=bins, bin=1.0)
    g = orc.Geom(geo)
    ell = [synth.Ellipse(0, 0, 9, 9, 0, 0.02), synth.Ellipse(3, -2, 4, 2.5, 0.4, 0.01)]
    y = synth.line_integrals(ell, geo)
    y = y + 0.01 * np.random.default_rng(seed).standard_normal(y.shape)
    return geo, g, y


def _dense(orc, g, n, mu, filt=1):
    return np.stack([orc.apply_normal(g, e.reshape(n, n), mu, filt).ravel() for e in np.eye(n * n)], axis=1)


def test_cg_converges_to_dense_cholesky(orc):
    """CG on Eq. (5), run to convergence, equals a dense Cholesky solve of
    (A^T C A + lambda I) X = A^T C Y."""
    geo, g, y = _small_problem(orc)
    lam = 0.005
    M = _dense(orc, g, geo.n, lam)
    rhs = orc.filtered_backproject(g, y, 1).ravel()
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(M), rhs)
    x, _ = orc.solve(g, y, lam, 1.0, 0, 400, reg=1)
    assert np.linalg.norm(x.ravel() - ref) < 1e-10 * np.linalg.norm(ref)
    assert np.abs(M - M.T).max() < 1e-13 * np.abs(M).max()


def test_eq5_cg_matches_dense_cholesky_32x32(orc):
    """The stated pin size: 32 x 32 image, parallel beam, 48 views over [0, pi),
    47 bins of 1 mm, lambda = 0.005.  CG run until its residual norm squared
    falls below 1e-26 equals the Cholesky solve of the dense
    (A^T C A + lambda I) X = A^T C Y to 1e-10."""
    geo, g, y = _small_problem(orc, n=32, views=48, bins=47, seed=17)
    lam = 0.005
    M = _dense(orc, g, geo.n, lam)
    rhs = orc.filtered_backproject(g, y, 1).ravel()
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(M), rhs)
    n_cg = 0
    x = np.zeros(geo.n * geo.n)
    while True:
        n_cg += 200
        x, _ = orc.solve(g, y, lam, 1.0, 0, n_cg, reg=1)
        r = rhs - M @ x.ravel()
        if float(r @ r) < 1e-26 or n_cg >= 4000:
            break
    assert float(r @ r) < 1e-26, (n_cg, float(r @ r))
    assert np.linalg.norm(x.ravel() - ref) < 1e-10 * np.linalg.norm(ref)


def test_cg_iterates_minimise_over_krylov_space(orc):
    """After n CG steps from x0, x_n minimises the M-norm error over x0 + K_n(M, r0)."""
    geo, g, y = _small_problem(orc, n=16, views=24, bins=25)
    mu = 0.3
    M = _dense(orc, g, geo.n, mu)
    rhs = orc.filtered_backproject(g, y, 1).ravel()
    x0 = np.random.default_rng(8).standard_normal(rhs.size) * 0.01
    r0 = rhs - M @ x0
    for n_it in (1, 3, 5):
        K = np.stack([np.linalg.matrix_power(M, i) @ r0 for i in range(n_it)], axis=1)
        Q, _ = np.linalg.qr(K)
        c = np.linalg.solve(Q.T @ M @ Q, Q.T @ r0)
        ref = x0 + Q @ c
        x = orc.cg(g, rhs.reshape(geo.n, geo.n), mu, n_it, x0.reshape(geo.n, geo.n))
        assert np.linalg.norm(x.ravel() - ref) < 1e-9 * np.linalg.norm(ref)


def test_split_bregman_reaches_optimality_conditions(orc):
    """At convergence split Bregman's X minimises ||P(AX-Y)||^2 + lambda ||W_d X||_1
    (Eq. (1) with the framelet regulariser, P^T P = C): with xi = (2 mu / lambda) b,
    A^T C (A X - Y) + (lambda / 2) W^T xi = 0, |xi| <= 1, xi = sign(W X) where
    W X != 0, and xi = 0 on the unpenalised low-pass band."""
    geo, g, y = _small_problem(orc)
    lam, mu = 0.005, 1.0
    x, res, b = orc.solve(g, y, lam, mu, 600, 40, return_b=True)
    assert res[-1] < 1e-3 * res[0]
    xi = b * (2.0 * mu / lam)
    grad = orc.filtered_backproject(g, orc.project(g, x) - y, 1)
    # stationarity; away from the limit its residual is mu W^T (d_k - d_{k+1})
    stat = grad + 0.5 * lam * orc.framelet_adjoint(xi)
    assert np.linalg.norm(stat) < 1e-4 * np.linalg.norm(grad)
    assert np.abs(xi).max() <= 1.0 + 1e-12
    assert not xi[0].any()
    z = orc.framelet(x)[1:]
    on = np.abs(z) > 1e-3
    assert on.sum() > 100 and (~on).sum() > 100      # a genuinely sparse solution
    np.testing.assert_allclose(xi[1:][on], np.sign(z[on]), atol=1e-12)


def test_split_bregman_objective_is_locally_minimal(orc):
    """Brute force: random perturbations of the converged X never lower the objective."""
    geo, g, y = _small_problem(orc)
    lam, mu = 0.005, 1.0
    x, _ = orc.solve(g, y, lam, mu, 600, 40)

    def objective(xx):
        r = orc.project(g, xx) - y
        return float(np.vdot(r, orc.ramp(g, r))) + lam * np.abs(orc.framelet(xx)[1:]).sum()

    f0 = objective(x)
    rng = np.random.default_rng(9)
    for _ in range(20):
        dx = rng.standard_normal(x.shape) * 1e-4
        assert objective(x + dx) >= f0 - 1e-12 * abs(f0)


def test_l2_mode_matches_eq5_dense_solve(orc):
    """reg = 1 solves Eq. (5), (A'^T A + lambda I) X = A'^T Y, here checked with lambda = 0.1."""
    geo, g, y = _small_problem(orc, n=16, views=24, bins=25)
    lam = 0.1
    M = _dense(orc, g, geo.n, lam)
    ref = np.linalg.solve(M, orc.filtered_backproject(g, y, 1).ravel())
    x, _ = orc.solve(g, y, lam, 1.0, 0, 300, reg=1)
    assert np.linalg.norm(x.ravel() - ref) < 1e-10 * np.linalg.norm(ref)


def test_ir_mode_uses_plain_adjoint(orc):
    """filter = 0 gives the plain IR arm: A^T instead of A'^T = A^T C."""
    geo, g, y = _small_problem(orc, n=16, views=24, bins=25)
    np.testing.assert_array_equal(orc.filtered_backproject(g, y, 0), orc.backproject(g, y))
    M0 = _dense(orc, g, geo.n, 0.0, 0)
    A = np.stack([orc.project(g, e.reshape(16, 16)).ravel() for e in np.eye(256)], axis=1)
    np.testing.assert_allclose(M0, A.T @ A, atol=1e-10 * np.abs(M0).max())


# ----------------------------------------------------------------------------- forward-backward splitting, Eq. (6)

def _dense_ops(orc, g, geo):
    """Dense A [rays x pixels] and C [rays x rays] from the oracle's pinned operators."""
    n, nr = geo.n, geo.n_views * geo.n_bins
    A = np.stack([orc.project(g, e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)
    C = np.stack([orc.ramp(g, e.reshape(geo.n_views, geo.n_bins)).ravel() for e in np.eye(nr)], axis=1)
    return A, C


@pytest.mark.parametrize("filt", [1, 0])
def test_fbs_without_prior_is_landweber(orc, filt):
    """lambda = 0: the proximal step is the identity (W^T W = I), so Eq. (6) is
    the Landweber iteration X <- X - mu A'^T (A X - Y), here with dense matrices."""
    geo, g, y = _small_problem(orc, n=12, views=16, bins=19)
    A, C = _dense_ops(orc, g, geo)
    At = A.T @ C if filt else A.T
    mu = 0.5 if filt else 0.5 / np.linalg.norm(A.T @ A, 2)
    x = np.zeros(geo.n * geo.n)
    for _ in range(6):
        x = x - mu * (At @ (A @ x - y.ravel()))
    xo, res = orc.solve(g, y, 0.0, mu, 6, 0, reg=2, filter=filt)
    assert np.linalg.norm(xo.ravel() - x) < 1e-12 * np.linalg.norm(x)
    assert res.shape == (6,) and res[0] > 0.0


def test_fbs_prox_with_large_lambda_is_the_low_pass_band(orc):
    """With Y = A X0 the forward step leaves X0 unchanged; a threshold above
    every detail coefficient keeps only band 0, and W^T of band 0 is
    (h0^T h0) in x and y: the periodic blur [1, 4, 6, 4, 1] / 16 per axis."""
    geo, g, _ = _small_problem(orc, n=12, views=16, bins=19)
    x0 = np.random.default_rng(3).uniform(size=(12, 12))
    y = orc.project(g, x0)
    xo, _ = orc.solve(g, y, 1e6, 1.0, 1, 0, reg=2, x0=x0)
    k = np.array([1, 4, 6, 4, 1]) / 16.0
    blur = sum(k[a + 2] * np.roll(x0, a, axis=1) for a in range(-2, 3))
    blur = sum(k[a + 2] * np.roll(blur, a, axis=0) for a in range(-2, 3))
    assert np.abs(xo - blur).max() < 1e-12


def test_fbs_converges_to_a_fixed_point(orc):
    """With a step inside the stability bound the forward-backward map is a
    contraction on this problem: the step norms ||X_{k+1} - X_k|| fall and the
    last iterate is (to 1e-9) a fixed point of one more forward-backward step."""
    geo, g, y = _small_problem(orc, n=16, views=24, bins=25)
    x, res = orc.solve(g, y, 0.01, 1.0, 400, 0, reg=2)
    assert res[-1] < 1e-9 * res[0]
    assert np.all(np.diff(res[5:]) <= 1e-15)
    x2, _ = orc.solve(g, y, 0.01, 1.0, 1, 0, reg=2, x0=x)
    assert np.linalg.norm(x2 - x) < 1e-9 * np.linalg.norm(x)


def test_fbs_prox_threshold_is_half_step_times_lambda(orc):
    """One step from a consistent start (Y = A X0): X1 = W^T shrink(W X0, mu lambda / 2)
    on the detail bands, with W built here from its filters by periodic shifts."""
    geo, g, _ = _small_problem(orc, n=12, views=16, bins=19)
    x0 = np.random.default_rng(5).uniform(size=(12, 12))
    y = orc.project(g, x0)
    lam, mu = 0.08, 0.7
    s2 = math.sqrt(2.0)
    h = [np.array([1, 2, 1]) / 4.0, s2 * np.array([1, 0, -1]) / 4.0, np.array([-1, 2, -1]) / 4.0]

    def corr(x, f, axis):            # (H x)[n] = sum_k f[k + 1] x[n + k], periodic
        return sum(f[k + 1] * np.roll(x, -k, axis=axis) for k in (-1, 0, 1))

    def corr_t(x, f, axis):          # adjoint of corr
        return sum(f[k + 1] * np.roll(x, k, axis=axis) for k in (-1, 0, 1))

    t = mu * lam / 2.0
    x1 = np.zeros_like(x0)
    for my in range(3):
        for mx in range(3):
            z = corr(corr(x0, h[my], 0), h[mx], 1)
            if my or mx:
                z = np.sign(z) * np.maximum(np.abs(z) - t, 0.0)
            x1 += corr_t(corr_t(z, h[mx], 1), h[my], 0)
    xo, res = orc.solve(g, y, lam, mu, 1, 0, reg=2, x0=x0)
    assert np.abs(xo - x1).max() < 1e-12
    assert res[0] == pytest.approx(np.linalg.norm(x1 - x0), rel=1e-12)
