/*
 * FP64 CPU oracle for the AIR reconstruction path.  TEST INFRASTRUCTURE ONLY:
 * see oracle.h for what may use it.  Plain loops, float64 throughout, OpenMP
 * only across independent outputs.  Shares no code with the GPU library.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared oracle.c -lm
 * (-ffp-contract=off: the ray intercepts below are evaluated exactly as
 * written, operation by operation, with no fused multiply-add).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int geom_ok(const orc_geom* g) {
    if (!g || g->n <= 0 || g->n_views <= 0 || g->n_bins <= 0) return 0;
    if (!(g->pixel > 0.0) || !(g->bin > 0.0) || !g->cosv || !g->sinv) return 0;
    if (g->beam == 1 && !(g->sdd > g->sod && g->sod > 0.0)) return 0;
    if ((g->ramp & ~31) != 0 || (g->ramp & 15) > 2) return 0;
    return g->beam == 0 || g->beam == 1;
}

/* One ray of the scan (scan geometry: a point on the ray and its direction).
 *   bin centre  u_k = (k - (n_bins-1)/2) * bin
 *   parallel:   p0 = u_k (cos, sin),  d = (-sin, cos)
 *   fan (flat): p0 = sod (cos, sin),  d = (-sdd cos - u_k sin, -sdd sin + u_k cos)
 * The ray is x-driven (steps over columns) iff |d_x| >= |d_y|. */
typedef struct {
    int axis;       /* 0: driving index is the column i; 1: the row j */
    double pa, pb;  /* p0 along the driving / interpolated coordinate */
    double da, db;  /* d along the driving / interpolated coordinate */
} orc_ray;

static orc_ray make_ray(const orc_geom* g, int v, int k) {
    const double c = g->cosv[v], s = g->sinv[v];
    const double u = ((double)k - 0.5 * (double)(g->n_bins - 1)) * g->bin;
    double px, py, dx, dy;
    if (g->beam == 0) {
        px = u * c;
        py = u * s;
        dx = -s;
        dy = c;
    } else {
        px = g->sod * c;
        py = g->sod * s;
        dx = -(g->sdd * c) - u * s;
        dy = -(g->sdd * s) + u * c;
    }
    orc_ray r;
    if (fabs(dx) >= fabs(dy)) {
        r.axis = 0; r.pa = px; r.pb = py; r.da = dx; r.db = dy;
    } else {
        r.axis = 1; r.pa = py; r.pb = px; r.da = dy; r.db = dx;
    }
    return r;
}

/* Joseph intercept: where the ray crosses the centre line of driving index a,
 * in pixel units of the interpolated coordinate measured from pixel centre 0. */
static double intercept(const orc_geom* g, const orc_ray* r, int a) {
    const double h = 0.5 * (double)(g->n - 1);
    const double slope = r->db / r->da;
    const double ca = ((double)a - h) * g->pixel;
    return ((r->pb + (ca - r->pa) * slope) + h * g->pixel) / g->pixel;
}

/* Path length per driving-axis step: pixel * |d| / |d_drive|. */
static double step_length(const orc_geom* g, const orc_ray* r) {
    return g->pixel * sqrt(r->da * r->da + r->db * r->db) / fabs(r->da);
}

/* image value at (driving index a, interpolated index b); 0 outside */
static double img_at(const double* x, int n, int axis, int a, int b) {
    if (b < 0 || b >= n) return 0.0;
    return axis == 0 ? x[(size_t)b * n + a] : x[(size_t)a * n + b];
}

int orc_tables(const orc_geom* g, int8_t* axis, int32_t* lo, int32_t* hi) {
    if (!geom_ok(g) || !axis || !lo || !hi) return -1;
    const int n = g->n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < g->n_views; v++) {
        for (int k = 0; k < g->n_bins; k++) {
            const orc_ray r = make_ray(g, v, k);
            int first = -1, last = -1;
            for (int a = 0; a < n; a++) {
                const double t = intercept(g, &r, a);
                if (t > -1.0 && t < (double)n) {
                    if (first < 0) first = a;
                    last = a;
                }
            }
            const size_t idx = (size_t)v * g->n_bins + k;
            axis[idx] = (int8_t)r.axis;
            lo[idx] = first < 0 ? 0 : first;
            hi[idx] = first < 0 ? -1 : last;
        }
    }
    return 0;
}

/* y_ray = step_length * sum_a [(1-f) X(a, floor t_a) + f X(a, floor t_a + 1)],
 * f = t_a - floor t_a; samples outside the image are zero. */
int orc_project(const orc_geom* g, const double* x, double* y) {
    if (!geom_ok(g) || !x || !y) return -1;
    const int n = g->n, nb = g->n_bins;
    const long nr = (long)g->n_views * nb;
#pragma omp parallel for schedule(dynamic, 64)
    for (long ridx = 0; ridx < nr; ridx++) {
        const int v = (int)(ridx / nb), k = (int)(ridx % nb);
        const orc_ray r = make_ray(g, v, k);
        double acc = 0.0;
        for (int a = 0; a < n; a++) {
            const double t = intercept(g, &r, a);
            if (!(t > -1.0 && t < (double)n)) continue;
            const double fl = floor(t);
            const int b0 = (int)fl;
            const double f = t - fl;
            acc += (1.0 - f) * img_at(x, n, r.axis, a, b0) + f * img_at(x, n, r.axis, a, b0 + 1);
        }
        y[ridx] = acc * step_length(g, &r);
    }
    return 0;
}

/* Exact transpose of orc_project, in scatter form: each ray adds its value,
 * times the same weights, to the pixels it sampled.  Views are split into a
 * fixed number of groups with one image buffer each, summed in group order,
 * so the result does not depend on the thread count. */
#define ORC_GROUPS 16
int orc_backproject(const orc_geom* g, const double* y, double* x) {
    if (!geom_ok(g) || !y || !x) return -1;
    const int n = g->n, nb = g->n_bins, nv = g->n_views;
    const size_t npix = (size_t)n * n;
    double* buf = (double*)calloc((size_t)ORC_GROUPS * npix, sizeof(double));
    if (!buf) return -3;
#pragma omp parallel for schedule(static, 1)
    for (int grp = 0; grp < ORC_GROUPS; grp++) {
        double* img = buf + (size_t)grp * npix;
        for (int v = grp; v < nv; v += ORC_GROUPS) {
            for (int k = 0; k < nb; k++) {
                const orc_ray r = make_ray(g, v, k);
                const double val = y[(size_t)v * nb + k] * step_length(g, &r);
                if (val == 0.0) continue;
                for (int a = 0; a < n; a++) {
                    const double t = intercept(g, &r, a);
                    if (!(t > -1.0 && t < (double)n)) continue;
                    const double fl = floor(t);
                    const int b0 = (int)fl;
                    const double f = t - fl;
                    if (b0 >= 0) {
                        const size_t p = r.axis == 0 ? (size_t)b0 * n + a : (size_t)a * n + b0;
                        img[p] += (1.0 - f) * val;
                    }
                    if (b0 + 1 <= n - 1) {
                        const size_t p = r.axis == 0 ? (size_t)(b0 + 1) * n + a : (size_t)a * n + b0 + 1;
                        img[p] += f * val;
                    }
                }
            }
        }
    }
    for (size_t p = 0; p < npix; p++) {
        double s = 0.0;
        for (int grp = 0; grp < ORC_GROUPS; grp++) s += buf[(size_t)grp * npix + p];
        x[p] = s;
    }
    free(buf);
    return 0;
}

/* Ram-Lak spatial taps (dimensionless): r(0) = 1/4, r(m) = -1/(pi^2 m^2) for
 * odd m, 0 for even m != 0. */
void orc_ramp_taps(int32_t n_bins, double* r) {
    for (int m = 0; m < n_bins; m++) {
        if (m == 0) r[m] = 0.25;
        else if (m % 2) r[m] = -1.0 / (ORC_PI * ORC_PI * (double)m * (double)m);
        else r[m] = 0.0;
    }
}

/* Apodised ramp windows (Methods: C is any symmetric positive semi-definite
 * filtration, Eq. (2)), in the same dimensionless units as the Ram-Lak taps:
 *   kind 0  Ram-Lak      frequency response |w| / (2 pi)
 *   kind 1  Shepp-Logan  r(m) = -2 / (pi^2 (4 m^2 - 1)),  response |sin(w / 2)| / pi
 *   kind 2  Hann         r(m) = r_RL(m) / 2 + (r_RL(m - 1) + r_RL(m + 1)) / 4,
 *                        response |w| / (2 pi) * (1 + cos w) / 2 */
int orc_ramp_taps_kind(int32_t kind, int32_t n_bins, double* r) {
    if (n_bins < 1 || !r) return -1;
    if (kind == 0) {
        orc_ramp_taps(n_bins, r);
        return 0;
    }
    if (kind == 1) {
        for (int m = 0; m < n_bins; m++) r[m] = -2.0 / (ORC_PI * ORC_PI * (4.0 * (double)m * (double)m - 1.0));
        return 0;
    }
    if (kind == 2) {
        double* rl = (double*)malloc(((size_t)n_bins + 1) * sizeof(double));
        if (!rl) return -3;
        orc_ramp_taps(n_bins + 1, rl);
        for (int m = 0; m < n_bins; m++) {
            const double left = rl[m == 0 ? 1 : m - 1];     /* r_RL is even: r(-1) = r(1) */
            r[m] = 0.5 * rl[m] + 0.25 * (left + rl[m + 1]);
        }
        free(rl);
        return 0;
    }
    return -1;
}

/* Fan-beam cosine weights of a flat detector, w_k = sdd / sqrt(sdd^2 + u_k^2)
 * (the cosine of the ray's angle to the central ray); 1 for parallel beams or
 * when the weighting bit is off. */
int orc_ramp_weights(const orc_geom* g, double* w) {
    if (!geom_ok(g) || !w) return -1;
    const int on = (g->ramp & 16) && g->beam == 1;
    for (int k = 0; k < g->n_bins; k++) {
        const double u = ((double)k - 0.5 * (g->n_bins - 1)) * g->bin;
        w[k] = on ? g->sdd / sqrt(g->sdd * g->sdd + u * u) : 1.0;
    }
    return 0;
}

/* C = kappa D^(1/2) R D^(1/2) per view: D the cosine weights (identity unless
 * requested), R the symmetric Toeplitz matrix of the window's taps, applied as
 * a linear (non-circular) convolution truncated to the detector,
 * kappa = pi / (n_views * pixel^2).  C stays symmetric positive semi-definite. */
int orc_ramp(const orc_geom* g, const double* y, double* yf) {
    if (!geom_ok(g) || !y || !yf) return -1;
    const int nb = g->n_bins, nv = g->n_views;
    double* r = (double*)malloc((size_t)nb * sizeof(double));
    double* w = (double*)malloc((size_t)nb * sizeof(double));
    if (!r || !w) { free(r); free(w); return -3; }
    int rc = orc_ramp_taps_kind(g->ramp & 15, nb, r);
    if (rc == 0) rc = orc_ramp_weights(g, w);
    if (rc) { free(r); free(w); return rc; }
    const double kappa = ORC_PI / ((double)nv * g->pixel * g->pixel);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; v++) {
        const double* row = y + (size_t)v * nb;
        for (int m = 0; m < nb; m++) {
            double s = 0.0;
            for (int k = 0; k < nb; k++) s += r[abs(m - k)] * sqrt(w[k]) * row[k];
            yf[(size_t)v * nb + m] = kappa * sqrt(w[m]) * s;
        }
    }
    free(r);
    free(w);
    return 0;
}

int orc_filtered_backproject(const orc_geom* g, const double* y, double* x, int32_t filter) {
    if (!geom_ok(g)) return -1;
    if (!filter) return orc_backproject(g, y, x);
    const size_t ns = (size_t)g->n_views * g->n_bins;
    double* yf = (double*)malloc(ns * sizeof(double));
    if (!yf) return -3;
    int rc = orc_ramp(g, y, yf);
    if (rc == 0) rc = orc_backproject(g, yf, x);
    free(yf);
    return rc;
}

/* Piecewise-linear framelet filters h_0 = [1,2,1]/4, h_1 = sqrt(2)[1,0,-1]/4,
 * h_2 = [-1,2,-1]/4, indexed by offset -1, 0, +1. */
static double fl_tap(int m, int off) {
    static const double s2 = 1.41421356237309504880;
    switch (m) {
    case 0: return off == 0 ? 0.5 : 0.25;
    case 1: return off == 0 ? 0.0 : (off < 0 ? s2 / 4.0 : -s2 / 4.0);
    default: return off == 0 ? 0.5 : -0.25;
    }
}

/* z[3 m_y + m_x][j][i] = sum_{dy,dx} h_{m_y}(dy) h_{m_x}(dx) x[(j+dy) mod n][(i+dx) mod n] */
int orc_framelet(int32_t n, const double* x, double* z) {
    if (n <= 0 || !x || !z) return -1;
    const size_t npix = (size_t)n * n;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; j++) {
        for (int i = 0; i < n; i++) {
            for (int my = 0; my < 3; my++) {
                for (int mx = 0; mx < 3; mx++) {
                    double s = 0.0;
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++)
                            s += fl_tap(my, dy) * fl_tap(mx, dx) *
                                 x[(size_t)((j + dy + n) % n) * n + (i + dx + n) % n];
                    z[(size_t)(3 * my + mx) * npix + (size_t)j * n + i] = s;
                }
            }
        }
    }
    return 0;
}

/* x[j][i] = sum_band sum_{dy,dx} h_{m_y}(dy) h_{m_x}(dx) z[band][(j-dy) mod n][(i-dx) mod n] */
int orc_framelet_adjoint(int32_t n, const double* z, double* x) {
    if (n <= 0 || !x || !z) return -1;
    const size_t npix = (size_t)n * n;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; j++) {
        for (int i = 0; i < n; i++) {
            double s = 0.0;
            for (int my = 0; my < 3; my++)
                for (int mx = 0; mx < 3; mx++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++)
                            s += fl_tap(my, dy) * fl_tap(mx, dx) *
                                 z[(size_t)(3 * my + mx) * npix +
                                   (size_t)((j - dy + n) % n) * n + (i - dx + n) % n];
            x[(size_t)j * n + i] = s;
        }
    }
    return 0;
}

/* d = sign(v) max(|v| - t, 0) on the detail bands 1..8; band 0 passes through. */
void orc_shrink(int32_t n, const double* v, double t, double* d) {
    const size_t npix = (size_t)n * n;
    for (size_t p = 0; p < npix; p++) d[p] = v[p];
    for (size_t p = npix; p < 9 * npix; p++) {
        const double a = fabs(v[p]) - t;
        d[p] = a > 0.0 ? (v[p] > 0.0 ? a : -a) : 0.0;
    }
}

/* out = A^T C A x + mu x   (C omitted when filter == 0) */
int orc_apply_normal(const orc_geom* g, const double* x, double mu, int32_t filter, double* out) {
    if (!geom_ok(g) || !x || !out) return -1;
    const size_t ns = (size_t)g->n_views * g->n_bins, npix = (size_t)g->n * g->n;
    double* y = (double*)malloc(ns * sizeof(double));
    if (!y) return -3;
    int rc = orc_project(g, x, y);
    if (rc == 0) rc = orc_filtered_backproject(g, y, out, filter);
    free(y);
    if (rc) return rc;
    for (size_t p = 0; p < npix; p++) out[p] += mu * x[p];
    return 0;
}

static double dot(const double* a, const double* b, size_t n) {
    double s = 0.0;
    for (size_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* n_iter conjugate-gradient steps on (A^T C A + mu I) x = rhs, starting from x. */
int orc_cg(const orc_geom* g, const double* rhs, double mu, int32_t filter, int32_t n_iter, double* x) {
    if (!geom_ok(g) || !rhs || !x || n_iter < 0) return -1;
    const size_t np = (size_t)g->n * g->n;
    double* r = (double*)malloc(np * sizeof(double));
    double* p = (double*)malloc(np * sizeof(double));
    double* q = (double*)malloc(np * sizeof(double));
    int rc = (r && p && q) ? 0 : -3;
    if (rc == 0) rc = orc_apply_normal(g, x, mu, filter, q);
    if (rc == 0) {
        for (size_t i = 0; i < np; i++) { r[i] = rhs[i] - q[i]; p[i] = r[i]; }
        double rho = dot(r, r, np);
        for (int it = 0; it < n_iter && rc == 0; it++) {
            if (rho == 0.0) break;
            rc = orc_apply_normal(g, p, mu, filter, q);
            if (rc) break;
            const double alpha = rho / dot(p, q, np);
            for (size_t i = 0; i < np; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            const double rho_new = dot(r, r, np);
            const double beta = rho_new / rho;
            for (size_t i = 0; i < np; i++) p[i] = r[i] + beta * p[i];
            rho = rho_new;
        }
    }
    free(r); free(p); free(q);
    return rc;
}

/* Forward-backward splitting (Eq. (6)) for min ||P(AX - Y)||^2 + lambda ||W X||_1:
 *   repeat n_outer times:
 *     X' = X - mu A^T C (A X - Y)                (forward step, Eq. (6); A^T alone when filter == 0)
 *     X  = W^T shrink(W X', mu lambda / 2)       (proximal step; band 0 passes through)
 *     resid[k] = ||X_new - X_old||_2
 * The data term's gradient is 2 A^T C (A X - Y), so the step of Eq. (6) is mu / 2
 * and the matching threshold mu lambda / 2.  For the tight frame (W^T W = I)
 * W^T shrink W stands in for the exact proximal map of lambda ||W X||_1. */
static int orc_fbs(const orc_geom* g, const double* y, const orc_params* prm, double* x, double* resid) {
    const int n = g->n;
    const size_t np = (size_t)n * n, nz = 9 * np, ns = (size_t)g->n_views * g->n_bins;
    double* ax = (double*)malloc(ns * sizeof(double));
    double* grad = (double*)malloc(np * sizeof(double));
    double* z = (double*)malloc(nz * sizeof(double));
    double* d = (double*)malloc(nz * sizeof(double));
    double* xn = (double*)malloc(np * sizeof(double));
    int rc = (ax && grad && z && d && xn) ? 0 : -3;
    const double thr = prm->mu * prm->lambda / 2.0;
    for (int k = 0; k < prm->n_outer && rc == 0; k++) {
        rc = orc_project(g, x, ax);                                    /* A X */
        if (rc) break;
        for (size_t i = 0; i < ns; i++) ax[i] -= y[i];                  /* A X - Y */
        rc = orc_filtered_backproject(g, ax, grad, prm->filter);      /* A'^T (A X - Y) */
        if (rc) break;
        for (size_t p = 0; p < np; p++) xn[p] = x[p] - prm->mu * grad[p];
        rc = orc_framelet(n, xn, z);
        if (rc) break;
        orc_shrink(n, z, thr, d);
        rc = orc_framelet_adjoint(n, d, xn);
        if (rc) break;
        double ss = 0.0;
        for (size_t p = 0; p < np; p++) {
            ss += (xn[p] - x[p]) * (xn[p] - x[p]);
            x[p] = xn[p];
        }
        if (resid) resid[k] = sqrt(ss);
    }
    free(ax); free(grad); free(z); free(d); free(xn);
    return rc;
}

/* Split Bregman for min ||P(AX - Y)||^2 + lambda ||W X||_1 (detail bands):
 *   g = A^T C Y;  d = b = 0
 *   repeat n_outer times:
 *     X <- CG_n(A^T C A + mu I, g + mu W^T (d - b), start X)     (L2 step, cf. Eq. (5))
 *     v = W X + b;  d = shrink(v, lambda / (2 mu));  b = v - d
 *     resid[k] = ||W X - d||_2
 * reg = 1: the L2-regularised case, Eq. (5): n_cg CG steps on
 * (A^T C A + lambda I) X = A^T C Y from the given X.
 * reg = 2: forward-backward splitting (orc_fbs), mu the step of Eq. (6).
 * X holds the start value on entry (zeros for the standard start); b_out, if
 * not NULL, receives the final Bregman variable b [9][n][n]. */
int orc_solve(const orc_geom* g, const double* y, const orc_params* prm, double* x, double* resid,
              double* b_out) {
    if (!geom_ok(g) || !y || !prm || !x) return -1;
    if (prm->n_outer < 0 || prm->n_cg < 0 || !(prm->mu > 0.0) || prm->lambda < 0.0) return -1;
    if (prm->reg == 2) return orc_fbs(g, y, prm, x, resid);
    const int n = g->n;
    const size_t np = (size_t)n * n, nz = 9 * np;
    double* gb = (double*)malloc(np * sizeof(double));
    if (!gb) return -3;
    int rc = orc_filtered_backproject(g, y, gb, prm->filter);
    if (rc) { free(gb); return rc; }
    if (prm->reg == 1) {
        rc = orc_cg(g, gb, prm->lambda, prm->filter, prm->n_cg, x);
        free(gb);
        return rc;
    }
    double* d = (double*)calloc(nz, sizeof(double));
    double* b = (double*)calloc(nz, sizeof(double));
    double* v = (double*)malloc(nz * sizeof(double));
    double* e = (double*)malloc(nz * sizeof(double));
    double* rhs = (double*)malloc(np * sizeof(double));
    if (!d || !b || !v || !e || !rhs) rc = -3;
    const double thr = prm->lambda / (2.0 * prm->mu);
    for (int k = 0; k < prm->n_outer && rc == 0; k++) {
        for (size_t p = 0; p < nz; p++) e[p] = d[p] - b[p];
        rc = orc_framelet_adjoint(n, e, rhs);
        if (rc) break;
        for (size_t p = 0; p < np; p++) rhs[p] = gb[p] + prm->mu * rhs[p];
        rc = orc_cg(g, rhs, prm->mu, prm->filter, prm->n_cg, x);
        if (rc) break;
        rc = orc_framelet(n, x, v);              /* v = W X */
        if (rc) break;
        for (size_t p = 0; p < nz; p++) v[p] += b[p];
        orc_shrink(n, v, thr, d);
        double ss = 0.0;
        for (size_t p = 0; p < nz; p++) {
            const double wx = v[p] - b[p];       /* W X */
            ss += (wx - d[p]) * (wx - d[p]);
            b[p] = v[p] - d[p];
        }
        if (resid) resid[k] = sqrt(ss);
    }
    if (rc == 0 && b_out) memcpy(b_out, b, nz * sizeof(double));
    free(gb); free(d); free(b); free(v); free(e); free(rhs);
    return rc;
}
