// Per-ray Joseph tables, built on the host in float64.
//
// Compiled with -ffp-contract=off: each intercept below is evaluated
// operation by operation as written, which is what makes the index ranges
// reproducible bit for bit by any other implementation of the same
// definition (an independent FP64 scan over all driving indices gives the
// same lo/hi).
//
// Definitions (scan model of the Joseph projector):
//   u_k = ((double)k - 0.5 (n_bins - 1)) * bin
//   parallel: p0 = (u_k c, u_k s), d = (-s, c)
//   fan:      p0 = (sod c, sod s), d = (-(sdd c) - u_k s, -(sdd s) + u_k c)
//   x-driven iff |d_x| >= |d_y|; (pa, pb, da, db) = p0 and d along (driving, other) axis
//   t(a) = ((pb + (((double)a - h) * pixel - pa) * (db / da)) + h * pixel) / pixel,  h = 0.5 (n - 1)
//   [lo, hi] = the driving indices with -1 < t(a) < n.
// t(a) is weakly monotone in a (each step is a monotone rounded operation), so
// the index set is an interval; it is found from the closed-form crossing
// points and then fixed up with the exact predicate.
#include "geometry.h"

#include <cmath>
#include <cstdlib>
#include <cstdio>

namespace air {

namespace {

struct Ray64 {
    int axis;
    double pa, pb, da, db;
};

Ray64 make_ray(const GeomHost& g, int v, int k) {
    const double c = g.cosv[v], s = g.sinv[v];
    const double u = ((double)k - 0.5 * (double)(g.n_bins - 1)) * g.bin;
    double px, py, dx, dy;
    if (g.beam == 0) {
        px = u * c;
        py = u * s;
        dx = -s;
        dy = c;
    } else {
        px = g.sod * c;
        py = g.sod * s;
        dx = -(g.sdd * c) - u * s;
        dy = -(g.sdd * s) + u * c;
    }
    Ray64 r;
    if (std::fabs(dx) >= std::fabs(dy)) {
        r.axis = 0; r.pa = px; r.pb = py; r.da = dx; r.db = dy;
    } else {
        r.axis = 1; r.pa = py; r.pb = px; r.da = dy; r.db = dx;
    }
    return r;
}

inline double t_at(const GeomHost& g, const Ray64& r, double slope, int a) {
    const double h = 0.5 * (double)(g.n - 1);
    const double ca = ((double)a - h) * g.pixel;
    return ((r.pb + (ca - r.pa) * slope) + h * g.pixel) / g.pixel;
}

}  // namespace

void ramp_taps64(int n_bins, int window, std::vector<double>& r) {
    const double pi = 3.14159265358979323846;
    auto ram_lak = [pi](int m) {
        m = std::abs(m);
        return m == 0 ? 0.25 : ((m & 1) ? -1.0 / (pi * pi * (double)m * (double)m) : 0.0);
    };
    r.assign(n_bins, 0.0);
    for (int m = 0; m < n_bins; m++) {
        if (window == 1) r[m] = -2.0 / (pi * pi * (4.0 * (double)m * (double)m - 1.0));   // Shepp-Logan
        else if (window == 2) r[m] = 0.5 * ram_lak(m) + 0.25 * (ram_lak(m - 1) + ram_lak(m + 1));   // Hann
        else r[m] = ram_lak(m);
    }
}

std::string build_ray_tables(const GeomHost& g, std::vector<RayEntry>& rays, std::vector<float>& step,
                             std::vector<int8_t>& axis, std::vector<int32_t>& lo, std::vector<int32_t>& hi) {
    const int n = g.n;
    const size_t nr = (size_t)g.n_views * g.n_bins;
    rays.resize(nr);
    step.resize(nr);
    axis.resize(nr);
    lo.resize(nr);
    hi.resize(nr);
    const int c0 = n / 2;
    const double dn = (double)n;
    for (int v = 0; v < g.n_views; v++) {
        for (int k = 0; k < g.n_bins; k++) {
            const Ray64 r = make_ray(g, v, k);
            const double slope = r.db / r.da;
            auto inside = [&](int a) {
                const double t = t_at(g, r, slope, a);
                return t > -1.0 && t < dn;
            };
            int a_lo = 0, a_hi = -1;
            const double t0 = t_at(g, r, slope, 0);
            const double t1 = t_at(g, r, slope, n - 1);
            const bool empty = (t0 <= -1.0 && t1 <= -1.0) || (t0 >= dn && t1 >= dn) ||
                               std::isnan(t0) || std::isnan(t1);
            if (!empty) {
                // crossing points of the exact line t0 + a * slope (a guess within an index or two)
                double lb = 0.0, ub = (double)(n - 1);
                if (slope > 0.0) {
                    lb = (-1.0 - t0) / slope;
                    ub = (dn - t0) / slope;
                } else if (slope < 0.0) {
                    lb = (dn - t0) / slope;
                    ub = (-1.0 - t0) / slope;
                }
                auto clampi = [&](double x) -> int {
                    if (!(x > 0.0)) return 0;
                    if (x > (double)(n - 1)) return n - 1;
                    return (int)x;
                };
                a_lo = clampi(std::floor(lb));
                a_hi = clampi(std::ceil(ub));
                // fix up against the exact predicate (the set is an interval)
                while (a_lo > 0 && inside(a_lo - 1)) a_lo--;
                while (a_lo < n - 1 && !inside(a_lo)) a_lo++;
                while (a_hi < n - 1 && inside(a_hi + 1)) a_hi++;
                while (a_hi > 0 && !inside(a_hi)) a_hi--;
                if (!inside(a_lo) || !inside(a_hi) || a_lo > a_hi) {
                    // the guesses bracketed nothing: scan (never expected; kept for safety)
                    a_lo = 0; a_hi = -1;
                    for (int a = 0; a < n; a++) {
                        if (inside(a)) {
                            if (a_hi < 0) a_lo = a;
                            a_hi = a;
                        }
                    }
                }
            }
            const size_t idx = (size_t)v * g.n_bins + k;
            axis[idx] = (int8_t)r.axis;
            lo[idx] = a_lo;
            hi[idx] = a_hi;
            RayEntry e;
            e.tc = std::llround((t_at(g, r, slope, c0) + (double)kPad) * std::ldexp(1.0, kFrac));
            const double ms = std::nearbyint(slope * std::ldexp(1.0, kSlopeFrac));   // |slope| <= 1
            e.m = (int32_t)(ms > 2147483647.0 ? 2147483647.0 : (ms < -2147483647.0 ? -2147483647.0 : ms));
            step[idx] = (float)(g.pixel * std::sqrt(r.da * r.da + r.db * r.db) / std::fabs(r.da));
            e.meta = (int32_t)((uint32_t)a_lo | ((uint32_t)(a_hi + 1) << 15) | ((uint32_t)r.axis << 30));
            if (a_hi < a_lo) e.meta = (int32_t)((uint32_t)r.axis << 30);
            // The kernels sample padded lines at T >> kFrac and the next sample;
            // both must stay inside the line (indices 0 .. n + 2 kPad - 1).
            if (a_hi >= a_lo) {
                const int64_t ta = e.tc + (int64_t)(a_lo - c0) * e.m * 2;
                const int64_t tb = e.tc + (int64_t)(a_hi - c0) * e.m * 2;
                const int64_t tmin = ta < tb ? ta : tb, tmax = ta < tb ? tb : ta;
                if (tmin < 0 || (tmax >> kFrac) > (int64_t)(n + 2 * kPad - 2)) {
                    char buf[160];
                    snprintf(buf, sizeof buf, "ray (%d, %d): intercept out of the padded range", v, k);
                    return buf;
                }
            }
            rays[idx] = e;
        }
    }
    return std::string();
}

}  // namespace air
