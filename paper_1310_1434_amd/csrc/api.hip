// C ABI of the AIR library: plans, operator entry points and the split
// Bregman solver.  Host code; all arithmetic runs in the kernels.
#include <algorithm>
#include <new>

#include "plan.h"

namespace air {

thread_local std::string g_err;

air_status fail(air_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

}  // namespace air

namespace {

// float -> IEEE half, round to nearest even (host side, for the 16-bit filter tables)
uint16_t f32_to_f16(float f) {
    uint32_t x;
    std::memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t e8 = (x >> 23) & 0xffu;
    uint32_t mant = x & 0x7fffffu;
    if (e8 == 0xffu) return (uint16_t)(sign | 0x7c00u | (mant ? 0x200u : 0u));
    const int exp = (int)e8 - 127 + 15;
    if (exp >= 31) return (uint16_t)(sign | 0x7c00u);
    if (exp <= 0) {
        if (exp < -10) return (uint16_t)sign;
        mant |= 0x800000u;
        const int shift = 14 - exp;
        uint32_t hm = mant >> shift;
        const uint32_t rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
        if (rem > half || (rem == half && (hm & 1u))) hm++;
        return (uint16_t)(sign | hm);
    }
    uint32_t h = sign | ((uint32_t)exp << 10) | (mant >> 13);
    const uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h++;
    return (uint16_t)h;
}

float f16_to_f32(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    const int e = (h >> 10) & 0x1f;
    const uint32_t m = h & 0x3ffu;
    float v;
    if (e == 0) v = std::ldexp((float)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = std::ldexp((float)(m | 0x400u), e - 25);
    uint32_t x;
    std::memcpy(&x, &v, 4);
    x |= sign;
    std::memcpy(&v, &x, 4);
    return v;
}

uint16_t f32_to_bf16(float f) {
    uint32_t x;
    std::memcpy(&x, &f, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
    x += 0x7fffu + ((x >> 16) & 1u);
    return (uint16_t)(x >> 16);
}

float bf16_to_f32(uint16_t h) {
    const uint32_t x = (uint32_t)h << 16;
    float v;
    std::memcpy(&v, &x, 4);
    return v;
}


}  // namespace

extern "C" {

const char* air_last_error(void) { return g_err.c_str(); }

air_status air_plan_create(const air_geometry* geom, int32_t max_batch, air_precision prec, uint32_t flags,
                           air_plan* out) {
    if (!out) return fail(AIR_E_INVALID, "out is null");
    *out = nullptr;
    if (!geom) return fail(AIR_E_INVALID, "geometry is null");
    if ((flags & ~(uint32_t)(AIR_RAMP_WINDOW_MASK | AIR_RAMP_COSINE_WEIGHTED)) != 0 ||
        (flags & AIR_RAMP_WINDOW_MASK) > AIR_RAMP_HANN)
        return fail(AIR_E_INVALID, "unknown plan flags");
    if (geom->beam != AIR_PARALLEL && geom->beam != AIR_FAN_FLAT) return fail(AIR_E_INVALID, "unknown beam");
    if (geom->n < 1 || geom->n_views < 1 || geom->n_bins < 1) return fail(AIR_E_INVALID, "sizes must be >= 1");
    if (geom->n > kMaxN) return fail(AIR_E_UNSUPPORTED, "n exceeds 16384");
    if (geom->n_bins > kMaxBins) return fail(AIR_E_UNSUPPORTED, "n_bins exceeds 8192");
    if ((int64_t)geom->n_views * geom->n_bins > (int64_t)1 << 30) return fail(AIR_E_UNSUPPORTED, "too many rays");
    if (!(geom->pixel_mm > 0.0) || !std::isfinite(geom->pixel_mm)) return fail(AIR_E_INVALID, "pixel_mm must be > 0");
    if (!(geom->bin_mm > 0.0) || !std::isfinite(geom->bin_mm)) return fail(AIR_E_INVALID, "bin_mm must be > 0");
    if (!geom->view_cos || !geom->view_sin) return fail(AIR_E_INVALID, "view tables are null");
    if (max_batch < 1) return fail(AIR_E_INVALID, "max_batch must be >= 1");
    if (prec != AIR_FP32 && prec != AIR_MIXED_F16 && prec != AIR_MIXED_BF16)
        return fail(AIR_E_INVALID, "unknown precision");
    if (geom->beam == AIR_FAN_FLAT) {
        if (!(geom->sod_mm > 0.0) || !(geom->sdd_mm > geom->sod_mm) || !std::isfinite(geom->sdd_mm))
            return fail(AIR_E_INVALID, "fan beam needs 0 < sod_mm < sdd_mm");
        // every pixel (grown by one pixel) must lie strictly in front of the source
        const double reach = (0.5 * geom->n + 1.5) * geom->pixel_mm * 1.41421356237309515;
        if (!(geom->sod_mm > reach)) return fail(AIR_E_UNSUPPORTED, "image reaches the source circle");
    }
    for (int v = 0; v < geom->n_views; v++) {
        const double c = geom->view_cos[v], s = geom->view_sin[v];
        if (!std::isfinite(c) || !std::isfinite(s) || std::fabs(c * c + s * s - 1.0) > 1e-6)
            return fail(AIR_E_INVALID, "view (cos, sin) must be finite unit vectors");
    }
    air_plan_s* p = new (std::nothrow) air_plan_s;
    if (!p) return fail(AIR_E_NOMEM, "host allocation failed");
    try {
        GeomHost& g = p->g;
        g.beam = geom->beam;
        g.n = geom->n;
        g.n_views = geom->n_views;
        g.n_bins = geom->n_bins;
        g.pixel = geom->pixel_mm;
        g.bin = geom->bin_mm;
        g.sod = geom->beam == AIR_FAN_FLAT ? geom->sod_mm : 0.0;
        g.sdd = geom->beam == AIR_FAN_FLAT ? geom->sdd_mm : 0.0;
        g.cosv.assign(geom->view_cos, geom->view_cos + g.n_views);
        g.sinv.assign(geom->view_sin, geom->view_sin + g.n_views);
        p->max_batch = max_batch;
        p->prec = prec;
        p->ds = (g.n_bins + 31) / 32 * 32;
        p->line = g.n + 2 * kPad;
        p->c0 = g.n / 2;
        p->kappa = 3.14159265358979323846 / ((double)g.n_views * g.pixel * g.pixel);
        std::vector<float> step;
        const std::string err = build_ray_tables(g, p->rays, step, p->axis, p->lo, p->hi);
        if (!err.empty()) {
            delete p;
            return fail(AIR_E_UNSUPPORTED, err);
        }
        p->step.assign((size_t)g.n_views * p->ds, 0.f);
        for (int v = 0; v < g.n_views; v++)
            for (int k = 0; k < g.n_bins; k++) p->step[(size_t)v * p->ds + k] = step[(size_t)v * g.n_bins + k];
        {
            // forward-projector block order: views whose rays are mostly x-driven
            // (they read only the column copies) first, then the mostly y-driven ones
            std::vector<int32_t> vx, vy;
            for (int v = 0; v < g.n_views; v++) {
                int ny = 0;
                for (int k = 0; k < g.n_bins; k++) ny += p->axis[(size_t)v * g.n_bins + k];
                (2 * ny > g.n_bins ? vy : vx).push_back(v);
            }
            p->v_half = (int)((std::max(vx.size(), vy.size()) + 3) / 4 * 4);
            p->vorder.assign(2 * (size_t)p->v_half, -1);
            std::copy(vx.begin(), vx.end(), p->vorder.begin());
            std::copy(vy.begin(), vy.end(), p->vorder.begin() + p->v_half);
        }
        p->views.resize(2 * (size_t)g.n_views);
        for (int v = 0; v < g.n_views; v++) {
            p->views[2 * v] = (float)g.cosv[v];
            p->views[2 * v + 1] = (float)g.sinv[v];
        }
        p->ramp_window = (int)(flags & AIR_RAMP_WINDOW_MASK);
        p->cos_weight = (flags & AIR_RAMP_COSINE_WEIGHTED) != 0;
        std::vector<double> r;
        ramp_taps64(g.n_bins, p->ramp_window, r);
        const int ds = p->ds;
        if (p->cos_weight) {
            // D^(1/2), D = diag(sdd / sqrt(sdd^2 + u_k^2)) for a flat fan-beam detector, identity for parallel beams
            p->wsq.assign(ds, 0.f);
            for (int k = 0; k < g.n_bins; k++) {
                const double u = ((double)k - 0.5 * (double)(g.n_bins - 1)) * g.bin;
                const double w = g.beam == AIR_FAN_FLAT ? g.sdd / std::sqrt(g.sdd * g.sdd + u * u) : 1.0;
                p->wsq[k] = (float)std::sqrt(w);
            }
        }
        p->taps32.assign(2 * (size_t)ds, 0.f);
        for (int idx = 0; idx < 2 * ds; idx++) {
            const int d = std::abs(idx - ds);
            if (d < g.n_bins) p->taps32[idx] = (float)(p->kappa * r[d]);
        }
        if (prec != AIR_FP32) {
            p->n_terms = prec == AIR_MIXED_F16 ? 2 : 3;
            const int tj = ramp_tab_j(ds);
            p->tab16.assign((size_t)p->n_terms * 4 * tj * 4, 0);
            for (int sh = 0; sh < 4; sh++)
                for (int j = 0; j < tj; j++)
                    for (int i = 0; i < 4; i++) {
                        const int d = std::abs(4 * j + sh + i - kRampZero - ds);
                        const float T = d < g.n_bins ? (float)(r[d] * 4096.0) : 0.f;
                        uint16_t term[3];
                        if (prec == AIR_MIXED_F16) {
                            term[0] = f32_to_f16(T);
                            term[1] = f32_to_f16((T - f16_to_f32(term[0])) * 2048.f);
                        } else {
                            term[0] = f32_to_bf16(T);
                            const float r1 = T - bf16_to_f32(term[0]);
                            term[1] = f32_to_bf16(r1);
                            term[2] = f32_to_bf16(r1 - bf16_to_f32(term[1]));
                        }
                        for (int u = 0; u < p->n_terms; u++)
                            p->tab16[(((size_t)u * 4 + sh) * tj + j) * 4 + i] = term[u];
                    }
        }
        // workspace layout
        Carver c;
        const size_t nr = (size_t)g.n_views * g.n_bins;
        p->off_rays = c.take(nr * sizeof(RayEntry));
        p->off_step = c.take(p->step.size() * sizeof(float));
        p->off_views = c.take(p->views.size() * sizeof(float));
        p->off_taps = c.take(p->taps32.size() * sizeof(float));
        p->off_vorder = c.take(p->vorder.size() * sizeof(int32_t));
        p->off_bpwin = c.take(bp_window_count(g.n, g.n_views) * sizeof(BpWin));
        p->off_bpwinx = c.take(bp_window_count(g.n, g.n_views) * sizeof(float2));
        if (!p->tab16.empty()) p->off_tab16 = c.take(p->tab16.size() * sizeof(uint16_t));
        if (p->cos_weight) p->off_wsq = c.take(p->wsq.size() * sizeof(float));
        const size_t mb = (size_t)max_batch;
        const size_t gi = (size_t)group_images(max_batch);
        p->off_pad = c.take(gi * 2 * g.n * p->line * sizeof(float));   // grouped padded copies
        p->off_s1 = c.take(mb * g.n_views * ds * sizeof(float));
        p->off_s2 = c.take(gi * g.n_views * ds * sizeof(float));       // group-interleaved backprojector input
        p->off_pscale = c.take((mb + 63) / 64 * 64 * sizeof(float));
        p->off_ppart = c.take(mb * (size_t)tiles16(g.n) * sizeof(double));
        p->off_rscale = c.take(mb * g.n_views * sizeof(float));
        p->total = c.off;
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(AIR_E_NOMEM, "host allocation failed");
    }
    *out = p;
    return AIR_OK;
}

air_status air_plan_workspace_size(air_plan p, size_t* bytes) {
    if (air_status st = check_plan(p, false)) return st;
    if (!bytes) return fail(AIR_E_INVALID, "bytes is null");
    *bytes = p->total;
    return AIR_OK;
}

air_status air_plan_bind_workspace(air_plan p, void* dev, size_t bytes, hipStream_t s) {
    if (air_status st = check_plan(p, false)) return st;
    if (!dev) return fail(AIR_E_INVALID, "workspace is null");
    if (reinterpret_cast<uintptr_t>(dev) & 255u) return fail(AIR_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < p->total) return fail(AIR_E_NOMEM, "workspace smaller than air_plan_workspace_size");
    char* ws = static_cast<char*>(dev);
    AIR_HIP(hipMemcpyAsync(ws + p->off_rays, p->rays.data(), p->rays.size() * sizeof(RayEntry),
                           hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(ws + p->off_step, p->step.data(), p->step.size() * sizeof(float),
                           hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(ws + p->off_views, p->views.data(), p->views.size() * sizeof(float),
                           hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(ws + p->off_taps, p->taps32.data(), p->taps32.size() * sizeof(float),
                           hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(ws + p->off_vorder, p->vorder.data(), p->vorder.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    if (!p->tab16.empty())
        AIR_HIP(hipMemcpyAsync(ws + p->off_tab16, p->tab16.data(), p->tab16.size() * sizeof(uint16_t),
                               hipMemcpyHostToDevice, s));
    if (p->cos_weight)
        AIR_HIP(hipMemcpyAsync(ws + p->off_wsq, p->wsq.data(), p->wsq.size() * sizeof(float), hipMemcpyHostToDevice, s));
    {
        // the backprojector's window table, from the tables just copied
        const KGeom kg = p->kgeom_at(ws);
        AIR_HIP(launch_bp_windows(kg, reinterpret_cast<BpWin*>(ws + p->off_bpwin),
                                  reinterpret_cast<float2*>(ws + p->off_bpwinx), s));
    }
    AIR_HIP(hipStreamSynchronize(s));
    p->ws = ws;
    return AIR_OK;
}

air_status air_plan_tables(air_plan p, int8_t* axis, int32_t* lo, int32_t* hi) {
    if (air_status st = check_plan(p, false)) return st;
    const size_t nr = p->axis.size();
    if (axis) std::memcpy(axis, p->axis.data(), nr);
    if (lo) std::memcpy(lo, p->lo.data(), nr * sizeof(int32_t));
    if (hi) std::memcpy(hi, p->hi.data(), nr * sizeof(int32_t));
    return AIR_OK;
}

void air_plan_destroy(air_plan p) { delete p; }

air_status air_project(air_plan p, const float* x, float* y, int32_t batch, hipStream_t s) {
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_batch(p, batch, true)) return st;
    if (!x || !y) return fail(AIR_E_INVALID, "null pointer");
    const KGeom kg = p->kgeom();
    const PadBuf pad = plan_pad(p, p->at<float>(p->off_pad), p->at<float>(p->off_pscale));
    if (air_status e = build_pad(p, x, pad, p->at<double>(p->off_ppart), batch, s)) return e;
    if (p->direct(y)) {
        AIR_K(AIR_K_PROJECT, launch_project(kg, pad, y, batch, s));
    } else {
        float* s1 = p->at<float>(p->off_s1);
        AIR_K(AIR_K_PROJECT, launch_project(kg, pad, s1, batch, s));
        AIR_K(AIR_K_OTHER, launch_repack(s1, p->ds, y, p->g.n_bins, batch * p->g.n_views, p->g.n_bins, p->g.n_bins, s));
    }
    return AIR_OK;
}

air_status air_ramp(air_plan p, const float* y, float* yf, int32_t batch, hipStream_t s) {
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_batch(p, batch, true)) return st;
    if (!y || !yf) return fail(AIR_E_INVALID, "null pointer");
    if (y == yf) return fail(AIR_E_INVALID, "air_ramp is not in-place");
    const float* src = nullptr;
    if (air_status st = stage_sino(p, y, batch, p->at<float>(p->off_s1), &src, s)) return st;
    const int rows = batch * p->g.n_views;
    if (p->direct(yf)) {
        AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(p->at<float>(p->off_rscale)), src, yf, rows, p->ds, 0, 0, s));
    } else {
        float* s2 = p->at<float>(p->off_s2);
        AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(p->at<float>(p->off_rscale)), src, s2, rows, p->ds, 0, 0, s));
        AIR_K(AIR_K_OTHER, launch_repack(s2, p->ds, yf, p->g.n_bins, rows, p->g.n_bins, p->g.n_bins, s));
    }
    return AIR_OK;
}

air_status air_filtered_backproject(air_plan p, const float* y, float* x, int32_t batch, int32_t filter,
                                    hipStream_t s) {
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_batch(p, batch, true)) return st;
    if (!y || !x) return fail(AIR_E_INVALID, "null pointer");
    if (filter != 0 && filter != 1) return fail(AIR_E_INVALID, "filter must be 0 or 1");
    // A^T C y = J^T (S C y); A^T y = J^T (S y)
    const float* src = nullptr;
    if (air_status st = stage_sino(p, y, batch, p->at<float>(p->off_s1), &src, s)) return st;
    float* s2 = p->at<float>(p->off_s2);
    const int grp = image_group(batch);
    if (filter) AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(p->at<float>(p->off_rscale)), src, s2, batch * p->g.n_views, p->ds,
                                              RAMP_POST, grp, s));
    else AIR_K(AIR_K_OTHER, launch_scale(p->kgeom(), src, s2, batch, grp, s));
    BpArgs a{};
    a.mode = BP_PLAIN;
    a.out = x;
    AIR_K(AIR_K_BACKPROJECT, launch_backproject(p->kgeom(), s2, a, batch, s));
    return AIR_OK;
}

air_status air_normal_apply(air_plan p, const float* x, float* out, int32_t batch, double mu, int32_t filter,
                            hipStream_t s) {
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_batch(p, batch, true)) return st;
    if (!x || !out) return fail(AIR_E_INVALID, "null pointer");
    if (x == out) return fail(AIR_E_INVALID, "air_normal_apply is not in-place");
    if (filter != 0 && filter != 1) return fail(AIR_E_INVALID, "filter must be 0 or 1");
    if (!std::isfinite(mu)) return fail(AIR_E_INVALID, "mu must be finite");
    const KGeom kg = p->kgeom();
    const PadBuf pad = plan_pad(p, p->at<float>(p->off_pad), p->at<float>(p->off_pscale));
    float* s1 = p->at<float>(p->off_s1);
    float* s2 = p->at<float>(p->off_s2);
    // A^T C A x = J^T (S C S) J x;  A^T A x = J^T S^2 J x  (the projector applies the first S)
    if (air_status e = build_pad(p, x, pad, p->at<double>(p->off_ppart), batch, s)) return e;
    AIR_K(AIR_K_PROJECT, launch_project(kg, pad, s1, batch, s));
    const int grp = image_group(batch);
    if (filter) AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(p->at<float>(p->off_rscale)), s1, s2, batch * p->g.n_views, p->ds,
                                              RAMP_POST, grp, s));
    else AIR_K(AIR_K_OTHER, launch_scale(kg, s1, s2, batch, grp, s));
    const float* src = s2;
    BpArgs a{};
    a.mode = BP_MATVEC;
    a.mu = (float)mu;
    a.aux = x;
    a.out = out;
    AIR_K(AIR_K_BACKPROJECT, launch_backproject(kg, src, a, batch, s));
    return AIR_OK;
}

air_status air_kernel_timing_enable(air_plan p, int32_t enable) {
    if (air_status st = check_plan(p, false)) return st;
    if (enable != AIR_TIMING_OFF && enable != AIR_TIMING_ON && enable != AIR_TIMING_ONE_STREAM)
        return fail(AIR_E_INVALID, "timing mode must be 0, 1 or 2");
    p->timing = enable;
    return AIR_OK;
}

air_status air_kernel_timing_collect(air_plan p, air_kernel_stats* stats) {
    if (air_status st = check_plan(p, false)) return st;
    if (!stats) return fail(AIR_E_INVALID, "stats is null");
    air_status result = AIR_OK;
    for (const air_plan_s::Timed& t : p->pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && result == AIR_OK) result = fail(AIR_E_HIP, std::string("event timing: ") + hipGetErrorString(e));
        stats->ms[t.kind] += ms;
        stats->launches[t.kind] += 1;
        p->pool.push_back(t.a);
        p->pool.push_back(t.b);
    }
    p->pending.clear();
    return result;
}

air_status air_framelet(air_plan p, const float* in, float* out, int32_t batch, int32_t adjoint, hipStream_t s) {
    if (air_status st = check_plan(p, false)) return st;
    if (air_status st = check_batch(p, batch, false)) return st;
    if (!in || !out) return fail(AIR_E_INVALID, "null pointer");
    if (in == out) return fail(AIR_E_INVALID, "air_framelet is not in-place");
    if (adjoint != 0 && adjoint != 1) return fail(AIR_E_INVALID, "adjoint must be 0 or 1");
    if (adjoint) AIR_K(AIR_K_FRAMELET, launch_framelet_adj(p->g.n, in, out, batch, s));
    else AIR_K(AIR_K_FRAMELET, launch_framelet_fwd(p->g.n, in, out, batch, s));
    return AIR_OK;
}

}  // extern "C"

extern "C" {

// A solve of at least kSplitMin images runs as two sub-batches, each on its own
// stream: one sub-batch's projections (bound by the gather issue rate) then
// overlap the other's backprojections (bound by VALU and LDS).  Measured at
// C2: 16 images as 2 x 8 run at 1.10x the throughput of one 16-image batch,
// 32 as 2 x 16 at 1.19x two 16-image batches in turn; every image gets the
// same bits either way.  Kernel timing in AIR_TIMING_ONE_STREAM mode keeps
// one stream, so the per-kernel times are those of kernels running alone.
constexpr int kSplitMin = 8;
static int solve_parts(const air_plan_s* p, int batch) {
    return batch >= kSplitMin && p->timing != AIR_TIMING_ONE_STREAM ? 2 : 1;
}
static int part_size(int batch, int parts, int i) { return parts == 1 ? batch : (i == 0 ? (batch + 1) / 2 : batch / 2); }
static size_t part_offset(const air_plan_s* p, int batch, int parts, int i) {
    return i == 0 ? 0 : (solve_layout(p, part_size(batch, parts, 0)).total + 255) / 256 * 256;
}
static size_t solve_bytes(const air_plan_s* p, int batch) {
    size_t one = solve_layout(p, batch).total;
    if (batch < kSplitMin) return one;
    const size_t two = part_offset(p, batch, 2, 1) + solve_layout(p, part_size(batch, 2, 1)).total;
    return std::max(one, two);    // (one-stream kernel timing runs one part)
}

air_status air_solve_workspace_size(air_plan p, int32_t batch, size_t* bytes) {
    if (air_status st = check_plan(p, false)) return st;
    if (air_status st = check_batch(p, batch, false)) return st;
    if (!bytes) return fail(AIR_E_INVALID, "bytes is null");
    *bytes = solve_bytes(p, batch);
    return AIR_OK;
}

// The two sub-batch streams of the current device (default priority), created
// once per device and kept until the process ends.  All plans share them: each
// stream is bound to a hardware queue when it is created, and two streams
// that end up on one queue run one after the other (measured: per-plan stream
// pairs, created after other streams, lost the overlap).
static hipError_t device_sub_streams(hipStream_t (&out)[2]) {
    static std::mutex mu;
    static hipStream_t streams[64][2] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < 2; i++)
        if (!streams[dev][i] && (e = hipStreamCreateWithFlags(&streams[dev][i], hipStreamNonBlocking)) != hipSuccess)
            return e;
    out[0] = streams[dev][0];
    out[1] = streams[dev][1];
    return hipSuccess;
}

static SolveSetup solve_setup(const air_solve_params* prm) {
    return SolveSetup{prm->reg, prm->filter, prm->lambda, prm->mu, prm->n_cg};
}
static int solve_outer_count(const air_solve_params* prm) { return prm->reg == 1 ? 1 : prm->n_outer; }

// Images [b0, b0 + nb) of a solve: buffers in ws, and the start (g = A'^T Y,
// d = b = 0) enqueued on s.
static air_status part_begin(air_plan p, const float* Y, float* X, int b0, int nb, const air_solve_params* prm,
                             double* resid, char* ws, hipStream_t s, SolveBufs& B) {
    const size_t np = (size_t)p->g.n * p->g.n, nyv = (size_t)p->g.n_views * p->g.n_bins;
    B = solve_bufs(p, solve_layout(p, nb), ws, X + b0 * np, nb);
    if (resid) {
        B.resid = resid + (size_t)b0 * prm->n_outer;
        B.resid_stride = prm->n_outer;
    } else {
        B.iters = nullptr;          // residual norms go to scratch, one slot per image
    }
    return solve_init(p, B, Y + b0 * nyv, nb, solve_setup(prm), false, s);
}

static air_status check_solve(air_plan p, const float* Y, float* X, int32_t batch, const air_solve_params* prm) {
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_batch(p, batch, false)) return st;
    if (!Y || !X || !prm) return fail(AIR_E_INVALID, "null pointer");
    if (prm->reg < 0 || prm->reg > 2) return fail(AIR_E_INVALID, "reg must be 0, 1 or 2");
    if (prm->filter != 0 && prm->filter != 1) return fail(AIR_E_INVALID, "filter must be 0 or 1");
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) return fail(AIR_E_INVALID, "lambda must be >= 0");
    if (prm->reg != 1 && (!(prm->mu > 0.0) || !std::isfinite(prm->mu))) return fail(AIR_E_INVALID, "mu must be > 0");
    if (prm->n_outer < 0 || prm->n_cg < 0) return fail(AIR_E_INVALID, "iteration counts must be >= 0");
    return AIR_OK;
}

// The solve on workspace w (checked by the caller), as `parts` sub-batches.
static air_status solve_run(air_plan p, const float* Y, float* X, int32_t batch, const air_solve_params* prm,
                            double* resid, char* w, int parts, hipStream_t s) {
    if (parts == 1) {
        SolveBufs B;
        if (air_status st = part_begin(p, Y, X, 0, batch, prm, resid, w, s, B)) return st;
        for (int k = 0; k < solve_outer_count(prm); k++)
            if (air_status st = solve_outer(p, B, batch, solve_setup(prm), s)) return st;
        return AIR_OK;
    }
    // fork: both sub-streams wait for the caller's stream; join: the caller's
    // stream waits for both (also after a failed launch, so that nothing of
    // this call is still running on the workspace once the stream moves on)
    hipStream_t sub[2];
    AIR_HIP(device_sub_streams(sub));
    std::lock_guard<std::mutex> lock(p->fork_mu);
    for (int i = 0; i < 2; i++)
        if (!p->join_ev[i]) AIR_HIP(hipEventCreateWithFlags(&p->join_ev[i], hipEventDisableTiming));
    if (!p->fork_ev) AIR_HIP(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    AIR_HIP(hipEventRecord(p->fork_ev, s));
    // the two parts' outer iterations are enqueued alternately, so that both
    // streams have queued work from the start whatever the depth of their
    // queues (with the default depth this measured the same as enqueuing one
    // part whole and then the other)
    air_status result = AIR_OK;
    SolveBufs B[2];
    int nb[2];
    for (int i = 0, b0 = 0; i < 2; b0 += nb[i], i++) {
        nb[i] = part_size(batch, 2, i);
        AIR_HIP(hipStreamWaitEvent(sub[i], p->fork_ev, 0));
        if (result == AIR_OK)
            result = part_begin(p, Y, X, b0, nb[i], prm, resid, w + part_offset(p, batch, 2, i), sub[i], B[i]);
    }
    for (int k = 0; k < solve_outer_count(prm) && result == AIR_OK; k++)
        for (int i = 0; i < 2 && result == AIR_OK; i++) result = solve_outer(p, B[i], nb[i], solve_setup(prm), sub[i]);
    for (int i = 0; i < 2; i++) {
        AIR_HIP(hipEventRecord(p->join_ev[i], sub[i]));
        AIR_HIP(hipStreamWaitEvent(s, p->join_ev[i], 0));
    }
    return result;
}

air_status air_solve(air_plan p, const float* Y, float* X, int32_t batch, const air_solve_params* prm,
                     double* resid, void* ws, size_t ws_bytes, hipStream_t s) {
    if (air_status st = check_solve(p, Y, X, batch, prm)) return st;
    if (!ws) return fail(AIR_E_INVALID, "null pointer");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(AIR_E_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < solve_bytes(p, batch)) return fail(AIR_E_NOMEM, "workspace smaller than air_solve_workspace_size");
    return solve_run(p, Y, X, batch, prm, resid, static_cast<char*>(ws), solve_parts(p, batch), s);
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// air_solve_noalloc: the solve's scratch in a file-scope device array, one copy per
// GPU (the runtime places it when it loads the library's code on that GPU).
namespace {

__device__ __align__(256) static unsigned char scratch[AIR_NOALLOC_SCRATCH_BYTES];

// Device address of the current GPU's copy of `scratch`, looked up once per
// device with that device current.  On the host, `scratch` names a host-side
// stand-in: only these addresses may reach a kernel or a copy.
air_status scratch_address(char** out) {
    static std::mutex mu;
    static char* addr[64] = {};
    int dev = 0;
    AIR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(AIR_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* a = nullptr;
        AIR_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a) return fail(AIR_E_HIP, "hipGetSymbolAddress returned no address for the static scratch");
        addr[dev] = static_cast<char*>(a);
    }
    *out = addr[dev];
    return AIR_OK;
}

}  // namespace

extern "C" air_status air_solve_noalloc(air_plan p, const float* Y, float* X, int32_t batch,
                                        const air_solve_params* prm, double* resid, hipStream_t s) {
    if (air_status st = check_solve(p, Y, X, batch, prm)) return st;
    const size_t need = solve_layout(p, batch).total;
    if (need > AIR_NOALLOC_SCRATCH_BYTES)
        return fail(AIR_E_NOMEM, "air_solve_noalloc: this batch needs " + std::to_string(need) +
                                     " bytes of scratch, above the static " +
                                     std::to_string((size_t)AIR_NOALLOC_SCRATCH_BYTES) + " bytes");
    char* w = nullptr;
    if (air_status st = scratch_address(&w)) return st;
    return solve_run(p, Y, X, batch, prm, resid, w, 1, s);    // one stream: no streams or events to create
}
