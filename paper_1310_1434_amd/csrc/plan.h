// Internal: the plan object, launch bracketing, argument checks and the
// split-Bregman iteration shared by air_solve and the solve slots.
#pragma once

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "air_internal.h"

namespace air {

air_status fail(air_status st, const std::string& msg);

#define AIR_HIP(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return air::fail(AIR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    }
};

}  // namespace air

using namespace air;

struct air_plan_s {
    GeomHost g;
    int max_batch = 1;
    air_precision prec = AIR_FP32;
    int ds = 0, line = 0, c0 = 0;
    double kappa = 0.0;
    std::vector<RayEntry> rays;
    std::vector<float> step;       // [n_views][ds] path length per driving step, 0 in the padding
    std::vector<int8_t> axis;
    std::vector<int32_t> lo, hi;
    std::vector<float> views;      // interleaved (cos, sin) as float
    std::vector<int32_t> vorder;   // [2][v_half] views by majority axis (-1 padded), see KGeom
    int v_half = 0;
    std::vector<float> taps32;     // [2 ds]
    int ramp_window = 0;           // 0 Ram-Lak, 1 Shepp-Logan, 2 Hann
    bool cos_weight = false;       // symmetric fan-beam cosine weighting of C
    std::vector<float> wsq;        // [ds] sqrt of the cosine weights (0 in the padding), if cos_weight
    std::vector<uint16_t> tab16;   // 16-bit split tap tables (RampTables::tab16)
    int n_terms = 0;
    // workspace layout (bytes)
    size_t off_rays = 0, off_step = 0, off_views = 0, off_taps = 0, off_tab16 = 0, off_wsq = 0,
           off_vorder = 0, off_bpwin = 0, off_bpwinx = 0;
    size_t off_pad = 0, off_s1 = 0, off_s2 = 0, off_pscale = 0, off_ppart = 0, off_rscale = 0, total = 0;
    char* ws = nullptr;
    // per-kernel event timing (air_kernel_timing_enable)
    struct Timed {
        int kind;
        hipEvent_t a, b;
    };
    int timing = AIR_TIMING_OFF;   // air_kernel_timing_mode
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    // air_solve's concurrent sub-batches: the events that fork the device's
    // two sub-batch streams from, and join them back to, the caller's stream;
    // created on first use, guarded by fork_mu.
    hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
    std::mutex fork_mu;

    ~air_plan_s() {
        for (const Timed& t : pending) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (int i = 0; i < 2; i++)
            if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
    }
    hipEvent_t take_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    KGeom kgeom() const { return kgeom_at(ws); }
    // the same for a workspace at base (before it is bound)
    KGeom kgeom_at(const char* base) const {
        KGeom k;
        k.n = g.n;
        k.n_views = g.n_views;
        k.n_bins = g.n_bins;
        k.ds = ds;
        k.line = line;
        k.c0 = c0;
        k.beam = g.beam;
        k.pixel = (float)g.pixel;
        k.half_n = (float)(0.5 * (g.n - 1));
        k.inv_bin = (float)(1.0 / g.bin);
        k.half_d = (float)(0.5 * (g.n_bins - 1));
        k.sod = (float)g.sod;
        k.sdd = (float)g.sdd;
        k.rays = reinterpret_cast<const RayEntry*>(base + off_rays);
        k.step = reinterpret_cast<const float*>(base + off_step);
        k.views = reinterpret_cast<const float2*>(base + off_views);
        k.vorder = reinterpret_cast<const int32_t*>(base + off_vorder);
        k.v_half = v_half;
        k.kdet = (float)(g.sdd / g.bin);
        k.bpwin = reinterpret_cast<const BpWin*>(base + off_bpwin);
        k.bpwinx = reinterpret_cast<const float2*>(base + off_bpwinx);
        return k;
    }
    // rscale: [rows] scratch of the float16 split's per-row scales (used by
    // AIR_MIXED_F16 plans only)
    RampTables ramp_tables(float* rscale) const {
        RampTables t;
        t.taps32 = reinterpret_cast<const float*>(ws + off_taps);
        t.step = reinterpret_cast<const float*>(ws + off_step);
        t.n_views = g.n_views;
        t.tab16 = n_terms > 0 ? reinterpret_cast<const uint2*>(ws + off_tab16) : nullptr;
        t.n_terms = n_terms;
        t.tab_j = ramp_tab_j(ds);
        t.out_scale = (float)(kappa / 4096.0);
        t.wsq = cos_weight ? reinterpret_cast<const float*>(ws + off_wsq) : nullptr;
        t.rscale = prec == AIR_MIXED_F16 ? rscale : nullptr;
        return t;
    }
    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    bool direct(const void* p) const { return g.n_bins == ds && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
    // mixed-precision plans keep the projector's padded copies in float16
    bool half_pad() const { return prec != AIR_FP32; }
};

namespace air {

// Brackets one kernel launch with events when timing is enabled on the plan.
struct KTimer {
    air_plan_s* p;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(air_plan_s* p_, int kind_, hipStream_t s_) : p(p_), kind(kind_), s(s_) {
        if (p->timing) {
            a = p->take_event();
            b = p->take_event();
            if (a && b && hipEventRecord(a, s) != hipSuccess) a = nullptr;
        }
    }
    void done() {
        if (a && b && hipEventRecord(b, s) == hipSuccess) p->pending.push_back({kind, a, b});
    }
};

#define AIR_K(kind, expr)             \
    do {                              \
        KTimer t_(p, kind, s);        \
        AIR_HIP(expr);                \
        t_.done();                    \
    } while (0)

inline air_status check_plan(air_plan p, bool need_ws) {
    if (!p) return fail(AIR_E_INVALID, "plan is null");
    if (need_ws && !p->ws) return fail(AIR_E_INVALID, "plan has no workspace bound");
    return AIR_OK;
}

inline air_status check_batch(air_plan p, int32_t batch, bool bounded) {
    if (batch < 1) return fail(AIR_E_INVALID, "batch must be >= 1");
    if (bounded && batch > p->max_batch) return fail(AIR_E_INVALID, "batch exceeds the plan's max_batch");
    return AIR_OK;
}

// y (public stride n_bins) -> internal rows of stride ds, unless it can be read in place.
inline air_status stage_sino(air_plan p, const float* y, int32_t batch, float* scratch, const float** out, hipStream_t s) {
    if (p->direct(y)) {
        *out = y;
        return AIR_OK;
    }
    const int rows = batch * p->g.n_views;
    AIR_K(AIR_K_OTHER, launch_repack(y, p->g.n_bins, scratch, p->ds, rows, p->g.n_bins, p->ds, s));
    *out = scratch;
    return AIR_OK;
}


// Device buffers of a batch of reconstructions in the split-Bregman loop
// (images at positions [0, batch); per-image buffers are contiguous per image).
struct SolveBufs {
    float* X;       // [batch][n][n] current image
    float* pad;     // grouped padded copies of X or p (PadBuf), rebuilt every outer iteration
    float* pscale;  // [batch] scales of float16 padded copies (mixed-precision plans)
    float* s1;      // [batch][n_views][ds] projections
    float* s2;      // group-interleaved backprojector input (G = image_group(batch))
    float* rscale;  // [batch][n_views] per-row scales of the float16 split ramp
    float* g;       // [batch][n][n]  A'^T Y; split Bregman and L2: g - M X after solve_init (M = A'^T A + mu I)
    float* r;       // [batch][n][n]  CG residual
    float* p;       // [batch][n][n]
    float* q;       // [batch][n][n]
    float* bb;      // [batch][8][n][n] Bregman b (bands 1..8)
    float* e;       // [batch][9][n][n] d - b
    double* part;   // [batch][tiles16(n)] block partial sums
    float* rmax;    // [batch][tiles16(n)] block maxima of |r| (float16 scales of p)
    float* pmax;    // [batch][tiles16(n)] block maxima of |p|
    double* rho;    // [batch]
    double* alpha;  // [batch]
    double* beta;   // [batch]
    double* resid;  // residual history, resid[b * resid_stride + iters[b]]
    int resid_stride;
    int* iters;     // [batch] per-image Bregman iteration counters, or null (then resid[b * stride])
};

struct SolveSetup {
    int reg;        // 0 split Bregman, 1 L2 (Eq. (5)), 2 forward-backward splitting (Eq. (6))
    int filter;     // 1 AIR, 0 IR
    double lambda, mu;
    int n_cg;
};

// Bytes of the per-image buffers of SolveBufs (excluding the sinogram scratch).
struct SolveLayout {
    size_t pad, pscale, s1, s2, rscale, g, r, p, q, bb, e, part, mx, scal, iters, total;
};
SolveLayout solve_layout(const air_plan_s* p, int batch);
SolveBufs solve_bufs(const air_plan_s* p, const SolveLayout& L, char* ws, float* X, int batch);
// The projector's padded copies of x: float32 image pairs, or (mixed-precision
// plans) float16 groups with per-image power-of-two scales from max |x|
// (partial: [batch][tiles16(n)] scratch).
PadBuf plan_pad(const air_plan_s* p, float* pad, float* scale);
air_status build_pad(air_plan p, const float* x, const PadBuf& pad, double* partial, int batch, hipStream_t s);

// g = A'^T Y (or A^T Y); zero b and e.  Y: [batch][V][D] (public layout).
// Split Bregman and L2: then g -= M X (one operator apply; none if x_zero,
// X = 0), the carried residual every L2 sub-problem starts from.
air_status solve_init(air_plan p, const SolveBufs& B, const float* Y, int batch, const SolveSetup& st, bool x_zero,
                      hipStream_t s);
// One outer iteration (split Bregman) or the whole CG run (L2) for images [0, batch).
air_status solve_outer(air_plan p, const SolveBufs& B, int batch, const SolveSetup& st, hipStream_t s);

}  // namespace air
