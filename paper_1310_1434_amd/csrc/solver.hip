// The split-Bregman iteration (and the L2 solve of Eq. (5)) as sequences of
// kernel launches on one stream.  Shared by air_solve and the solve slots of
// air_state; an outer iteration has fixed launch parameters, so it can be
// captured once in a HIP graph and replayed.
#include "plan.h"

namespace air {

SolveLayout solve_layout(const air_plan_s* p, int batch) {
    const size_t B = (size_t)batch, n = (size_t)p->g.n, np = n * n;
    Carver c;
    SolveLayout L;
    const size_t gi = (size_t)group_images(batch);     // (solve slots run any batch up to their capacity)
    L.pad = c.take(gi * 2 * n * p->line * sizeof(float));   // grouped padded copies
    L.pscale = c.take((B + 63) / 64 * 64 * sizeof(float));
    L.s1 = c.take(B * p->g.n_views * p->ds * sizeof(float));
    L.s2 = c.take(gi * p->g.n_views * p->ds * sizeof(float));   // group-interleaved backprojector input
    L.rscale = c.take(B * p->g.n_views * sizeof(float));
    L.g = c.take(B * np * sizeof(float));
    L.r = c.take(B * np * sizeof(float));
    L.p = c.take(B * np * sizeof(float));
    L.q = c.take(B * np * sizeof(float));
    L.bb = c.take(B * 8 * np * sizeof(float));
    L.e = c.take(B * 9 * np * sizeof(float));
    L.part = c.take(B * tiles16((int)n) * sizeof(double));
    L.mx = c.take(2 * B * tiles16((int)n) * sizeof(float));
    L.scal = c.take(B * 4 * sizeof(double));
    L.iters = c.take(B * sizeof(int));
    L.total = c.off;
    return L;
}

SolveBufs solve_bufs(const air_plan_s* p, const SolveLayout& L, char* w, float* X, int batch) {
    auto F = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
    SolveBufs B;
    B.X = X;
    B.pad = F(L.pad);
    B.pscale = F(L.pscale);
    B.s1 = F(L.s1);
    B.s2 = F(L.s2);
    B.rscale = F(L.rscale);
    B.g = F(L.g);
    B.r = F(L.r);
    B.p = F(L.p);
    B.q = F(L.q);
    B.bb = F(L.bb);
    B.e = F(L.e);
    B.part = reinterpret_cast<double*>(w + L.part);
    B.rmax = reinterpret_cast<float*>(w + L.mx);
    B.pmax = B.rmax + (size_t)batch * tiles16(p->g.n);
    double* scal = reinterpret_cast<double*>(w + L.scal);
    B.rho = scal;
    B.alpha = scal + batch;
    B.beta = scal + 2 * batch;
    B.resid = scal + 3 * batch;     // scratch: one norm per image (stride 1, no counters)
    B.resid_stride = 1;
    B.iters = reinterpret_cast<int*>(w + L.iters);
    return B;
}

air_status solve_init(air_plan p, const SolveBufs& B, const float* Y, int batch, const SolveSetup& st, bool x_zero,
                      hipStream_t s) {
    const KGeom kg = p->kgeom();
    const int rows = batch * p->g.n_views;
    const size_t np = (size_t)p->g.n * p->g.n;
    // g = A'^T Y = J^T (S C Y), or A^T Y = J^T (S Y) for the IR arm
    const float* src = nullptr;
    if (air_status e = stage_sino(p, Y, batch, B.s1, &src, s)) return e;
    const int grp = image_group(batch);
    if (st.filter) AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(B.rscale), src, B.s2, rows, p->ds, RAMP_POST, grp, s));
    else AIR_K(AIR_K_OTHER, launch_scale(kg, src, B.s2, batch, grp, s));
    BpArgs a{};
    a.mode = BP_PLAIN;
    a.out = B.g;
    AIR_K(AIR_K_BACKPROJECT, launch_backproject(kg, B.s2, a, batch, s));
    if (st.reg == 0) {
        AIR_K(AIR_K_OTHER, launch_fill(B.bb, (size_t)batch * 8 * np, 0.f, s));
        AIR_K(AIR_K_OTHER, launch_fill(B.e, (size_t)batch * 9 * np, 0.f, s));
    }
    if (B.iters) AIR_K(AIR_K_OTHER, launch_fill(reinterpret_cast<float*>(B.iters), (size_t)batch, 0.f, s));
    // carried residual c = g - M X of the start image, in place of g (the
    // iterations never read g itself again); M 0 = 0, so c = g for X = 0
    if (st.reg != 2 && !x_zero) {
        const PadBuf pad = plan_pad(p, B.pad, B.pscale);
        if (air_status e = build_pad(p, B.X, pad, B.part, batch, s)) return e;
        AIR_K(AIR_K_PROJECT, launch_project(kg, pad, B.s1, batch, s));
        if (st.filter)
            AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(B.rscale), B.s1, B.s2, rows, p->ds, RAMP_POST, grp, s));
        else AIR_K(AIR_K_OTHER, launch_scale(kg, B.s1, B.s2, batch, grp, s));
        BpArgs r{};
        r.mode = BP_RESIDUAL;
        r.mu = (float)(st.reg == 0 ? st.mu : st.lambda);
        r.aux = B.X;
        r.out = B.g;
        r.p_out = B.p;      // (scratch here)
        r.partial = B.part;
        AIR_K(AIR_K_BACKPROJECT, launch_backproject(kg, B.s2, r, batch, s));
    }
    return AIR_OK;
}

PadBuf plan_pad(const air_plan_s* p, float* pad, float* scale) {
    PadBuf b;
    if (p->half_pad()) {
        b.half = reinterpret_cast<uint16_t*>(pad);
        b.scale = scale;
    } else {
        b.base = pad;
    }
    return b;
}

air_status build_pad(air_plan p, const float* x, const PadBuf& pad, double* partial, int batch, hipStream_t s) {
    const KGeom kg = p->kgeom();
    if (pad.half) {
        AIR_K(AIR_K_OTHER, launch_absmax(kg.n, x, partial, batch, s));
        AIR_K(AIR_K_OTHER, launch_pad_scale(partial, tiles16(kg.n), batch, pad.scale, s));
        AIR_K(AIR_K_OTHER, launch_pad16(kg, x, pad, batch, s));
    } else {
        AIR_K(AIR_K_OTHER, launch_pad(kg, x, pad, batch, s));
    }
    return AIR_OK;
}

// One forward-backward iteration (Eq. (6) and the framelet proximal step):
//   X' = X + mu (g - A'^T A X)  (= X - mu A'^T (A X - Y), g = A'^T Y from solve_init)
//   X  = W^T shrink(W X', mu lambda / 2);  resid = ||X_new - X_old||_2
static air_status fbs_iteration(air_plan p, const SolveBufs& B, int batch, const SolveSetup& st, hipStream_t s) {
    const KGeom kg = p->kgeom();
    const int n = p->g.n, rows = batch * p->g.n_views;
    const int grp = image_group(batch);
    const PadBuf pad = plan_pad(p, B.pad, B.pscale);
    if (air_status e = build_pad(p, B.X, pad, B.part, batch, s)) return e;
    AIR_K(AIR_K_PROJECT, launch_project(kg, pad, B.s1, batch, s));
    if (st.filter)
        AIR_K(AIR_K_RAMP, launch_ramp(p->prec, p->ramp_tables(B.rscale), B.s1, B.s2, rows, p->ds, RAMP_POST, grp, s));
    else AIR_K(AIR_K_OTHER, launch_scale(kg, B.s1, B.s2, batch, grp, s));
    BpArgs a{};
    a.mode = BP_STEP;
    a.mu = (float)st.mu;
    a.aux = B.X;
    a.rhs = B.g;
    a.out = B.r;
    AIR_K(AIR_K_BACKPROJECT, launch_backproject(kg, B.s2, a, batch, s));
    TfArgs t{};
    t.n = n;
    t.x = B.r;
    t.e = B.e;
    t.bb = B.X;
    t.thr = (float)(st.mu * st.lambda / 2.0);
    t.partial = B.part;
    AIR_K(AIR_K_FRAMELET, launch_fbs_shrink(t, batch, s));
    AIR_K(AIR_K_FRAMELET, launch_fbs_adjoint(t, batch, s));
    AIR_K(AIR_K_FRAMELET, launch_finalize(FIN_RESID, B.part, tiles16(n), batch, nullptr, nullptr, B.resid,
                                          B.resid_stride, B.iters, s));
    return AIR_OK;
}

air_status solve_outer(air_plan p, const SolveBufs& B, int batch, const SolveSetup& st, hipStream_t s) {
    if (st.reg == 2) return fbs_iteration(p, B, batch, st, s);
    const KGeom kg = p->kgeom();
    const RampTables rt = p->ramp_tables(B.rscale);
    const int n = p->g.n, rows = batch * p->g.n_views, nblk = tiles16(n), nblk_bp = bp_blocks(n, batch);
    const int grp = image_group(batch);
    const bool tf = st.reg == 0;
    const float mu_op = (float)(tf ? st.mu : st.lambda);
    const PadBuf pad = plan_pad(p, B.pad, B.pscale);
    // the padded copies of p come out of k_cg_p, which produces p; float16
    // copies take a power-of-two scale per image, which the k_finalize before
    // it derives from a bound on max |p| (block maxima of r and of the last p)
    HalfScaleArgs hs{};
    if (pad.half) hs = HalfScaleArgs{B.rmax, B.pmax, pad.scale};
    // operator A'^T A + mu I = J^T (S C S) J + mu I (IR arm: J^T S^2 J + mu I)
    auto filtered = [&]() -> air_status {
        if (st.filter)
            AIR_K(AIR_K_RAMP, launch_ramp(p->prec, rt, B.s1, B.s2, rows, p->ds, RAMP_POST, grp, s));
        else AIR_K(AIR_K_OTHER, launch_scale(kg, B.s1, B.s2, batch, grp, s));
        return AIR_OK;
    };
    // r = c + mu W^T e (L2: r = c), rho = r.r, p = r.  c = g - M X is carried
    // from the last CG step of the previous outer iteration (solve_init for the
    // first), so the start residual costs no operator apply: in exact
    // arithmetic it is the right-hand side g + mu W^T e minus M X.
    // (with no CG step X stays as it is, and so does c)
    if (st.n_cg > 0) {
        AIR_K(AIR_K_CG, launch_cg_start(n, B.g, tf ? B.e : nullptr, (float)st.mu, B.r, B.part,
                                        pad.half ? B.rmax : nullptr, batch, s));
        AIR_K(AIR_K_CG, launch_finalize(FIN_RHO, B.part, nblk, batch, B.rho, nullptr, nullptr, 0, nullptr, s, hs));
        CgArgs c0{};
        c0.n = n;
        c0.r = B.r;
        c0.p = B.p;
        c0.pad = pad;
        c0.pmax = pad.half ? B.pmax : nullptr;
        AIR_K(AIR_K_CG, launch_cg_update_p(c0, batch, s));
    }
    for (int it = 0; it < st.n_cg; it++) {
        AIR_K(AIR_K_PROJECT, launch_project(kg, pad, B.s1, batch, s));
        if (air_status e = filtered()) return e;
        BpArgs a{};
        a.mode = BP_MATVEC;
        a.mu = mu_op;
        a.aux = B.p;
        a.out = B.q;
        a.partial = B.part;
        AIR_K(AIR_K_BACKPROJECT, launch_backproject(kg, B.s2, a, batch, s));
        AIR_K(AIR_K_CG, launch_finalize(FIN_ALPHA, B.part, nblk_bp, batch, B.rho, B.alpha, nullptr, 0, nullptr, s));
        CgArgs cg{};
        cg.n = n;
        cg.x = B.X;
        cg.r = B.r;
        cg.p = B.p;
        cg.q = B.q;
        cg.alpha = B.alpha;
        cg.beta = B.beta;
        cg.partial = B.part;
        if (it == st.n_cg - 1) {
            // the last step leaves c = g - M X for the next outer iteration
            cg.c = B.g;
            cg.framelet = tf;
            cg.mu = (float)st.mu;
            AIR_K(AIR_K_CG, launch_cg_update_xc(cg, batch, s));
            break;
        }
        cg.rmax = pad.half ? B.rmax : nullptr;
        AIR_K(AIR_K_CG, launch_cg_update_xr(cg, batch, s));
        AIR_K(AIR_K_CG, launch_finalize(FIN_BETA, B.part, nblk, batch, B.rho, B.beta, nullptr, 0, nullptr, s, hs));
        cg.pad = pad;
        cg.pmax = pad.half ? B.pmax : nullptr;
        AIR_K(AIR_K_CG, launch_cg_update_p(cg, batch, s));
    }
    if (tf) {
        TfArgs t{};
        t.n = n;
        t.x = B.X;
        t.bb = B.bb;
        t.e = B.e;
        t.thr = (float)(st.lambda / (2.0 * st.mu));
        t.partial = B.part;
        AIR_K(AIR_K_FRAMELET, launch_tf_shrink(t, batch, s));
        AIR_K(AIR_K_FRAMELET, launch_finalize(FIN_RESID, B.part, nblk, batch, nullptr, nullptr, B.resid,
                                              B.resid_stride, B.iters, s));
    }
    return AIR_OK;
}

}  // namespace air
