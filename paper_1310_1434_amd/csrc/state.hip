// Device-resident solve slots for continuous batching (air_state_*).
//
// A state holds up to `capacity` split-Bregman reconstructions of one plan's
// geometry.  Every slot keeps its image X, the carried residual
// c = A'^T Y - (A'^T A + mu I) X, the Bregman variables b and e = d - b, its
// residual history and its iteration counter on the device; the CG state is
// rebuilt from them at the start of every outer iteration, so nothing else
// needs to persist.  Active slots are kept packed at positions
// [0, nact): retiring a slot moves the last active one into its place (a few
// device copies), so every step runs the batched kernels on a dense batch.
// Each image's arithmetic does not depend on its neighbours, so a slot's
// result is the same bits alone, in any mix, and at any position.
//
// One outer iteration for nact active slots is captured once into a HIP
// graph (on a non-default stream) and replayed for every later step with the
// same nact.
#include <new>

#include "plan.h"

namespace {

constexpr uint32_t kSnapMagic = 0x41495253u;   // "AIRS"

struct SnapHeader {
    uint32_t magic;
    int32_t n, n_views, n_bins;
    int32_t n_outer, iters, max_outer;
    int32_t filter;
    double lambda, mu;
    int32_t n_cg;
    int32_t reserved;
};

}  // namespace

struct air_state_s {
    air_plan plan = nullptr;
    int capacity = 0;
    int max_outer = 0;
    SolveSetup setup{};
    SolveLayout L{};
    char* ws = nullptr;
    size_t off_x = 0, off_hist = 0;
    SolveBufs B{};                     // positions [0, capacity)
    int nact = 0;
    std::vector<int> pos_of;           // slot -> position, -1 if free
    std::vector<int> slot_at;          // position -> slot
    std::vector<int> n_outer, iters;   // per slot (host mirror of the device counters)
    std::vector<hipGraphExec_t> graphs;   // indexed by nact, captured lazily

    ~air_state_s() {
        for (hipGraphExec_t g : graphs)
            if (g) (void)hipGraphExecDestroy(g);
    }
    size_t np() const { return (size_t)plan->g.n * plan->g.n; }
    // SolveBufs viewing a single image at position `pos` (batch 1)
    SolveBufs at(int pos) const {
        SolveBufs b = B;
        const size_t n = np();
        b.X += pos * n;
        b.g += pos * n;
        b.r += pos * n;
        b.p += pos * n;
        b.q += pos * n;
        b.bb += pos * 8 * n;
        b.e += pos * 9 * n;
        b.part += (size_t)pos * tiles16(plan->g.n);
        b.rmax += (size_t)pos * tiles16(plan->g.n);
        b.pmax += (size_t)pos * tiles16(plan->g.n);
        b.rho += pos;
        b.alpha += pos;
        b.beta += pos;
        b.resid += (size_t)pos * max_outer;
        b.iters += pos;
        return b;
    }
};

namespace {

size_t state_bytes(const air_plan_s* p, int capacity, int max_outer, SolveLayout* L, size_t* off_x,
                   size_t* off_hist) {
    const SolveLayout l = solve_layout(p, capacity);
    Carver c;
    c.off = l.total;
    const size_t ox = c.take((size_t)capacity * p->g.n * p->g.n * sizeof(float));
    const size_t oh = c.take((size_t)capacity * max_outer * sizeof(double));
    if (L) *L = l;
    if (off_x) *off_x = ox;
    if (off_hist) *off_hist = oh;
    return c.off;
}

air_status check_params(const air_solve_params* prm) {
    if (!prm) return fail(AIR_E_INVALID, "params are null");
    if (prm->reg != 0) return fail(AIR_E_UNSUPPORTED, "solve slots run the split Bregman solver (reg = 0)");
    if (prm->filter != 0 && prm->filter != 1) return fail(AIR_E_INVALID, "filter must be 0 or 1");
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) return fail(AIR_E_INVALID, "lambda must be >= 0");
    if (!(prm->mu > 0.0) || !std::isfinite(prm->mu)) return fail(AIR_E_INVALID, "mu must be > 0");
    if (prm->n_outer < 1 || prm->n_cg < 0) return fail(AIR_E_INVALID, "need n_outer >= 1 and n_cg >= 0");
    return AIR_OK;
}

// copy one position's persistent data to another (device to device, on the stream)
air_status move_slot(air_state st, int from, int to, hipStream_t s) {
    const SolveBufs a = st->at(from), b = st->at(to);
    const size_t n = st->np() * sizeof(float);
    AIR_HIP(hipMemcpyAsync(b.X, a.X, n, hipMemcpyDeviceToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.g, a.g, n, hipMemcpyDeviceToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.bb, a.bb, 8 * n, hipMemcpyDeviceToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.e, a.e, 9 * n, hipMemcpyDeviceToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.resid, a.resid, st->max_outer * sizeof(double), hipMemcpyDeviceToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.iters, a.iters, sizeof(int), hipMemcpyDeviceToDevice, s));
    return AIR_OK;
}

air_status take_position(air_state st, int n_outer, int iters, int* slot_out) {
    int slot = -1;
    for (int i = 0; i < st->capacity; i++)
        if (st->pos_of[i] < 0) {
            slot = i;
            break;
        }
    if (slot < 0 || st->nact >= st->capacity) return fail(AIR_E_NOMEM, "no free slot");
    const int pos = st->nact++;
    st->pos_of[slot] = pos;
    st->slot_at[pos] = slot;
    st->n_outer[slot] = n_outer;
    st->iters[slot] = iters;
    *slot_out = slot;
    return AIR_OK;
}

air_status check_slot(air_state st, int32_t slot) {
    if (!st) return fail(AIR_E_INVALID, "state is null");
    if (slot < 0 || slot >= st->capacity || st->pos_of[slot] < 0) return fail(AIR_E_INVALID, "no such active slot");
    return AIR_OK;
}

}  // namespace

extern "C" {

air_status air_state_workspace_size(air_plan p, int32_t capacity, const air_solve_params* prm, size_t* bytes) {
    if (air_status st = check_plan(p, false)) return st;
    if (air_status st = check_params(prm)) return st;
    if (capacity < 1) return fail(AIR_E_INVALID, "capacity must be >= 1");
    if (!bytes) return fail(AIR_E_INVALID, "bytes is null");
    *bytes = state_bytes(p, capacity, prm->n_outer, nullptr, nullptr, nullptr);
    return AIR_OK;
}

air_status air_state_create(air_plan p, int32_t capacity, const air_solve_params* prm, void* ws, size_t ws_bytes,
                            air_state* out) {
    if (!out) return fail(AIR_E_INVALID, "out is null");
    *out = nullptr;
    if (air_status st = check_plan(p, true)) return st;
    if (air_status st = check_params(prm)) return st;
    if (capacity < 1) return fail(AIR_E_INVALID, "capacity must be >= 1");
    if (!ws) return fail(AIR_E_INVALID, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(AIR_E_INVALID, "workspace must be 256-byte aligned");
    air_state_s* st = new (std::nothrow) air_state_s;
    if (!st) return fail(AIR_E_NOMEM, "host allocation failed");
    const size_t need = state_bytes(p, capacity, prm->n_outer, &st->L, &st->off_x, &st->off_hist);
    if (ws_bytes < need) {
        delete st;
        return fail(AIR_E_NOMEM, "workspace smaller than air_state_workspace_size");
    }
    st->plan = p;
    st->capacity = capacity;
    st->max_outer = prm->n_outer;
    st->setup = SolveSetup{0, prm->filter, prm->lambda, prm->mu, prm->n_cg};
    st->ws = static_cast<char*>(ws);
    st->B = solve_bufs(p, st->L, st->ws, reinterpret_cast<float*>(st->ws + st->off_x), capacity);
    st->B.resid = reinterpret_cast<double*>(st->ws + st->off_hist);
    st->B.resid_stride = st->max_outer;
    st->pos_of.assign(capacity, -1);
    st->slot_at.assign(capacity, -1);
    st->n_outer.assign(capacity, 0);
    st->iters.assign(capacity, 0);
    st->graphs.assign(capacity + 1, nullptr);
    *out = st;
    return AIR_OK;
}

void air_state_destroy(air_state st) { delete st; }

air_status air_state_admit(air_state st, const float* Y, const float* X0, int32_t n_outer, hipStream_t s,
                           int32_t* slot_out) {
    if (!st) return fail(AIR_E_INVALID, "state is null");
    if (!Y || !slot_out) return fail(AIR_E_INVALID, "null pointer");
    if (n_outer < 1 || n_outer > st->max_outer) return fail(AIR_E_INVALID, "n_outer outside [1, the state's n_outer]");
    if (st->nact >= st->capacity) return fail(AIR_E_NOMEM, "no free slot");
    int slot = -1;
    if (air_status e = take_position(st, n_outer, 0, &slot)) return e;
    air_plan p = st->plan;
    const int pos = st->pos_of[slot];
    const SolveBufs b = st->at(pos);
    const size_t n = st->np();
    air_status e = AIR_OK;
    if (X0) {
        const hipError_t h = hipMemcpyAsync(b.X, X0, n * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (h != hipSuccess) e = fail(AIR_E_HIP, std::string("admit: ") + hipGetErrorString(h));
    } else {
        const hipError_t h = launch_fill(b.X, n, 0.f, s);
        if (h != hipSuccess) e = fail(AIR_E_HIP, std::string("admit: ") + hipGetErrorString(h));
    }
    if (e == AIR_OK) {   // residual history starts at zero (deterministic snapshots)
        const hipError_t h = launch_fill(reinterpret_cast<float*>(b.resid), 2 * (size_t)st->max_outer, 0.f, s);
        if (h != hipSuccess) e = fail(AIR_E_HIP, std::string("admit: ") + hipGetErrorString(h));
    }
    if (e == AIR_OK) e = solve_init(p, b, Y, 1, st->setup, X0 == nullptr, s);
    if (e != AIR_OK) {     // give the position back
        st->pos_of[slot] = -1;
        st->slot_at[pos] = -1;
        st->nact--;
        return e;
    }
    *slot_out = slot;
    return AIR_OK;
}

air_status air_state_step(air_state st, int32_t max_iters, hipStream_t s, int32_t* done_iters) {
    if (!st) return fail(AIR_E_INVALID, "state is null");
    if (max_iters < 0) return fail(AIR_E_INVALID, "max_iters must be >= 0");
    int k = max_iters;
    for (int pos = 0; pos < st->nact; pos++) {
        const int slot = st->slot_at[pos];
        k = std::min(k, st->n_outer[slot] - st->iters[slot]);
    }
    if (st->nact == 0) k = 0;
    if (done_iters) *done_iters = k;
    if (k <= 0) return AIR_OK;
    air_plan p = st->plan;
    const int nact = st->nact;
    SolveBufs b = st->B;                // positions [0, nact)
    hipGraphExec_t& exec = st->graphs[nact];
    const bool graphs = s != nullptr && !p->timing;
    if (graphs && !exec) {
        AIR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const air_status e = solve_outer(p, b, nact, st->setup, s);
        hipGraph_t graph = nullptr;
        const hipError_t h = hipStreamEndCapture(s, &graph);
        if (e != AIR_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return e;
        }
        if (h != hipSuccess) return fail(AIR_E_HIP, std::string("graph capture: ") + hipGetErrorString(h));
        const hipError_t h2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (h2 != hipSuccess) {
            exec = nullptr;
            return fail(AIR_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(h2));
        }
    }
    for (int i = 0; i < k; i++) {
        if (graphs) AIR_HIP(hipGraphLaunch(exec, s));
        else if (air_status e = solve_outer(p, b, nact, st->setup, s)) return e;
    }
    for (int pos = 0; pos < nact; pos++) st->iters[st->slot_at[pos]] += k;
    return AIR_OK;
}

air_status air_state_query(air_state st, int32_t slot, int32_t* iters_done, int32_t* n_outer) {
    if (air_status e = check_slot(st, slot)) return e;
    if (iters_done) *iters_done = st->iters[slot];
    if (n_outer) *n_outer = st->n_outer[slot];
    return AIR_OK;
}

air_status air_state_active(air_state st, int32_t* count) {
    if (!st || !count) return fail(AIR_E_INVALID, "null pointer");
    *count = st->nact;
    return AIR_OK;
}

air_status air_state_poll(air_state st, int32_t* done_mask) {
    if (!st || !done_mask) return fail(AIR_E_INVALID, "null pointer");
    const int words = (st->capacity + 31) / 32;
    for (int w = 0; w < words; w++) done_mask[w] = 0;
    for (int slot = 0; slot < st->capacity; slot++)
        if (st->pos_of[slot] >= 0 && st->iters[slot] >= st->n_outer[slot])
            done_mask[slot / 32] = (int32_t)((uint32_t)done_mask[slot / 32] | (1u << (slot % 32)));
    return AIR_OK;
}

air_status air_state_retire(air_state st, int32_t slot, float* X_out, double* resid_out, hipStream_t s) {
    if (air_status e = check_slot(st, slot)) return e;
    const int pos = st->pos_of[slot];
    const SolveBufs b = st->at(pos);
    const int n_out = st->n_outer[slot];
    std::vector<double> hist;
    try {
        hist.assign(n_out, 0.0);
    } catch (const std::bad_alloc&) {
        return fail(AIR_E_NOMEM, "host allocation failed");
    }
    // the history is read before the slot's position can be reused below
    AIR_HIP(hipMemcpyAsync(hist.data(), b.resid, n_out * sizeof(double), hipMemcpyDeviceToHost, s));
    if (X_out) AIR_HIP(hipMemcpyAsync(X_out, b.X, st->np() * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (resid_out) AIR_HIP(hipMemcpyAsync(resid_out, b.resid, n_out * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int last = st->nact - 1;
    if (pos != last) {
        if (air_status e = move_slot(st, last, pos, s)) return e;
        const int moved = st->slot_at[last];
        st->slot_at[pos] = moved;
        st->pos_of[moved] = pos;
    }
    st->slot_at[last] = -1;
    st->pos_of[slot] = -1;
    st->nact--;
    AIR_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < n_out; k++)
        if (!std::isfinite(hist[k]))
            return fail(AIR_E_NONFINITE, "the slot's residual history holds a non-finite value (iteration " +
                                             std::to_string(k) + ")");
    return AIR_OK;
}

air_status air_state_snapshot_size(air_state st, size_t* bytes) {
    if (!st || !bytes) return fail(AIR_E_INVALID, "null pointer");
    const size_t n = st->np();
    *bytes = sizeof(SnapHeader) + (1 + 1 + 8 + 9) * n * sizeof(float) + st->max_outer * sizeof(double);
    return AIR_OK;
}

air_status air_state_snapshot(air_state st, int32_t slot, void* host_buf, hipStream_t s) {
    if (air_status e = check_slot(st, slot)) return e;
    if (!host_buf) return fail(AIR_E_INVALID, "buffer is null");
    const air_plan p = st->plan;
    SnapHeader h{};
    h.magic = kSnapMagic;
    h.n = p->g.n;
    h.n_views = p->g.n_views;
    h.n_bins = p->g.n_bins;
    h.n_outer = st->n_outer[slot];
    h.iters = st->iters[slot];
    h.max_outer = st->max_outer;
    h.filter = st->setup.filter;
    h.lambda = st->setup.lambda;
    h.mu = st->setup.mu;
    h.n_cg = st->setup.n_cg;
    char* o = static_cast<char*>(host_buf);
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    const SolveBufs b = st->at(st->pos_of[slot]);
    const size_t n = st->np() * sizeof(float);
    AIR_HIP(hipMemcpyAsync(o, b.X, n, hipMemcpyDeviceToHost, s));
    AIR_HIP(hipMemcpyAsync(o + n, b.g, n, hipMemcpyDeviceToHost, s));
    AIR_HIP(hipMemcpyAsync(o + 2 * n, b.bb, 8 * n, hipMemcpyDeviceToHost, s));
    AIR_HIP(hipMemcpyAsync(o + 10 * n, b.e, 9 * n, hipMemcpyDeviceToHost, s));
    AIR_HIP(hipMemcpyAsync(o + 19 * n, b.resid, st->max_outer * sizeof(double), hipMemcpyDeviceToHost, s));
    return AIR_OK;
}

air_status air_state_restore(air_state st, const void* host_buf, hipStream_t s, int32_t* slot_out) {
    if (!st || !host_buf || !slot_out) return fail(AIR_E_INVALID, "null pointer");
    SnapHeader h;
    std::memcpy(&h, host_buf, sizeof h);
    const air_plan p = st->plan;
    if (h.magic != kSnapMagic || h.n != p->g.n || h.n_views != p->g.n_views || h.n_bins != p->g.n_bins)
        return fail(AIR_E_INVALID, "snapshot does not match this state's geometry");
    if (h.max_outer != st->max_outer || h.filter != st->setup.filter || h.lambda != st->setup.lambda ||
        h.mu != st->setup.mu || h.n_cg != st->setup.n_cg)
        return fail(AIR_E_INVALID, "snapshot was taken with different solver parameters");
    if (h.iters < 0 || h.iters > h.n_outer || h.n_outer > st->max_outer)
        return fail(AIR_E_INVALID, "corrupt snapshot header");
    int slot = -1;
    if (air_status e = take_position(st, h.n_outer, h.iters, &slot)) return e;
    const SolveBufs b = st->at(st->pos_of[slot]);
    const char* o = static_cast<const char*>(host_buf) + sizeof h;
    const size_t n = st->np() * sizeof(float);
    AIR_HIP(hipMemcpyAsync(b.X, o, n, hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.g, o + n, n, hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.bb, o + 2 * n, 8 * n, hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.e, o + 10 * n, 9 * n, hipMemcpyHostToDevice, s));
    AIR_HIP(hipMemcpyAsync(b.resid, o + 19 * n, st->max_outer * sizeof(double), hipMemcpyHostToDevice, s));
    const int it = h.iters;
    AIR_HIP(hipMemcpyAsync(b.iters, &it, sizeof(int), hipMemcpyHostToDevice, s));
    AIR_HIP(hipStreamSynchronize(s));     // `it` and the caller's buffer are read before returning
    *slot_out = slot;
    return AIR_OK;
}

}  // extern "C"
