/*
 * air.h -- C ABI of the MI355X (gfx950) AIR reconstruction library.
 *
 * AIR, the fused analytical and iterative reconstruction of arXiv 1310.1434,
 * minimises ||P(AX - Y)||^2 + lambda R(X) with P^T P = C, the analytic
 * method's filtration (Methods, Eq. (1)-(3)).  Its solvers only ever need
 * A, the filtered adjoint A'^T = A^T C (Methods, text before Eq. (5)) and,
 * for R = ||W X||_1 with a tensor framelet W (Materials), the split Bregman
 * L2 step, solved like Eq. (5).  This library runs exactly that hot path on
 * one GPU with hand-written HIP kernels.
 *
 * Conventions
 *   - Every function returns air_status; AIR_OK is 0.  On failure
 *     air_last_error() gives a thread-local message.  No C++ exception
 *     crosses the ABI.  Argument checks happen before any GPU work is
 *     queued, so they need no GPU.
 *   - The library never allocates device memory.  The caller owns every
 *     device buffer (inputs, outputs and workspaces) and passes plain device
 *     pointers; host pointers are marked "host".
 *   - Work is queued on the caller's hipStream_t (0 = the legacy default
 *     stream) and is asynchronous unless stated otherwise.  Calls that use
 *     the same plan workspace must be ordered on one stream.
 *   - Layouts are row-major, last index fastest, batch outermost:
 *       image    X[b][j][i]       j = row (y), i = column (x), n x n
 *       sinogram Y[b][v][k]       v = view, k = detector bin
 *       framelet Z[b][band][j][i] band = 3 m_y + m_x, band 0 = low-pass
 *     All are float32.
 *
 * Geometry (shared with the scan model the inputs come from)
 *   pixel (i, j) centre: ((i - (n-1)/2) pixel, (j - (n-1)/2) pixel)
 *   bin k: u_k = (k - (n_bins-1)/2) bin
 *   parallel beam, view (c, s) = (cos, sin):  ray through u_k (c, s), direction (-s, c)
 *   flat fan beam: source sod (c, s), ray direction (-sdd c - u_k s, -sdd s + u_k c)
 *   The view cosines/sines are passed in (float64, host) so the caller's
 *   angle set is used bit for bit.
 */
#ifndef AIR_H
#define AIR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AIR_OK = 0,
    AIR_E_INVALID = -1,      /* bad argument (null pointer, size, geometry, batch > max_batch) */
    AIR_E_UNSUPPORTED = -2,  /* valid but outside what the kernels handle (e.g. n > 16384) */
    AIR_E_NOMEM = -3,        /* workspace too small, or host allocation failed */
    AIR_E_HIP = -4,          /* a HIP call failed (message holds hipGetErrorString) */
    AIR_E_NONFINITE = -5     /* a solve slot's residual history holds a non-finite value
                                (air_state_retire; the slot is still copied out and freed) */
} air_status;

typedef enum { AIR_PARALLEL = 0, AIR_FAN_FLAT = 1 } air_beam;

/* Arithmetic of the ramp filtration (the only dense contraction on the path).
 *   AIR_FP32        float32 MFMA (v_mfma_f32_16x16x4f32), float32 accumulation
 *   AIR_MIXED_F16   float16 MFMA on a hi/lo split of sinogram and filter,
 *                   three products, float32 accumulation
 *   AIR_MIXED_BF16  bfloat16 MFMA on a three-way split, six products,
 *                   float32 accumulation
 * In the two mixed modes the forward projector also reads its image copies
 * in float16 (each image scaled by a power of two so that its largest value
 * lies in [2^13, 2^14); inside a solve's CG steps, so that a bound on the
 * direction's largest value, at most twice that value, does; the scale is
 * undone exactly on the float32 sums), which halves the bytes of its gathers.  Projector accumulation, images,
 * sinograms and CG vectors are float32 in all modes; CG inner products, the
 * step sizes alpha/beta and the Bregman residual norm are float64.
 * Range: the projector and backprojector sum interpolation weights scaled by
 * 2^32 (the scale is undone exactly), so float32 images and sinograms must
 * stay below 2^80 (about 1.2e24) in magnitude, and their products with the
 * operators below float32's largest value; within that range every operator
 * commutes with power-of-two scaling bit for bit.  Larger values overflow to
 * infinity (the mixed modes' scaled image copies lift the limit for the
 * projector's input only). */
typedef enum { AIR_FP32 = 0, AIR_MIXED_F16 = 1, AIR_MIXED_BF16 = 2 } air_precision;

typedef struct {
    air_beam beam;
    int32_t n;                 /* image is n x n, 1 <= n <= 16384 */
    double pixel_mm;           /* pixel side > 0 */
    int32_t n_views;           /* >= 1 */
    const double* view_cos;    /* host, [n_views]; copied at plan creation */
    const double* view_sin;    /* host, [n_views]; copied at plan creation */
    int32_t n_bins;            /* 1 <= n_bins <= 8192 */
    double bin_mm;             /* detector pitch > 0 */
    double sod_mm, sdd_mm;     /* fan beam: 0 < sod < sdd; ignored for parallel beam */
} air_geometry;

typedef struct air_plan_s* air_plan;

/* Plan flags: the filtration C of AIR (Methods, Eqs. (2)-(3): any symmetric
 * positive semi-definite C = P^T P; the analytic method's filter is the
 * natural choice).  C = kappa D^(1/2) R D^(1/2) per view, R the symmetric
 * Toeplitz matrix of a ramp window's taps (dimensionless, see air_ramp):
 *   AIR_RAMP_RAM_LAK      r(0) = 1/4, r(odd m) = -1/(pi m)^2, else 0   (response |w| / 2 pi)
 *   AIR_RAMP_SHEPP_LOGAN  r(m) = -2 / (pi^2 (4 m^2 - 1))               (response |sin(w/2)| / pi)
 *   AIR_RAMP_HANN         Ram-Lak apodised by (1 + cos w) / 2:
 *                         r(m) / 2 + (r(m - 1) + r(m + 1)) / 4
 * and D the identity, or with AIR_RAMP_COSINE_WEIGHTED the flat-detector
 * fan-beam cosine weights D = diag(sdd / sqrt(sdd^2 + u_k^2)) (identity for
 * parallel beams), applied on both sides so that C stays symmetric. */
enum {
    AIR_RAMP_RAM_LAK = 0,
    AIR_RAMP_SHEPP_LOGAN = 1,
    AIR_RAMP_HANN = 2,
    AIR_RAMP_WINDOW_MASK = 15,
    AIR_RAMP_COSINE_WEIGHTED = 16
};

/* Create a plan: validates the geometry and builds, on the host in float64,
 * the per-ray Joseph tables (driving axis, index range, intercept, slope,
 * step length) and the ramp taps.  Nothing touches the GPU.
 * max_batch bounds the batch of the operator calls that use the plan's
 * workspace (air_project, air_filtered_backproject, air_ramp,
 * air_normal_apply).  flags: a ramp window, optionally or-ed with
 * AIR_RAMP_COSINE_WEIGHTED; any other bit is AIR_E_INVALID. */
air_status air_plan_create(const air_geometry* geom, int32_t max_batch, air_precision prec,
                           uint32_t flags, air_plan* out);

/* Device bytes the plan needs: tables, taps, the backprojector's window table
 * (24 bytes per 16 x 32 pixel tile and view) and operator scratch for max_batch. */
air_status air_plan_workspace_size(air_plan plan, size_t* bytes);

/* Hand the plan its workspace (device, 256-byte aligned, >= workspace_size
 * bytes, caller-owned, must outlive the plan's use), upload the tables and
 * build the backprojector's window table from them (one kernel on `stream`).
 * Synchronises `stream` once (the host tables are copied before returning). */
air_status air_plan_bind_workspace(air_plan plan, void* dev_ptr, size_t bytes, hipStream_t stream);

/* Host copies of the index tables, each [n_views * n_bins]:
 *   axis 0 = x-driven (steps over columns), 1 = y-driven;
 *   lo/hi = first/last driving index whose intercept t satisfies -1 < t < n,
 *   evaluated in float64 without fused multiply-add; (0, -1) if none.
 * Any pointer may be NULL. */
air_status air_plan_tables(air_plan plan, int8_t* axis, int32_t* lo, int32_t* hi);

void air_plan_destroy(air_plan plan);

/* y = A x, the X-ray transform of the AIR data term (Methods, Eq. (1): A maps
 * the image X to the projections Y; Materials: the forward projector of
 * ref. [26]), computed as Joseph's ray-driven projector: for each ray, the sum
 * over its driving axis (x if |d_x| >= |d_y|, else y) of the linear
 * interpolation between the two nearest pixels of the other axis, times the
 * step length pixel |d| / |d_drive|.  x [batch][n][n] -> y [batch][V][D], both
 * device, float32, caller-owned.  1 <= batch <= max_batch; x and y must not
 * overlap.  Uses the plan's workspace (calls on one plan must be ordered on one
 * stream). */
air_status air_project(air_plan plan, const float* x, float* y, int32_t batch, hipStream_t stream);

/* y' = C y, C = kappa D^(1/2) R D^(1/2) per view (the plan's window and
 * weighting, see the plan flags; Ram-Lak and D = I by default), kappa =
 * pi / (n_views pixel^2); R acts as a linear convolution truncated to the
 * detector (paper: Methods, Eq. (2): C is a filtration diagonal in Fourier
 * space).  In-place (y == yf) is not allowed. */
air_status air_ramp(air_plan plan, const float* y, float* yf, int32_t batch, hipStream_t stream);

/* x = A'^T y = A^T C y (filter = 1, the filtered adjoint of AIR), or the plain
 * adjoint x = A^T y (filter = 0, the IR arm).  A^T is the matched transpose of
 * air_project, computed per pixel (gather form, no atomics).
 * y [batch][V][D] -> x [batch][n][n]. */
air_status air_filtered_backproject(air_plan plan, const float* y, float* x, int32_t batch,
                                    int32_t filter, hipStream_t stream);

/* out = A^T C A x + mu x (filter = 1) or A^T A x + mu x (filter = 0): the
 * operator of Eq. (5) and of the split Bregman L2 step.  out != x. */
air_status air_normal_apply(air_plan plan, const float* x, float* out, int32_t batch, double mu,
                            int32_t filter, hipStream_t stream);

/* Tensor framelet (Materials): one level, undecimated, periodic boundary,
 * filters h0 = [1,2,1]/4, h1 = sqrt2 [1,0,-1]/4, h2 = [-1,2,-1]/4 (correlation
 * form, taps at offsets -1, 0, +1); band (m_y, m_x) applies h_{m_y} along
 * rows' index j and h_{m_x} along i.
 *   adjoint = 0: out[b][9][n][n] = W in[b][n][n]
 *   adjoint = 1: out[b][n][n] = W^T in[b][9][n][n]       (W^T W = I)
 * Uses no plan workspace (batch is not bounded by max_batch). */
air_status air_framelet(air_plan plan, const float* in, float* out, int32_t batch, int32_t adjoint,
                        hipStream_t stream);

typedef struct {
    double lambda;     /* framelet weight (reg = 0, 2) or L2 weight of Eq. (5) (reg = 1), >= 0 */
    double mu;         /* Bregman penalty (reg = 0) or step of Eq. (6) (reg = 2), > 0; unused for reg = 1 */
    int32_t n_outer;   /* Bregman (reg = 0) or forward-backward (reg = 2) iterations, >= 0 */
    int32_t n_cg;      /* CG steps per L2 sub-problem, >= 0 (unused for reg = 2) */
    int32_t reg;       /* 0 = tensor framelet via split Bregman, 1 = L2 (Eq. (5)),
                          2 = tensor framelet via forward-backward splitting (Eq. (6)) */
    int32_t filter;    /* 1 = AIR (A'^T = A^T C), 0 = IR (A^T) */
} air_solve_params;

/* Device bytes of the solve workspace for `batch` reconstructions. */
air_status air_solve_workspace_size(air_plan plan, int32_t batch, size_t* bytes);

/* Reconstruct `batch` independent images from Y [batch][V][D].
 * X [batch][n][n] holds the start image on entry (zeros for the standard
 * start) and the result on exit.  Split Bregman (reg = 0):
 *   g = A'^T Y;  d = b = 0
 *   n_outer times:  X <- n_cg CG steps on (A'^T A + mu I) X = g + mu W^T (d - b),
 *                   started from X (a fresh CG each time);
 *                   v = W X + b; d = shrink(v, lambda / (2 mu)) on bands 1..8,
 *                   d = v on band 0; b = v - d
 * L2 (reg = 1): n_cg CG steps on (A'^T A + lambda I) X = A'^T Y from X.
 * The residual each CG run starts from, rhs - M X (M the system matrix), is
 * not recomputed with an operator apply: the call computes c = g - M X once
 * for the start image, every CG run's last step carries it forward
 * (c = its recursive residual minus mu W^T (d - b)), and a run starts from
 * c + mu W^T (d - b): equal in exact arithmetic, one apply per outer
 * iteration fewer.
 * Forward-backward splitting (reg = 2; Methods, Eq. (6) and the proximal step):
 *   n_outer times:  X' = X - mu A'^T (A X - Y)
 *                   X  = W^T shrink(W X', mu lambda / 2)   (band 0 passes through)
 *   (the data term's gradient is 2 A'^T (A X - Y), so the step is mu / 2 and the
 *   threshold mu lambda / 2; W^T shrink W stands in for the proximal map of the
 *   tight frame).  Stable for mu < 2 / ||A'^T A||.
 * resid (device, may be NULL) receives [batch][n_outer] float64 ||W X - d||_2
 * (split Bregman) or ||X_new - X_old||_2 (forward-backward).
 * ws: device, >= air_solve_workspace_size(plan, batch) bytes, 256-byte
 * aligned; it is scratch for this call only.  The plan's own workspace is
 * not used, so batch may exceed max_batch.
 * A batch of 8 or more runs as two sub-batches (the first ceil(batch / 2)
 * images, then the rest) on two streams that the plan creates on first use
 * (default priority): they wait on an event recorded on `stream`, and
 * `stream` waits on an event recorded on each, so the call stays ordered on
 * `stream` (and can be captured there).  With kernel timing in
 * AIR_TIMING_ONE_STREAM mode the whole batch runs on `stream`.  Results are
 * the same bits either way.  Calls on one plan must come from one host thread
 * at a time.  Non-finite values are not reported by status here (the call is
 * asynchronous): they show in X and in resid. */
air_status air_solve(air_plan plan, const float* Y, float* X, int32_t batch, const air_solve_params* p,
                     double* resid, void* ws, size_t ws_bytes, hipStream_t stream);

/* air_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no workspace
 * argument, and nothing is allocated (with kernel timing off).  The solve's
 * scratch is a static device array of AIR_NOALLOC_SCRATCH_BYTES in the library,
 * one copy per GPU, held from the library's load on that GPU until the process
 * ends.  The whole batch runs on `stream` (no sub-batch streams, so none is
 * created), with the same kernels as air_solve and the same results, bit for
 * bit.  Every value the solve reads from the scratch it has written first in
 * the same call, so the previous call's contents never matter.
 * Errors: as air_solve, and AIR_E_NOMEM (before any GPU work) if the batch needs
 * more scratch than AIR_NOALLOC_SCRATCH_BYTES (at 512 x 512 with 720 views x 736
 * bins, about 27 MB per image: batches of up to 9).  All calls on one GPU share
 * its copy of the array:
 * calls that overlap on one GPU (different streams or threads without ordering
 * between them) race and corrupt each other's results; order them on one stream. */
#define AIR_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
air_status air_solve_noalloc(air_plan plan, const float* Y, float* X, int32_t batch, const air_solve_params* p,
                             double* resid, hipStream_t stream);

/* ---------------------------------------------------------------------------------
 * Solve slots (continuous batching).  A state holds up to `capacity` split-Bregman
 * reconstructions of one plan's geometry, each with its own sinogram, start image
 * and Bregman iteration count, and all sharing lambda, mu, n_cg and filter.  Every
 * slot keeps X, g = A'^T Y, the Bregman variables b and d - b, its residual
 * history and its counter resident on the device; the CG state is rebuilt every
 * outer iteration.  air_state_step advances all active slots together with the
 * batched kernels; slots can be admitted and retired between steps, so requests
 * that arrive while others run join the next step.  A slot's result is the same
 * bits whatever else is in the state (each image's arithmetic is independent).
 * Steps on a non-default stream replay one HIP graph per number of active slots.
 * The state object lives on the host; its device memory is the caller's `ws`.
 * Calls on one state must be ordered on one stream.
 * --------------------------------------------------------------------------------- */
typedef struct air_state_s* air_state;

/* Device bytes for a state of `capacity` slots; p->reg must be 0 and p->n_outer
 * is the largest Bregman iteration count a slot may ask for. */
air_status air_state_workspace_size(air_plan plan, int32_t capacity, const air_solve_params* p, size_t* bytes);
air_status air_state_create(air_plan plan, int32_t capacity, const air_solve_params* p, void* ws, size_t ws_bytes,
                            air_state* out);
void air_state_destroy(air_state state);
/* Start a reconstruction in a free slot: g = A'^T Y, b = d = 0, X = X0 (device
 * [n][n]) or zeros when X0 is NULL, and the carried residual g - M X (see
 * air_solve; one operator apply when X0 is given).  Y: device [V][D].  n_outer
 * in [1, the state's n_outer].  *slot receives the slot id.  AIR_E_NOMEM if
 * all slots are busy. */
air_status air_state_admit(air_state state, const float* Y, const float* X0, int32_t n_outer, hipStream_t stream,
                           int32_t* slot);
/* Advance every active slot by k = min(max_iters, the fewest iterations any
 * active slot still needs) Bregman iterations; *done_iters (may be NULL) = k. */
air_status air_state_step(air_state state, int32_t max_iters, hipStream_t stream, int32_t* done_iters);
/* Host-side bookkeeping, no GPU call. */
air_status air_state_query(air_state state, int32_t slot, int32_t* iters_done, int32_t* n_outer);
air_status air_state_active(air_state state, int32_t* count);
/* Which slots are finished (active and through all their Bregman iterations),
 * as a host bitmask: bit s % 32 of done_mask[s / 32] for slot s; done_mask has
 * (capacity + 31) / 32 words.  Host-side bookkeeping, no GPU call: the
 * iterations counted are those queued by air_state_step, so a finished slot's
 * last step may still be running (air_state_retire orders its copies after it). */
air_status air_state_poll(air_state state, int32_t* done_mask);
/* Copy the slot's image (device [n][n], may be NULL) and residual history
 * (device [n_outer] float64 ||W X - d||, may be NULL) out, then free the slot.
 * Synchronises `stream` once, to read the slot's residual history on the host:
 * if any of its values is not finite (a non-finite input or a diverged solve),
 * the slot is still copied out and freed, and the call returns AIR_E_NONFINITE. */
air_status air_state_retire(air_state state, int32_t slot, float* X_out, double* resid_out, hipStream_t stream);
/* Checkpoint: the slot's whole continuation state (X, g - M X, b, d - b, residual
 * history, iteration count) to a host buffer of air_state_snapshot_size bytes.
 * The copy is asynchronous: synchronise `stream` before reading the buffer.
 * Restore admits it into a free slot of a state with the same geometry and
 * solver parameters (it synchronises `stream` before returning); continuing
 * gives the same bits as never having stopped. */
air_status air_state_snapshot_size(air_state state, size_t* bytes);
air_status air_state_snapshot(air_state state, int32_t slot, void* host_buf, hipStream_t stream);
air_status air_state_restore(air_state state, const void* host_buf, hipStream_t stream, int32_t* slot);

/* Per-kernel timing (measurement support).  While enabled on a plan, every
 * kernel launch that plan makes (operators and air_solve) is bracketed by a
 * pair of HIP events on the launch stream.  air_kernel_timing_collect waits
 * for the recorded events and adds their elapsed times to *stats, then
 * forgets them.  Kinds index air_kernel_stats' arrays.  Modes:
 *   AIR_TIMING_OFF         no events
 *   AIR_TIMING_ON          events; air_solve keeps its two sub-batch streams, so
 *                          a kernel's time is measured while it shares the GPU
 *                          with the other sub-batch's kernels, as in a plain solve
 *   AIR_TIMING_ONE_STREAM  events, and every air_solve runs on the caller's
 *                          stream: the times of kernels running alone
 * Solve slots do not replay captured graphs while timing is on. */
enum { AIR_TIMING_OFF = 0, AIR_TIMING_ON = 1, AIR_TIMING_ONE_STREAM = 2 };
typedef enum {
    AIR_K_PROJECT = 0,      /* Joseph forward projector */
    AIR_K_BACKPROJECT = 1,  /* gather-form matched backprojector (all epilogues) */
    AIR_K_RAMP = 2,         /* Toeplitz ramp GEMM (MFMA) */
    AIR_K_CG = 3,           /* CG vector updates */
    AIR_K_FRAMELET = 4,     /* framelet, shrink and right-hand side */
    AIR_K_OTHER = 5,        /* padded copies, repacking, fills */
    AIR_K_COUNT = 6
} air_kernel_kind;
typedef struct {
    double ms[AIR_K_COUNT];        /* summed kernel time */
    int64_t launches[AIR_K_COUNT]; /* number of launches */
} air_kernel_stats;
air_status air_kernel_timing_enable(air_plan plan, int32_t mode);
air_status air_kernel_timing_collect(air_plan plan, air_kernel_stats* stats /* host */);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* air_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
