// Internal declarations of the AIR library: plan layout, kernel parameter
// blocks and kernel launchers.  Not part of the ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "air.h"
#include "geometry.h"

namespace air {

struct BpWin;

// Geometry block passed by value to the projector kernels.
struct KGeom {
    int n;          // image side
    int n_views;
    int n_bins;
    int ds;         // sinogram row stride of internal buffers (n_bins rounded up to 32)
    int line;       // padded image line length, n + 2 kPad
    int c0;         // reference driving index of the intercept tables (n / 2)
    int beam;       // 0 parallel, 1 fan
    float pixel;    // mm
    float half_n;   // (n - 1) / 2
    float inv_bin;  // 1 / bin (1/mm)
    float half_d;   // (n_bins - 1) / 2
    float sod, sdd; // fan geometry, mm
    const RayEntry* rays;   // [n_views][n_bins]
    const float* step;      // [n_views][ds] path length per driving step (0 in the padding)
    const float2* views;    // [n_views] (cos, sin) as float
    // Forward-projector block order: [2][v_half] view indices (-1 = none), the
    // views whose rays are mostly x-driven first, then the mostly y-driven ones.
    const int32_t* vorder;
    int v_half;
    float kdet;             // sdd / bin: fan-beam detector bins per unit of ap / bp
    // backprojector windows: [tile][view] over the 16 x 32 pixel tiles, row-major
    // (see BpWin), and the same for horizontal pixel pairs
    const BpWin* bpwin;
    const float2* bpwinx;
};

// Window record of one 16 x 32 pixel tile of the backprojector (two vertically
// adjacent pixels per thread) and one view, built once per plan by
// launch_bp_windows.  The tile stages the bins kb0 .. kb0 + nb - 1; a thread
// whose pixel pair has its midpoint projected to the continuous bin km takes the
// staged slots ceil(km - lo) .. floor(km + hi) (relative to kb0), which hold
// every ray that can give either pixel a non-zero weight.
struct BpWin {
    int32_t kb0;
    int32_t meta;   // bits 0-15: nb; bit 16: some staged ray is x-driven; bit 17: some is y-driven
    float lo, hi;   // kb0 + h and h - kb0, h the window's half-width in bins
};
static_assert(sizeof(BpWin) == 16, "BpWin is read as one 16-byte scalar load");
constexpr int kBpTileW = 16, kBpTileH = 32;
__host__ __device__ inline size_t bp_window_count(int n, int n_views) {
    return (size_t)((n + kBpTileW - 1) / kBpTileW) * ((n + kBpTileH - 1) / kBpTileH) * n_views;
}
// Fills win[bp_window_count] and winx (the same half-widths for horizontal pixel
// pairs, as {lo, hi}) from the geometry and the ray table of g.
hipError_t launch_bp_windows(const KGeom& g, BpWin* win, float2* winx, hipStream_t s);

// Images are processed in groups of image_group(batch) in {1, 2, 4, 8, 16}: the
// group a backprojector thread serves.  The choice minimises
// ceil(batch / G) * (2 + G), i.e. it shares the per-sample index work over as
// many images as possible without too many idle lanes in the last group.
int image_group(int batch);
// Padded image copies of a batch, image-interleaved in pairs:
// [ceil(batch / P)][2][n][line][P] with P = pad_group(batch) (1 for a single
// image, else 2; P divides image_group(batch)); line set 0 = columns (for
// x-driven rays), 1 = rows.  A lane of the last pair beyond the batch holds
// zeros.  A pair keeps the projector's gathers at 16 bytes while the working
// set of one pair of 512^2 images (4 MB) still fits an XCD's L2.
int pad_group(int batch);
// Mixed-precision plans keep the padded copies as float16 instead:
// [ceil(batch / P)][2][n][line][P] halves with P = pad_group16(batch) in
// {1, 2, 4} (four images per 16-byte gather; the same working set as a float32
// pair), image b holding round_to_half(scale[b] * x) with scale[b] a power of
// two chosen from max |x| (so the largest value lands in [2^13, 2^14)).  The
// projector multiplies its float32 sums by 1 / scale[b], exactly.
int pad_group16(int batch);
// Images the grouped buffers (padded copies, backprojector input) must hold for
// any batch up to max_batch: the kernels write whole groups, so the last group's
// idle lanes need room too.
int group_images(int max_batch);
struct PadBuf {
    float* base = nullptr;           // float32 copies, or
    uint16_t* half = nullptr;        // float16 copies (when set)
    float* scale = nullptr;          // [batch] their power-of-two scales
};
// Block partial maxima of |x| per image ([batch][tiles16(n)], as float64), and
// the float16 scale per image from them: 2^(14 - e) with max = m 2^e, m in [0.5, 1)
// (1 if the image is zero or not finite).
hipError_t launch_absmax(int n, const float* x, double* partial, int batch, hipStream_t s);
hipError_t launch_pad_scale(const double* partial, int nblk, int batch, float* scale, hipStream_t s);
hipError_t launch_pad16(const KGeom& g, const float* x, PadBuf pad, int batch, hipStream_t s);

// ---- kernel launchers (kernels_*.hip) -------------------------------------------------
hipError_t launch_pad(const KGeom& g, const float* x, PadBuf pad, int batch, hipStream_t s);
// y = A x = S J x (rows [batch * n_views][ds]; bins past n_bins zero).
hipError_t launch_project(const KGeom& g, PadBuf pad, float* y, int batch, hipStream_t s);
// Backprojector input layout: group-interleaved [ceil(batch / G)][n_views][ds][G]
// with G = image_group(batch), so that the images a backprojector thread serves
// are contiguous and each group is one dense block (sized for roundup(batch, 16)).  Lanes of the last group
// beyond the batch are never written (and their results never stored).
// out (group-interleaved, G = grp) = S y (y: rows [batch * n_views][ds]).
hipError_t launch_scale(const KGeom& g, const float* y, float* out, int batch, int grp, hipStream_t s);

// Backprojection epilogue modes (per pixel, acc = (J^T y)_pixel, J the bare
// interpolation weights; callers fold the path lengths into y, which is in the
// group-interleaved layout with G = image_group(batch)):
enum BpMode {
    BP_PLAIN = 0,     // out = acc
    BP_MATVEC = 1,    // out = acc + mu * p;  partial sums of p . out (float64)
    BP_RESIDUAL = 2,  // r = rhs - (acc + mu * x) (rhs read from `out`, r written there);
                      // p = r, padded copy of p; partial sums of r . r
    BP_STEP = 3,      // out = x + mu * (rhs - acc): the forward step of Eq. (6), rhs = A'^T Y
};
struct BpArgs {
    int mode;
    float mu;
    const float* aux;   // p (MATVEC) or x (RESIDUAL, STEP)
    const float* rhs;   // STEP: A'^T Y
    float* out;         // [batch][n][n]
    float* p_out;       // RESIDUAL: p
    PadBuf pad_out;     // RESIDUAL: padded copy of p
    double* partial;    // [batch][bp_blocks(n, batch)] block partial sums, or null (MATVEC only)
};
hipError_t launch_backproject(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s);
// Blocks per image of the backprojector (16 x 16 PIX pixel tiles, PIX depends on
// the batch): its partial sums per image.
int bp_blocks(int n, int batch);

// Sinogram repacking between the public [V][D] layout and internal [V][ds] rows.
hipError_t launch_repack(const float* src, int src_stride, float* dst, int dst_stride, int rows, int cols,
                         int dst_cols, hipStream_t s);

// Ramp filtration y' = C y over rows of stride ds (internal layout).
struct RampTables {
    const float* taps32;       // [2 ds] kappa r(m) at index m + ds
    const float* step;         // [n_views][ds] path lengths (for the scaled variants)
    int n_views;
    // 16-bit split terms of T(d) = r(|d|) 2^12 (f16: hi, lo 2^11; bf16: three
    // terms), as [term][shift s < 4][j < tab_j] entries of 4 values
    // T(4 j + s + i - kRampZero - ds), i < 4 (zero outside |d| < n_bins)
    const uint2* tab16;
    int n_terms, tab_j;
    float out_scale;           // kappa * 2^-12 for the 16-bit modes
    const float* wsq;          // [ds] D^(1/2) of a cosine-weighted C (applied before and after R), or null
    // float16 split only: [rows] scratch for a power-of-two scale per input row
    // (b * n_views + v), chosen from the row's max |y| so that the split terms
    // neither overflow nor fall into the float16 subnormal range; null = no
    // scaling (the float32 and bfloat16 modes, whose range is float32's)
    float* rscale;
};
// scale: 0 = C y;  RAMP_POST = S C y  (S = diag(step); the projector's output
// is already S J x, so S C S J x is RAMP_POST applied to it).
// Input rows [batch * n_views][ds].  Output: the same layout when grp == 0, else
// group-interleaved with G = grp (the backprojector's input).
enum { RAMP_POST = 2 };
// Zero entries below the 16-bit tables' index 0 (columns of a last, partial
// column tile past ds read them; up to 128 columns per tile).
constexpr int kRampZero = 128;
inline int ramp_tab_j(int ds) { return (2 * ds + kRampZero + 3) / 4 + 1; }
hipError_t launch_ramp(int prec, const RampTables& t, const float* y, float* yf, int rows, int ds, int scale,
                       int grp, hipStream_t s);

// CG vector updates on 16x16 tiles (float32 vectors, float64 scalars).
struct CgArgs {
    int n;
    float* x; float* r; float* p; const float* q;
    PadBuf pad;                 // padded copy of p (update_p)
    const double* alpha;        // [batch] (update_xr)
    const double* beta;         // [batch] (update_p)
    double* partial;            // [batch][tiles16(n)] partial sums of r . r (update_xr)
    float* rmax;                // or null: [batch][tiles16(n)] per-tile max |r| (update_xr)
    float* pmax;                // or null: [batch][tiles16(n)] per-tile max |p| (update_p)
    float* c;                   // in: W^T e (with framelet); out: carried residual g - M x (update_xc)
    bool framelet;              // split Bregman: subtract mu W^T e (update_xc)
    float mu;                   // (update_xc)
};
hipError_t launch_cg_update_xr(const CgArgs& a, int batch, hipStream_t s);   // x += a p, r -= a q; partials of r.r
// p = r + b p (p = r if !beta), and its pad (float16 copies scaled by pad.scale,
// which must hold the scales k_finalize derived for this p)
hipError_t launch_cg_update_p(const CgArgs& a, int batch, hipStream_t s);
// last CG step: x += a p, c = (r - a q) - mu W^T e, W^T e read from c (no partials)
hipError_t launch_cg_update_xc(const CgArgs& a, int batch, hipStream_t s);
// start of an L2 sub-problem: r = c + mu W^T e (r = c if e is null), then W^T e
// written over c (if e); partials of r.r, and per-tile max |r| if rmax
hipError_t launch_cg_start(int n, float* c, const float* e, float mu, float* r, double* partial, float* rmax,
                           int batch, hipStream_t s);

// Fixed-order sums of the block partials [batch][nblk] and the scalars derived from them:
enum FinalizeMode {
    FIN_RHO = 0,    // rho[b] = sum                                    (initial residual)
    FIN_ALPHA = 1,  // pq = sum; alpha[b] = rho / pq (0 if either is 0)
    FIN_BETA = 2,   // rho' = sum; beta[b] = rho' / rho (0 if rho is 0); rho[b] = rho'
    FIN_RESID = 3,  // out[b * stride + k] = sqrt(sum), k = iters[b]++ (k = 0 if iters is null)
};
// With scale (FIN_RHO, FIN_BETA only): also scale[b], the power-of-two scale
// of the float16 copies of the next CG direction, from the bound
// max |r| + beta max |p_old| (rmax, pmax: [batch][nblk] block maxima; pmax
// unused for FIN_RHO, where p = r).
struct HalfScaleArgs {
    const float* rmax = nullptr;
    const float* pmax = nullptr;
    float* scale = nullptr;
};
hipError_t launch_finalize(int mode, const double* partial, int nblk, int batch, double* rho, double* coef,
                           double* out, int stride, int* iters, hipStream_t s,
                           const HalfScaleArgs& sc = HalfScaleArgs{});

// Framelet kernels.
hipError_t launch_framelet_fwd(int n, const float* x, float* z, int batch, hipStream_t s);
hipError_t launch_framelet_adj(int n, const float* z, float* x, int batch, hipStream_t s);
// v = W x + b (bands 1..8 of b), d = shrink(v, thr) (band 0: d = v), b <- v - d, e <- d - b;
// partial sums of ||W x - d||^2.
struct TfArgs {
    int n;
    const float* x;
    float* bb;          // [batch][8][n][n]
    float* e;           // [batch][9][n][n]
    float thr;
    double* partial;    // [batch][tiles16(n)]
};
hipError_t launch_tf_shrink(const TfArgs& a, int batch, hipStream_t s);
// Proximal step of forward-backward splitting: e = shrink(W x, thr) on bands
// 1..8 (band 0 passes through), then x_new = W^T e written over bb (= the
// iterate X) with partial sums of (x_new - X)^2.  TfArgs: x = the forward-step
// image, e = 9 band scratch, bb = X (in/out), thr = mu lambda / 2.
hipError_t launch_fbs_shrink(const TfArgs& a, int batch, hipStream_t s);
hipError_t launch_fbs_adjoint(const TfArgs& a, int batch, hipStream_t s);
hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s);

// Number of 16x16 tiles of an n x n image (blocks per batch item of tile kernels).
inline int tiles16(int n) { return ((n + 15) / 16) * ((n + 15) / 16); }

}  // namespace air
