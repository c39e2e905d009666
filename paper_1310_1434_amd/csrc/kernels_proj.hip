// Joseph forward projector, its matched gather-form adjoint, and the padded
// image copies the projector reads.  gfx950, wave64.
//
// Memory layout the projector samples from: every image is kept twice, as
// padded column lines (for x-driven rays, which step over columns and
// interpolate between rows) and padded row lines (for y-driven rays), each
// line with two zero samples at both ends, and the images of a group
// interleaved sample by sample (PadBuf).  A wavefront holds 64 neighbouring
// detector bins of one view; at each driving step they all read the same line
// at nearby positions, so the gathers are coalesced, one gather serves every
// image of the group, and no bounds test is needed in the inner loop.
#include "common.cuh"

namespace air {

// ---------------------------------------------------------------------------- image groups
int image_group(int batch) {
    if (batch <= 1) return 1;
    int best = 1, best_cost = batch * 3;
    for (int g : {2, 4, 8}) {
        const int cost = (batch + g - 1) / g * (2 + g);
        if (cost < best_cost) {
            best = g;
            best_cost = cost;
        }
    }
    return best;
}

int pad_group(int batch) { return batch >= 2 ? 2 : 1; }

// ---------------------------------------------------------------------------- padded copies
template <int P>
__global__ __launch_bounds__(256) void k_pad(const float* __restrict__ x, float* __restrict__ pad, int n, int line,
                                             int batch) {
    __shared__ float lds[16 * 17 * P];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16, b0 = blockIdx.z * P;
    const int i = i0 + tx, j = j0 + ty;
    float v[P];
#pragma unroll
    for (int q = 0; q < P; q++)
        v[q] = (i < n && j < n && b0 + q < batch) ? x[((size_t)(b0 + q) * n + j) * n + i] : 0.f;
    store_padded_group<P, P>(pad + (size_t)b0 * 2 * n * line, n, line, i0, j0, tx, ty, v, lds);
}

hipError_t launch_pad(const KGeom& g, const float* x, PadBuf pad, int batch, hipStream_t s) {
    const int pg = pad_group(batch);
    dim3 grid((g.n + 15) / 16, (g.n + 15) / 16, (batch + pg - 1) / pg), block(256);
    if (pg == 2) hipLaunchKernelGGL(k_pad<2>, grid, block, 0, s, x, pad.base, g.n, g.line, batch);
    else hipLaunchKernelGGL(k_pad<1>, grid, block, 0, s, x, pad.base, g.n, g.line, batch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- forward A
// One thread per ray and pair of images (PadBuf).
//   y[b][v][k] = s * sum_{a=lo..hi} (1-f) L_a[j] + f L_a[j+1],
//   T = tc + (a - c0) m (fixed point), j = T >> kFrac, f = frac(T) as float32,
// L_a the padded line a of image b.  Bins k in [n_bins, ds) are written as zero.
// The driving index runs over the union of the wavefront's ranges, so at every
// step all lanes of one axis read the same image line (coalesced gathers); a
// lane outside its own range samples the zero padding.  The two samples of
// both images of a pair are 4 contiguous floats, read as one 16-byte load.
constexpr int kProjBlock = 256;

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Sample index (high word) and fraction (low word) of a fixed-point intercept.
static_assert(kFrac == 32 && kSlopeFrac == 31, "fixed-point layout");
__device__ __forceinline__ int fx_index(int64_t t) { return (int)(t >> 32); }
__device__ __forceinline__ float fx_frac(int64_t t) { return (float)(uint32_t)t * 0x1p-32f; }
// intercept at driving index a: tc + 2 (a - c0) m, as one 32x32->64 multiply and one shift-add
__device__ __forceinline__ int64_t fx_at(const RayEntry& e, int a_minus_c0) {
    int64_t prod = (int64_t)a_minus_c0 * (int64_t)e.m;
    asm volatile("" : "+v"(prod));      // keep the product 32x32 (no reassociation with the shift)
    return e.tc + prod * 2;
}

// Index of the first of the two samples in a padded line of n + 4: clamping
// into [0, n + 2] only ever moves samples onto the zero padding, so an
// out-of-range step contributes exactly zero (no range test needed).
__device__ __forceinline__ int fx_clamped_index(int64_t t, int n) { return min(max(fx_index(t), 0), n + 2); }

typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef float float4_a8 __attribute__((ext_vector_type(4), aligned(8)));

template <bool SCALED, int P>
__global__ __launch_bounds__(kProjBlock) void k_project(KGeom g, const float* __restrict__ pad,
                                                         float* __restrict__ y, int chunks, int batch) {
    static_assert(P == 1 || P == 2, "images per thread");
    const int v = blockIdx.x / chunks;
    const int k = (blockIdx.x - v * chunks) * kProjBlock + threadIdx.x;
    const int b0 = blockIdx.y * P;
    const bool ray = k < g.n_bins;
    RayEntry e;
    e.tc = 0;
    e.m = 0;
    e.meta = 0;
    if (ray) e = g.rays[(size_t)v * g.n_bins + k];
    const bool hits = ray && ray_hi(e.meta) >= ray_lo(e.meta);
    const int lo = hits ? ray_lo(e.meta) : 0x7fffffff;    // misses do not widen the wave's range
    const int hi = hits ? ray_hi(e.meta) : -1;
    const int axis = ray_axis(e.meta);
    // The union of the wave's ranges, one step wider on each side (the float64
    // range test and the fixed-point intercept may disagree at the very edge).
    const int a_lo = max(0, __builtin_amdgcn_readfirstlane(wave_min_i(lo)) - 1);
    const int a_hi = min(g.n - 1, __builtin_amdgcn_readfirstlane(wave_max_i(hi)) + 1);
    const int line = g.line;
    const float* lines = pad + ((size_t)blockIdx.y * 2 + axis) * g.n * line * P;
    float acc[P];
#pragma unroll
    for (int q = 0; q < P; q++) acc[q] = 0.f;
    int64_t t = fx_at(e, a_lo - g.c0);
    const int64_t m = (int64_t)e.m * 2;
    uint32_t row = (uint32_t)(a_lo * line);
#pragma unroll 4
    for (int a = a_lo; a <= a_hi; a++, t += m, row += line) {
        const float f = fx_frac(t);
        const float* p = lines + (size_t)((row + (uint32_t)fx_clamped_index(t, g.n)) * (uint32_t)P);
        if constexpr (P == 1) {
            const float2_a4 u = *reinterpret_cast<const float2_a4*>(p);
            acc[0] = fmaf(1.f - f, u.x, acc[0]);
            acc[0] = fmaf(f, u.y, acc[0]);
        } else {
            const float4_a8 u = *reinterpret_cast<const float4_a8*>(p);    // [j][0..1], [j + 1][0..1]
            acc[0] = fmaf(1.f - f, u.x, acc[0]);
            acc[0] = fmaf(f, u.z, acc[0]);
            acc[1] = fmaf(1.f - f, u.y, acc[1]);
            acc[1] = fmaf(f, u.w, acc[1]);
        }
    }
    if (k >= g.ds) return;
    const float sv = (SCALED && ray) ? g.step[(size_t)v * g.ds + k] : 1.f;
#pragma unroll
    for (int q = 0; q < P; q++) {
        if (b0 + q >= batch) break;
        float out = 0.f;
        if (ray) out = SCALED ? acc[q] * sv : acc[q];
        y[((size_t)(b0 + q) * g.n_views + v) * g.ds + k] = out;
    }
}

template <bool SCALED>
static void launch_project_g(const KGeom& g, PadBuf pad, float* y, int batch, hipStream_t s) {
    const int chunks = (g.ds + kProjBlock - 1) / kProjBlock;
    const int pg = pad_group(batch);
    dim3 grid(g.n_views * chunks, (batch + pg - 1) / pg), block(kProjBlock);
    if (pg == 2) hipLaunchKernelGGL((k_project<SCALED, 2>), grid, block, 0, s, g, pad.base, y, chunks, batch);
    else hipLaunchKernelGGL((k_project<SCALED, 1>), grid, block, 0, s, g, pad.base, y, chunks, batch);
}

hipError_t launch_project(const KGeom& g, PadBuf pad, float* y, int batch, bool scaled, hipStream_t s) {
    if (scaled) launch_project_g<true>(g, pad, y, batch, s);
    else launch_project_g<false>(g, pad, y, batch, s);
    return hipGetLastError();
}

// out[b / grp][v][k][b % grp] = y[b][v][k] * step[v][k]^power  (power 1: S y, power 2: S^2 y).
__global__ __launch_bounds__(256) void k_scale(KGeom g, const float* __restrict__ y, float* __restrict__ out,
                                               size_t count, int power, int grp) {
    const size_t per_batch = (size_t)g.n_views * g.ds;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
        const size_t b = i / per_batch, vk = i - b * per_batch;
        const float sv = g.step[vk];
        const size_t gi = b / grp;
        out[(gi * per_batch + vk) * grp + (b - gi * grp)] = power == 2 ? y[i] * sv * sv : y[i] * sv;
    }
}

hipError_t launch_scale(const KGeom& g, const float* y, float* out, int batch, int power, int grp, hipStream_t s) {
    const size_t count = (size_t)batch * g.n_views * g.ds;
    const size_t blocks = (count + 255) / 256 < 8192 ? (count + 255) / 256 : 8192;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, s, g, y, out, count, power, grp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- adjoint J^T
// One thread per pixel and up to BT images, 16x16 pixels per block.  For every
// view the pixel finds the bins whose rays can give it a non-zero Joseph
// weight: the detector interval covered by the diamond |dx| + |dy| <= pixel
// around its centre (any sample that touches the pixel lies inside it),
// widened by 0.01 bin.  For each candidate it re-evaluates the forward
// projector's own fixed-point intercept and float32 weight, so the result is
// the exact transpose of k_project (unscaled) up to summation order.
// Candidates are taken two at a time with predication, so that their table
// and sinogram loads are in flight together.  Per view the (few) terms are
// summed in float32, across views in float64.  No atomics.
__device__ __forceinline__ float joseph_weight(const RayEntry& e, int i, int j, int c0) {
    const int ax = ray_axis(e.meta);
    const int da = ax ? j : i;      // driving index of this pixel for the ray
    const int ob = ax ? i : j;      // interpolated index
    const int64_t t = fx_at(e, da - c0);
    const float f = fx_frac(t);
    const int j0 = fx_index(t) - kPad;
    // ob in {j0, j0 + 1} implies -1 <= t < n: exactly the samples the forward
    // projector takes with non-zero weight, so no range test is needed
    return (ob == j0) ? (1.f - f) : ((ob == j0 + 1) ? f : 0.f);
}

template <int MODE, bool REDUCE, int BT>
__global__ __launch_bounds__(256) void k_backproject(KGeom g, const float* __restrict__ y, BpArgs a, int batch) {
    __shared__ float lds[MODE == BP_RESIDUAL ? 16 * 17 * BT : 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const int i = i0 + tx, j = j0 + ty;
    const int b0 = blockIdx.z * BT;
    const int n = g.n;
    const bool valid = i < n && j < n;
    const float px = ((float)i - g.half_n) * g.pixel;
    const float py = ((float)j - g.half_n) * g.pixel;
    // group-interleaved input [group][v][k][BT]: this thread's BT images are
    // contiguous and 4 * BT-byte aligned
    const float* yb = y + (size_t)blockIdx.z * g.n_views * g.ds * BT;
    double tot[BT];
#pragma unroll
    for (int q = 0; q < BT; q++) tot[q] = 0.0;
    if (valid) {
        for (int v = 0; v < g.n_views; v++) {
            const float2 cs = g.views[v];
            const float c = cs.x, s = cs.y;
            float umin, umax;
            if (g.beam == 0) {
                const float uc = fmaf(px, c, py * s);
                const float hw = g.pixel * fmaxf(fabsf(c), fabsf(s));
                umin = uc - hw;
                umax = uc + hw;
            } else {
                const float ap = fmaf(py, c, -px * s);
                const float bp = g.sod - fmaf(px, c, py * s);
                const float ds_ = g.pixel * s, dc = g.pixel * c;
                const float u1 = (ap - ds_) * __builtin_amdgcn_rcpf(bp - dc);
                const float u2 = (ap + ds_) * __builtin_amdgcn_rcpf(bp + dc);
                const float u3 = (ap + dc) * __builtin_amdgcn_rcpf(bp - ds_);
                const float u4 = (ap - dc) * __builtin_amdgcn_rcpf(bp + ds_);
                umin = g.sdd * fminf(fminf(u1, u2), fminf(u3, u4));
                umax = g.sdd * fmaxf(fmaxf(u1, u2), fmaxf(u3, u4));
            }
            const float kmin = fmaf(umin, g.inv_bin, g.half_d) - 0.01f;
            const float kmax = fmaf(umax, g.inv_bin, g.half_d) + 0.01f;
            const int klo = max(0, (int)ceilf(fmaxf(kmin, -1.f)));
            const int khi = min(g.n_bins - 1, (int)floorf(fminf(kmax, (float)g.n_bins)));
            const RayEntry* rv = g.rays + (size_t)v * g.n_bins;
            const float* yv = yb + (size_t)v * g.ds * BT;
            float part[BT];
#pragma unroll
            for (int q = 0; q < BT; q++) part[q] = 0.f;
            for (int k = klo; k <= khi; k += 2) {
                const bool two = k + 1 <= khi;
                const int k1 = two ? k + 1 : k;
                const RayEntry e0 = rv[k], e1 = rv[k1];
                float yv0[BT], yv1[BT];
                load_group<BT>(yv + (size_t)k * BT, yv0);
                load_group<BT>(yv + (size_t)k1 * BT, yv1);
                const float w0 = joseph_weight(e0, i, j, g.c0);
                const float w1 = joseph_weight(e1, i, j, g.c0) * (two ? 1.f : 0.f);
#pragma unroll
                for (int q = 0; q < BT; q++) part[q] = fmaf(w1, yv1[q], fmaf(w0, yv0[q], part[q]));
            }
#pragma unroll
            for (int q = 0; q < BT; q++) tot[q] += (double)part[q];
        }
    }
    const int nblk = gridDim.x * gridDim.y;
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    float rq[BT];     // RESIDUAL: r of every image of the group (0 beyond the batch)
#pragma unroll
    for (int q = 0; q < BT; q++) {
        rq[q] = 0.f;
        const int b = b0 + q;
        if (b >= batch) continue;     // uniform across the block
        const size_t idx = (size_t)b * n * n + (size_t)j * n + i;
        double part = 0.0;
        if (MODE == BP_PLAIN) {
            if (valid) a.out[idx] = (float)tot[q];
        } else if (MODE == BP_MATVEC) {
            if (valid) {
                const float pv = a.aux[idx];
                const float qv = (float)fma((double)a.mu, (double)pv, tot[q]);
                a.out[idx] = qv;
                part = (double)pv * (double)qv;
            }
        } else {  // BP_RESIDUAL
            if (valid) {
                const float xv = a.aux[idx];
                const float r = (float)((double)a.out[idx] - fma((double)a.mu, (double)xv, tot[q]));
                a.out[idx] = r;
                a.p_out[idx] = r;
                rq[q] = r;
                part = (double)r * (double)r;
            }
        }
        if (REDUCE) block_partial<256>(part, a.partial + (size_t)b * nblk + blk);
    }
    if (MODE == BP_RESIDUAL) {
        constexpr int P = BT < 2 ? BT : 2;    // pad_group(batch)
        store_padded_group<BT, P>(a.pad_out.base + (size_t)b0 * 2 * n * g.line, n, g.line, i0, j0, tx, ty, rq, lds);
    }
}

template <int MODE, bool REDUCE>
static void launch_bp_mode(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s) {
    const int bt = image_group(batch);
    dim3 grid((g.n + 15) / 16, (g.n + 15) / 16, (batch + bt - 1) / bt), block(256);
    if (bt == 8) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 8>), grid, block, 0, s, g, y, a, batch);
    else if (bt == 4) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 4>), grid, block, 0, s, g, y, a, batch);
    else if (bt == 2) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 2>), grid, block, 0, s, g, y, a, batch);
    else hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 1>), grid, block, 0, s, g, y, a, batch);
}

hipError_t launch_backproject(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s) {
    const bool red = a.partial != nullptr;
    switch (a.mode) {
    case BP_PLAIN:
        launch_bp_mode<BP_PLAIN, false>(g, y, a, batch, s);
        break;
    case BP_MATVEC:
        if (red) launch_bp_mode<BP_MATVEC, true>(g, y, a, batch, s);
        else launch_bp_mode<BP_MATVEC, false>(g, y, a, batch, s);
        break;
    case BP_RESIDUAL:
        launch_bp_mode<BP_RESIDUAL, true>(g, y, a, batch, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- repack
__global__ __launch_bounds__(256) void k_repack(const float* __restrict__ src, int src_stride,
                                                float* __restrict__ dst, int dst_stride, int rows, int cols,
                                                int dst_cols) {
    const size_t count = (size_t)rows * dst_cols;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
        const size_t r = i / dst_cols;
        const int c = (int)(i - r * dst_cols);
        dst[r * dst_stride + c] = c < cols ? src[r * src_stride + c] : 0.f;
    }
}

hipError_t launch_repack(const float* src, int src_stride, float* dst, int dst_stride, int rows, int cols,
                         int dst_cols, hipStream_t s) {
    const size_t count = (size_t)rows * dst_cols;
    const size_t blocks = (count + 255) / 256 < 8192 ? (count + 255) / 256 : 8192;
    hipLaunchKernelGGL(k_repack, dim3((unsigned)blocks), dim3(256), 0, s, src, src_stride, dst, dst_stride, rows,
                       cols, dst_cols);
    return hipGetLastError();
}

}  // namespace air
