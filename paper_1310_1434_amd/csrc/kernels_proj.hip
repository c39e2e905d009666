// Joseph forward projector, its matched gather-form adjoint, and the padded
// image copies the projector reads.  gfx950, wave64.
//
// Memory layout the projector samples from: every image is kept twice, as
// padded column lines (for x-driven rays, which step over columns and
// interpolate between rows) and padded row lines (for y-driven rays), each
// line with two zero samples at both ends.  A wavefront holds 64 neighbouring
// detector bins of one view; at each driving step they all read the same line
// at nearby positions, so the gathers are coalesced and no bounds test is
// needed in the inner loop.
#include "common.cuh"

namespace air {

// ---------------------------------------------------------------------------- padded copies
__global__ __launch_bounds__(256) void k_pad(const float* __restrict__ x, float* __restrict__ pad, int n,
                                             int line) {
    __shared__ float tile[32][33];
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    const float* xb = x + (size_t)b * n * n;
    float* cols = pad + (size_t)b * 2 * n * line;
    float* rows = cols + (size_t)n * line;
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + tx;
        const float v = (j < n && i < n) ? xb[(size_t)j * n + i] : 0.f;
        tile[r][tx] = v;
        if (j < n && i < n) rows[(size_t)j * line + kPad + i] = v;
        if (j < n && tx < kPad) {
            if (i0 == 0) rows[(size_t)j * line + tx] = 0.f;
            if (i0 + 32 >= n) rows[(size_t)j * line + kPad + n + tx] = 0.f;
        }
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        if (i < n && j < n) cols[(size_t)i * line + kPad + j] = tile[tx][r];
        if (i < n && tx < kPad) {
            if (j0 == 0) cols[(size_t)i * line + tx] = 0.f;
            if (j0 + 32 >= n) cols[(size_t)i * line + kPad + n + tx] = 0.f;
        }
    }
}

hipError_t launch_pad(const KGeom& g, const float* x, PadBuf pad, int batch, hipStream_t s) {
    dim3 grid((g.n + 31) / 32, (g.n + 31) / 32, batch), block(32, 8);
    hipLaunchKernelGGL(k_pad, grid, block, 0, s, x, pad.base, g.n, g.line);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- forward A
// One thread per ray.  y[b][v][k] = s * sum_{a=lo..hi} (1-f) L_a[j0] + f L_a[j0+1],
// t = fmaf(a - c0, m, tc), j0 = floor(t), f = t - j0, L_a the padded line a.
// Bins k in [n_bins, ds) of the internal row stride are written as zero.
constexpr int kProjBlock = 256;

__global__ __launch_bounds__(kProjBlock) void k_project(KGeom g, const float* __restrict__ pad,
                                                         float* __restrict__ y, int chunks) {
    const int v = blockIdx.x / chunks;
    const int k = (blockIdx.x - v * chunks) * kProjBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (k >= g.ds) return;
    float* yrow = y + ((size_t)b * g.n_views + v) * g.ds;
    if (k >= g.n_bins) {
        yrow[k] = 0.f;
        return;
    }
    const RayEntry e = g.rays[(size_t)v * g.n_bins + k];
    const int lo = ray_lo(e.meta), hi = ray_hi(e.meta), axis = ray_axis(e.meta);
    const float* lines = pad + ((size_t)b * 2 + axis) * g.n * g.line + kPad;
    const int line = g.line;
    float acc0 = 0.f, acc1 = 0.f;
    float fa = (float)(lo - g.c0);
    int a = lo;
    for (; a + 1 <= hi; a += 2, fa += 2.f) {
        const float t0 = fmaf(fa, e.m, e.tc);
        const float t1 = fmaf(fa + 1.f, e.m, e.tc);
        const float fl0 = floorf(t0), fl1 = floorf(t1);
        const float f0 = t0 - fl0, f1 = t1 - fl1;
        const float* p0 = lines + (size_t)a * line + (int)fl0;
        const float* p1 = lines + (size_t)(a + 1) * line + (int)fl1;
        const float u0 = p0[0], u1 = p0[1], w0 = p1[0], w1 = p1[1];
        acc0 = fmaf(1.f - f0, u0, acc0);
        acc0 = fmaf(f0, u1, acc0);
        acc1 = fmaf(1.f - f1, w0, acc1);
        acc1 = fmaf(f1, w1, acc1);
    }
    if (a <= hi) {
        const float t0 = fmaf(fa, e.m, e.tc);
        const float fl0 = floorf(t0);
        const float f0 = t0 - fl0;
        const float* p0 = lines + (size_t)a * line + (int)fl0;
        acc0 = fmaf(1.f - f0, p0[0], acc0);
        acc0 = fmaf(f0, p0[1], acc0);
    }
    yrow[k] = (acc0 + acc1) * e.s;
}

hipError_t launch_project(const KGeom& g, PadBuf pad, float* y, int batch, hipStream_t s) {
    const int chunks = (g.ds + kProjBlock - 1) / kProjBlock;
    dim3 grid(g.n_views * chunks, batch);
    hipLaunchKernelGGL(k_project, grid, dim3(kProjBlock), 0, s, g, pad.base, y, chunks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- adjoint A^T
// One thread per pixel, 16x16 pixels per block.  For every view the pixel
// finds the bins whose rays can give it a non-zero Joseph weight: the
// detector interval covered by the diamond |dx| + |dy| <= pixel around its
// centre (any sample that touches the pixel lies inside it), widened by 0.01
// bin.  For each candidate it re-evaluates the forward projector's own
// float32 intercept and weight, so the result is the transpose of
// k_project up to summation order.  No atomics.
template <int MODE, bool REDUCE>
__global__ __launch_bounds__(256) void k_backproject(KGeom g, const float* __restrict__ y, BpArgs a) {
    __shared__ float tile[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const int i = i0 + tx, j = j0 + ty;
    const int b = blockIdx.z;
    const int n = g.n;
    const bool valid = i < n && j < n;
    const float px = ((float)i - g.half_n) * g.pixel;
    const float py = ((float)j - g.half_n) * g.pixel;
    const float* yb = y + (size_t)b * g.n_views * g.ds;
    float acc = 0.f;
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
                const float u1 = (ap - ds_) / (bp - dc);
                const float u2 = (ap + ds_) / (bp + dc);
                const float u3 = (ap + dc) / (bp - ds_);
                const float u4 = (ap - dc) / (bp + ds_);
                umin = g.sdd * fminf(fminf(u1, u2), fminf(u3, u4));
                umax = g.sdd * fmaxf(fmaxf(u1, u2), fmaxf(u3, u4));
            }
            const float kmin = fmaf(umin, g.inv_bin, g.half_d) - 0.01f;
            const float kmax = fmaf(umax, g.inv_bin, g.half_d) + 0.01f;
            const int klo = max(0, (int)ceilf(fmaxf(kmin, -1.f)));
            const int khi = min(g.n_bins - 1, (int)floorf(fminf(kmax, (float)g.n_bins)));
            const RayEntry* rv = g.rays + (size_t)v * g.n_bins;
            const float* yv = yb + (size_t)v * g.ds;
            for (int k = klo; k <= khi; k++) {
                const RayEntry e = rv[k];
                const int ax = ray_axis(e.meta);
                const int da = ax ? j : i;      // driving index of this pixel for the ray
                const int ob = ax ? i : j;      // interpolated index
                if (da < ray_lo(e.meta) || da > ray_hi(e.meta)) continue;
                const float t = fmaf((float)(da - g.c0), e.m, e.tc);
                const float fl = floorf(t);
                const float f = t - fl;
                const int j0r = (int)fl;
                const float w = (ob == j0r) ? (1.f - f) : ((ob == j0r + 1) ? f : 0.f);
                acc = fmaf(w, e.s * yv[k], acc);
            }
        }
    }
    const size_t idx = (size_t)b * n * n + (size_t)j * n + i;
    double part = 0.0;
    if (MODE == BP_PLAIN) {
        if (valid) a.out[idx] = acc;
    } else if (MODE == BP_MATVEC) {
        if (valid) {
            const float pv = a.aux[idx];
            const float q = fmaf(a.mu, pv, acc);
            a.out[idx] = q;
            part = (double)pv * (double)q;
        }
    } else {  // BP_RESIDUAL
        float r = 0.f;
        if (valid) {
            const float xv = a.aux[idx];
            r = a.out[idx] - fmaf(a.mu, xv, acc);
            a.out[idx] = r;
            a.p_out[idx] = r;
            part = (double)r * (double)r;
        }
        store_padded_tile(a.pad_out.base + (size_t)b * 2 * n * g.line, n, g.line, i0, j0, tx, ty, r, tile);
    }
    if (REDUCE) {
        const int nblk = gridDim.x * gridDim.y;
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        block_reduce_last<256>(part, a.red_partial + (size_t)b * nblk, a.red_count + b, a.red_out + b, nblk, blk);
    }
}

hipError_t launch_backproject(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s) {
    dim3 grid((g.n + 15) / 16, (g.n + 15) / 16, batch), block(256);
    const bool red = a.red_partial != nullptr;
    switch (a.mode) {
    case BP_PLAIN:
        hipLaunchKernelGGL((k_backproject<BP_PLAIN, false>), grid, block, 0, s, g, y, a);
        break;
    case BP_MATVEC:
        if (red) hipLaunchKernelGGL((k_backproject<BP_MATVEC, true>), grid, block, 0, s, g, y, a);
        else hipLaunchKernelGGL((k_backproject<BP_MATVEC, false>), grid, block, 0, s, g, y, a);
        break;
    case BP_RESIDUAL:
        hipLaunchKernelGGL((k_backproject<BP_RESIDUAL, true>), grid, block, 0, s, g, y, a);
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
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (r >= rows || c >= dst_cols) return;
    dst[(size_t)r * dst_stride + c] = c < cols ? src[(size_t)r * src_stride + c] : 0.f;
}

hipError_t launch_repack(const float* src, int src_stride, float* dst, int dst_stride, int rows, int cols,
                         int dst_cols, hipStream_t s) {
    dim3 grid((dst_cols + 255) / 256, rows);
    hipLaunchKernelGGL(k_repack, grid, dim3(256), 0, s, src, src_stride, dst, dst_stride, rows, cols, dst_cols);
    return hipGetLastError();
}

}  // namespace air
