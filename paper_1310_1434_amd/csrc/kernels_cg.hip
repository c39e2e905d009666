// Conjugate-gradient vector updates and the tensor-framelet kernels.
//
// All image kernels work on 16 x 16 pixel tiles (256 threads), one batch item
// per grid z.  Vectors are float32; inner products, alpha, beta and the
// Bregman residual norm are float64.  Each block writes one partial sum;
// k_finalize adds them in index order (one block per batch item) and derives
// alpha or beta, so every batch item gets the same bits whatever the batch
// size, and no atomics are used.  Scalars never leave the device.
#include "common.h"

namespace air {

// ---------------------------------------------------------------------------- CG
// x += alpha p, r -= alpha q; partial sums of r . r.
__global__ __launch_bounds__(256) void k_cg_xr(CgArgs a) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16, b = blockIdx.z;
    const int n = a.n, i = i0 + tx, j = j0 + ty;
    const double alpha = a.alpha[b];
    const size_t idx = (size_t)b * n * n + (size_t)j * n + i;
    double part = 0.0;
    float rn = 0.f;
    if (i < n && j < n) {
        const float xn = (float)fma(alpha, (double)a.p[idx], (double)a.x[idx]);
        rn = (float)fma(-alpha, (double)a.q[idx], (double)a.r[idx]);
        a.x[idx] = xn;
        a.r[idx] = rn;
        part = (double)rn * (double)rn;
    }
    const int nblk = gridDim.x * gridDim.y, blk = (j0 / 16) * gridDim.x + i0 / 16;
    block_partial<256>(part, a.partial + (size_t)b * nblk + blk);
    if (a.rmax) block_max<256>(fabsf(rn), a.rmax + (size_t)b * nblk + blk);
}

// p = r + beta p (p = r without beta) for a group of G images; p also goes to
// its padded line sets (float16 ones scaled by the image's scale, which
// k_finalize derived from a bound on max |p|), and the block's max |p| of each
// image to pmax (the next bound needs it).
template <int G>
__global__ __launch_bounds__(256) void k_cg_p(CgArgs a, int batch) {
    __shared__ float lds[16 * 17 * G];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16, b0 = blockIdx.z * G;
    const int n = a.n, i = i0 + tx, j = j0 + ty;
    const bool valid = i < n && j < n;
    float pn[G];
#pragma unroll
    for (int q = 0; q < G; q++) {
        pn[q] = 0.f;
        const int b = b0 + q;
        if (valid && b < batch) {
            const size_t idx = (size_t)b * n * n + (size_t)j * n + i;
            // (no beta: the first direction of a CG run, p = r)
            pn[q] = a.beta ? (float)fma(a.beta[b], (double)a.p[idx], (double)a.r[idx]) : a.r[idx];
            a.p[idx] = pn[q];
        }
    }
    if (a.pmax) {
        // the block's max |p| of each image, reduced for all G at once
        __shared__ float mx[4][G];
        float m[G];
#pragma unroll
        for (int q = 0; q < G; q++) {
            m[q] = fabsf(pn[q]);
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) m[q] = fmaxf(m[q], __shfl_xor(m[q], off, kWave));
        }
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q < G; q++) mx[threadIdx.x >> 6][q] = m[q];
        __syncthreads();
        if (threadIdx.x < G && b0 + (int)threadIdx.x < batch) {
            const int q = threadIdx.x, nblk = gridDim.x * gridDim.y, blk = blockIdx.y * gridDim.x + blockIdx.x;
            a.pmax[(size_t)(b0 + q) * nblk + blk] = fmaxf(fmaxf(mx[0][q], mx[1][q]), fmaxf(mx[2][q], mx[3][q]));
        }
    }
    const int line = n + 2 * kPad;
    if (a.pad.half) {
        constexpr int P = G < 4 ? G : 4;    // pad_group16(batch)
        float h[G];
#pragma unroll
        for (int q = 0; q < G; q++) h[q] = b0 + q < batch ? pn[q] * a.pad.scale[b0 + q] : 0.f;   // (exact: 2^k)
        store_padded_group<G, P>(a.pad.half + (size_t)b0 * 2 * n * line, n, line, i0, j0, tx, ty, h, lds);
    } else if (a.pad.base) {
        constexpr int P = G < 2 ? G : 2;    // pad_group(batch)
        store_padded_group<G, P>(a.pad.base + (size_t)b0 * 2 * n * line, n, line, i0, j0, tx, ty, pn, lds);
    }
}

hipError_t launch_cg_update_xr(const CgArgs& a, int batch, hipStream_t s) {
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, batch);
    hipLaunchKernelGGL(k_cg_xr, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cg_update_p(const CgArgs& a, int batch, hipStream_t s) {
    const int grp = image_group(batch);
    // (the kernel writes float16 copies in sub-groups of min(G, 4) images)
    if (a.pad.half && (std::min(grp, 4) != pad_group16(batch) || !a.pad.scale)) return hipErrorInvalidValue;
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, (batch + grp - 1) / grp), block(256);
    if (grp == 16) hipLaunchKernelGGL(k_cg_p<16>, grid, block, 0, s, a, batch);
    else if (grp == 8) hipLaunchKernelGGL(k_cg_p<8>, grid, block, 0, s, a, batch);
    else if (grp == 4) hipLaunchKernelGGL(k_cg_p<4>, grid, block, 0, s, a, batch);
    else if (grp == 2) hipLaunchKernelGGL(k_cg_p<2>, grid, block, 0, s, a, batch);
    else hipLaunchKernelGGL(k_cg_p<1>, grid, block, 0, s, a, batch);
    return hipGetLastError();
}

// One block per batch item: sum the block partials in index order (each
// thread a fixed stride, then a fixed tree) and derive the CG scalar.
// With sc.scale (FIN_RHO, FIN_BETA), also the scale of the float16 copies of
// the direction p = r + beta p that k_cg_p builds next: from the bound
// max |r| + beta max |p_old| on max |p| (max |r| for p = r), over the block
// maxima sc.rmax and sc.pmax ([batch][nblk]), as in k_pad_scale.
__global__ __launch_bounds__(256) void k_finalize(int mode, const double* __restrict__ partial, int nblk,
                                                  double* __restrict__ rho, double* __restrict__ coef,
                                                  double* __restrict__ out, int stride, int* __restrict__ iters,
                                                  HalfScaleArgs sc) {
    __shared__ double sh[4];
    __shared__ float shm[2][4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* pb = partial + (size_t)b * nblk;
    double s = 0.0;
    for (int i = tid; i < nblk; i += 256) s += pb[i];
    s = wave_sum(s);
    if (tid % kWave == 0) sh[tid / kWave] = s;
    if (sc.scale) {     // (uniform)
        float mr = 0.f, mp = 0.f;
        for (int i = tid; i < nblk; i += 256) {
            mr = fmaxf(mr, sc.rmax[(size_t)b * nblk + i]);
            if (mode == FIN_BETA) mp = fmaxf(mp, sc.pmax[(size_t)b * nblk + i]);
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            mr = fmaxf(mr, __shfl_xor(mr, off, kWave));
            mp = fmaxf(mp, __shfl_xor(mp, off, kWave));
        }
        if (tid % kWave == 0) {
            shm[0][tid / kWave] = mr;
            shm[1][tid / kWave] = mp;
        }
    }
    __syncthreads();
    if (tid != 0) return;
    const double sum = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    double bound = 0.0;
    if (sc.scale) bound = fmaxf(fmaxf(shm[0][0], shm[0][1]), fmaxf(shm[0][2], shm[0][3]));
    switch (mode) {
    case FIN_RHO:
        rho[b] = sum;
        break;
    case FIN_ALPHA: {
        const double r = rho[b];
        coef[b] = (r == 0.0 || sum == 0.0) ? 0.0 : r / sum;
        break;
    }
    case FIN_BETA: {
        const double r = rho[b];
        coef[b] = r == 0.0 ? 0.0 : sum / r;
        rho[b] = sum;
        if (sc.scale)
            bound += coef[b] * (double)fmaxf(fmaxf(shm[1][0], shm[1][1]), fmaxf(shm[1][2], shm[1][3]));
        break;
    }
    default: {
        const int k = iters ? iters[b] : 0;
        out[(size_t)b * stride + k] = sqrt(sum);
        if (iters) iters[b] = k + 1;
    }
    }
    if (sc.scale) {
        // |p| <= max |r| + beta max |p_old| up to one rounding (|p| (1 + 2^-24)),
        // so p's scaled copy stays below 2^14 (1 + 2^-24), far from float16's
        // overflow; the bound is at most twice max |p|, which only moves values
        // below 2^-26 max |p| into float16's subnormal range
        float sv = 1.f;
        if (bound > 0.0 && isfinite(bound)) {
            int e;
            frexp(bound, &e);                                // bound = f 2^e, f in [0.5, 1)
            sv = ldexpf(1.f, min(max(14 - e, -126), 126));   // bound * s in [2^13, 2^14)
        }
        sc.scale[b] = sv;
    }
}

hipError_t launch_finalize(int mode, const double* partial, int nblk, int batch, double* rho, double* coef,
                           double* out, int stride, int* iters, hipStream_t s, const HalfScaleArgs& sc) {
    if (sc.scale && (mode != FIN_RHO && mode != FIN_BETA)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_finalize, dim3(batch), dim3(256), 0, s, mode, partial, nblk, rho, coef, out, stride, iters,
                       sc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- framelet
// Piecewise-linear filters at offsets -1, 0, +1 (correlation form):
//   h0 = [1, 2, 1] / 4,  h1 = sqrt2 [1, 0, -1] / 4,  h2 = [-1, 2, -1] / 4.
__device__ __forceinline__ float fl_h(int m, int off) {
    const float q = 0.35355339059327373f;   // sqrt(2) / 4
    if (m == 0) return off == 0 ? 0.5f : 0.25f;
    if (m == 1) return off == 0 ? 0.f : (off < 0 ? q : -q);
    return off == 0 ? 0.5f : -0.25f;
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// The 16x16 tile of a framelet block.  Blocks reach the eight XCDs round-robin;
// when the tile grid divides into eight, block L works on tile (L mod 8) T/8 +
// L/8 (T tiles, row-major), so each XCD covers one contiguous band of tile rows
// and the halo rows and cache lines that neighbouring tiles share stay in its
// L2.  The block's partial sum keeps the tile's own index.
__device__ __forceinline__ void framelet_tile(int& i0, int& j0) {
    const int gx = gridDim.x, T = gx * gridDim.y;
    int t = blockIdx.y * gx + blockIdx.x;
    if (T % 8 == 0) t = (t % 8) * (T / 8) + t / 8;
    i0 = (t % gx) * 16;
    j0 = (t / gx) * 16;
}

// All nine bands of W x at pixel (i, j), periodic boundary.
__device__ __forceinline__ void framelet_at(const float* __restrict__ xb, int n, int i, int j, float z[9]) {
    float rowf[3][3];   // [dy][m_x]: filtered along x
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
        const float* row = xb + (size_t)wrap(j + dy, n) * n;
        const float l = row[wrap(i - 1, n)], c = row[i], r = row[wrap(i + 1, n)];
#pragma unroll
        for (int mx = 0; mx < 3; mx++) rowf[dy + 1][mx] = fl_h(mx, -1) * l + fl_h(mx, 0) * c + fl_h(mx, 1) * r;
    }
#pragma unroll
    for (int my = 0; my < 3; my++)
#pragma unroll
        for (int mx = 0; mx < 3; mx++)
            z[3 * my + mx] = fl_h(my, -1) * rowf[0][mx] + fl_h(my, 0) * rowf[1][mx] + fl_h(my, 1) * rowf[2][mx];
}

// (W^T z)(i, j) = sum_band sum_{dy,dx} h_{my}(dy) h_{mx}(dx) z_band(j - dy, i - dx).
// The 3 x 3 neighbourhood is addressed by 32-bit byte offsets from the bands'
// (uniform) bases (n <= 16384, so n^2 floats span less than 2^32 bytes), and
// the terms whose filter tap is zero are left out (adding 0 * z changes no
// finite sum).
__device__ __forceinline__ float framelet_adj_at(const float* __restrict__ zb, int n, int i, int j) {
    const size_t np = (size_t)n * n;
    uint32_t off[3][3];
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
        const uint32_t ro = (uint32_t)wrap(j - dy, n) * (uint32_t)n;
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) off[dy + 1][dx + 1] = (ro + (uint32_t)wrap(i - dx, n)) * 4u;
    }
    float s = 0.f;
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
#pragma unroll
            for (int my = 0; my < 3; my++) {
                if (fl_h(my, dy) == 0.f) continue;
                float t = 0.f;
#pragma unroll
                for (int mx = 0; mx < 3; mx++) {
                    if (fl_h(mx, dx) == 0.f) continue;
                    const char* band = reinterpret_cast<const char*>(zb + (3 * my + mx) * np);
                    t = fmaf(fl_h(mx, dx), *reinterpret_cast<const float*>(band + off[dy + 1][dx + 1]), t);
                }
                s = fmaf(fl_h(my, dy), t, s);
            }
        }
    }
    return s;
}

__global__ __launch_bounds__(256) void k_framelet_fwd(const float* __restrict__ x, float* __restrict__ z, int n) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    if (i >= n || j >= n) return;
    const size_t np = (size_t)n * n;
    float zz[9];
    framelet_at(x + b * np, n, i, j, zz);
#pragma unroll
    for (int band = 0; band < 9; band++) z[(size_t)b * 9 * np + band * np + (size_t)j * n + i] = zz[band];
}

__global__ __launch_bounds__(256) void k_framelet_adj(const float* __restrict__ z, float* __restrict__ x, int n) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    if (i >= n || j >= n) return;
    const size_t np = (size_t)n * n;
    x[b * np + (size_t)j * n + i] = framelet_adj_at(z + (size_t)b * 9 * np, n, i, j);
}

// Start residual of an L2 sub-problem: r = c + mu W^T e (r = c without e),
// where c = g - M x carries the data part of the residual from the previous
// sub-problem (M = A'^T A + mu I); partial sums of r . r.  With e, W^T e then
// takes c's place (in ct: c is not read again before the sub-problem's last
// CG step writes the next c there, and that step needs W^T e).
__global__ __launch_bounds__(256) void k_cg_start(float* __restrict__ ct, const float* __restrict__ e, float mu,
                                                  float* __restrict__ r, double* __restrict__ partial,
                                                  float* __restrict__ rmax, int n) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    const size_t np = (size_t)n * n;
    double part = 0.0;
    float rv = 0.f;
    if (i < n && j < n) {
        const size_t idx = b * np + (size_t)j * n + i;
        rv = ct[idx];
        if (e) {
            const float adj = framelet_adj_at(e + (size_t)b * 9 * np, n, i, j);
            rv = fmaf(mu, adj, rv);
            ct[idx] = adj;
        }
        r[idx] = rv;
        part = (double)rv * (double)rv;
    }
    const int nblk = gridDim.x * gridDim.y, blk = (j0 / 16) * gridDim.x + i0 / 16;
    block_partial<256>(part, partial + (size_t)b * nblk + blk);
    if (rmax) block_max<256>(fabsf(rv), rmax + (size_t)b * nblk + blk);
}

// Last CG step of an L2 sub-problem: x += alpha p, and instead of r the carried
// part c = (r - alpha q) - mu W^T e (c = r - alpha q without e; W^T e is what
// k_cg_start left in c's place).  r - alpha q is the step's recursive residual
// g + mu W^T e - M x, so c = g - M x for the new x up to rounding, and the next
// sub-problem starts from c + mu W^T e'.
__global__ __launch_bounds__(256) void k_cg_xc(CgArgs a) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15), j = blockIdx.y * 16 + (threadIdx.x >> 4), b = blockIdx.z;
    const int n = a.n;
    if (i >= n || j >= n) return;
    const size_t idx = b * (size_t)n * n + (size_t)j * n + i;
    const double alpha = a.alpha[b];
    const float xn = (float)fma(alpha, (double)a.p[idx], (double)a.x[idx]);
    const float rn = (float)fma(-alpha, (double)a.q[idx], (double)a.r[idx]);
    a.x[idx] = xn;
    a.c[idx] = a.framelet ? fmaf(-a.mu, a.c[idx], rn) : rn;
}

// Bregman update after the L2 step: z = W x; v = z + b; d = shrink(v, thr) on
// bands 1..8 (band 0: d = v, b stays 0); b <- v - d; e <- d - b (what the next
// right-hand side needs); resid = ||z - d||_2.
__global__ __launch_bounds__(256) void k_tf_shrink(TfArgs a) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    const int n = a.n;
    const size_t np = (size_t)n * n;
    double part = 0.0;
    if (i < n && j < n) {
        float z[9];
        framelet_at(a.x + b * np, n, i, j, z);
        const size_t pix = (size_t)j * n + i;
        float* eb = a.e + (size_t)b * 9 * np;
        float* bb = a.bb + (size_t)b * 8 * np;
        eb[pix] = z[0];                           // d0 = z0, b0 = 0
#pragma unroll
        for (int band = 1; band < 9; band++) {
            const float bo = bb[(band - 1) * np + pix];
            const float v = z[band] + bo;
            const float mag = fabsf(v) - a.thr;
            const float d = mag > 0.f ? copysignf(mag, v) : 0.f;
            const float bn = v - d;
            bb[(band - 1) * np + pix] = bn;
            eb[band * np + pix] = d - bn;
            const double dz = (double)z[band] - (double)d;
            part = fma(dz, dz, part);
        }
    }
    const int nblk = gridDim.x * gridDim.y, blk = (j0 / 16) * gridDim.x + i0 / 16;
    block_partial<256>(part, a.partial + (size_t)b * nblk + blk);
}

// Forward-backward splitting, proximal step part 1: e = shrink(W x, thr), band 0 kept.
__global__ __launch_bounds__(256) void k_fbs_shrink(TfArgs a) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    const int n = a.n;
    if (i >= n || j >= n) return;
    const size_t np = (size_t)n * n, pix = (size_t)j * n + i;
    float z[9];
    framelet_at(a.x + b * np, n, i, j, z);
    float* eb = a.e + (size_t)b * 9 * np;
    eb[pix] = z[0];
#pragma unroll
    for (int band = 1; band < 9; band++) {
        const float mag = fabsf(z[band]) - a.thr;
        eb[band * np + pix] = mag > 0.f ? copysignf(mag, z[band]) : 0.f;
    }
}

// part 2: X_new = W^T e over X (= a.bb), partial sums of (X_new - X)^2.
__global__ __launch_bounds__(256) void k_fbs_adjoint(TfArgs a) {
    int i0, j0;
    framelet_tile(i0, j0);
    const int i = i0 + (threadIdx.x & 15), j = j0 + (threadIdx.x >> 4), b = blockIdx.z;
    const int n = a.n;
    const size_t np = (size_t)n * n;
    double part = 0.0;
    if (i < n && j < n) {
        const size_t idx = b * np + (size_t)j * n + i;
        const float xn = framelet_adj_at(a.e + (size_t)b * 9 * np, n, i, j);
        const double dx = (double)xn - (double)a.bb[idx];
        part = dx * dx;
        a.bb[idx] = xn;
    }
    const int nblk = gridDim.x * gridDim.y, blk = (j0 / 16) * gridDim.x + i0 / 16;
    block_partial<256>(part, a.partial + (size_t)b * nblk + blk);
}

hipError_t launch_fbs_shrink(const TfArgs& a, int batch, hipStream_t s) {
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, batch);
    hipLaunchKernelGGL(k_fbs_shrink, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fbs_adjoint(const TfArgs& a, int batch, hipStream_t s) {
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, batch);
    hipLaunchKernelGGL(k_fbs_adjoint, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_framelet_fwd(int n, const float* x, float* z, int batch, hipStream_t s) {
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_framelet_fwd, grid, dim3(256), 0, s, x, z, n);
    return hipGetLastError();
}

hipError_t launch_framelet_adj(int n, const float* z, float* x, int batch, hipStream_t s) {
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_framelet_adj, grid, dim3(256), 0, s, z, x, n);
    return hipGetLastError();
}

hipError_t launch_cg_start(int n, float* c, const float* e, float mu, float* r, double* partial, float* rmax,
                           int batch, hipStream_t s) {
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_cg_start, grid, dim3(256), 0, s, c, e, mu, r, partial, rmax, n);
    return hipGetLastError();
}

hipError_t launch_cg_update_xc(const CgArgs& a, int batch, hipStream_t s) {
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, batch);
    hipLaunchKernelGGL(k_cg_xc, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tf_shrink(const TfArgs& a, int batch, hipStream_t s) {
    dim3 grid((a.n + 15) / 16, (a.n + 15) / 16, batch);
    hipLaunchKernelGGL(k_tf_shrink, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- fills
__global__ void k_fill(float* __restrict__ p, size_t count, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const size_t blocks = (count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

}  // namespace air
