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
#include "common.h"

namespace air {

// ---------------------------------------------------------------------------- image groups
int image_group(int batch) {
    if (batch <= 1) return 1;
    int best = 1, best_cost = batch * 3;
    for (int g : {2, 4, 8, 16}) {
        const int cost = (batch + g - 1) / g * (2 + g);
        if (cost < best_cost) {
            best = g;
            best_cost = cost;
        }
    }
    return best;
}

int pad_group(int batch) { return batch >= 2 ? 2 : 1; }
int pad_group16(int batch) { return batch >= 3 ? 4 : batch; }

int group_images(int max_batch) {
    int most = 0;
    for (int b = 1; b <= max_batch; b++) {
        const int g = std::max(image_group(b), std::max(pad_group(b), pad_group16(b)));
        most = std::max(most, (b + g - 1) / g * g);
    }
    return most;
}

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

// float16 copies: 16x16 tiles of P images, scaled per image; the column copy
// goes through shared memory so both copies are written as contiguous runs.
template <int P>
__global__ __launch_bounds__(256) void k_pad16(const float* __restrict__ x, uint16_t* __restrict__ pad,
                                               const float* __restrict__ scale, int n, int line, int batch) {
    __shared__ float lds[16 * 17 * P];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16, b0 = blockIdx.z * P;
    const int i = i0 + tx, j = j0 + ty;
    float v[P];
#pragma unroll
    for (int q = 0; q < P; q++)
        v[q] = (i < n && j < n && b0 + q < batch) ? x[((size_t)(b0 + q) * n + j) * n + i] * scale[b0 + q] : 0.f;
    const float zero[P] = {};
    uint16_t* cols = pad + (size_t)blockIdx.z * 2 * n * line * P;
    uint16_t* rows = cols + (size_t)n * line * P;
    if (i < n && j < n) store_half_group<P>(rows + ((size_t)j * line + kPad + i) * P, v);
    if (j < n && tx < kPad) {
        if (i0 == 0) store_half_group<P>(rows + ((size_t)j * line + tx) * P, zero);
        if (i0 + 16 >= n) store_half_group<P>(rows + ((size_t)j * line + kPad + n + tx) * P, zero);
    }
#pragma unroll
    for (int q = 0; q < P; q++) lds[(ty * 17 + tx) * P + q] = v[q];
    __syncthreads();
    const int ic = i0 + ty, jc = j0 + tx;
    float w[P];
#pragma unroll
    for (int q = 0; q < P; q++) w[q] = lds[(tx * 17 + ty) * P + q];
    if (ic < n && jc < n) store_half_group<P>(cols + ((size_t)ic * line + kPad + jc) * P, w);
    if (ic < n && tx < kPad) {
        if (j0 == 0) store_half_group<P>(cols + ((size_t)ic * line + tx) * P, zero);
        if (j0 + 16 >= n) store_half_group<P>(cols + ((size_t)ic * line + kPad + n + tx) * P, zero);
    }
}

hipError_t launch_pad16(const KGeom& g, const float* x, PadBuf pad, int batch, hipStream_t s) {
    const int pg = pad_group16(batch);
    dim3 grid((g.n + 15) / 16, (g.n + 15) / 16, (batch + pg - 1) / pg), block(256);
    if (pg == 4) hipLaunchKernelGGL(k_pad16<4>, grid, block, 0, s, x, pad.half, pad.scale, g.n, g.line, batch);
    else if (pg == 2) hipLaunchKernelGGL(k_pad16<2>, grid, block, 0, s, x, pad.half, pad.scale, g.n, g.line, batch);
    else hipLaunchKernelGGL(k_pad16<1>, grid, block, 0, s, x, pad.half, pad.scale, g.n, g.line, batch);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ x, double* __restrict__ partial, int n) {
    __shared__ float sh[4];
    const int i = blockIdx.x * 16 + (threadIdx.x & 15), j = blockIdx.y * 16 + (threadIdx.x >> 4), b = blockIdx.z;
    float m = 0.f;
    if (i < n && j < n) m = fabsf(x[((size_t)b * n + j) * n + i]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x * gridDim.y, blk = blockIdx.y * gridDim.x + blockIdx.x;
        partial[(size_t)b * nblk + blk] = (double)fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    }
}

hipError_t launch_absmax(int n, const float* x, double* partial, int batch, hipStream_t s) {
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_absmax, grid, dim3(256), 0, s, x, partial, n);
    return hipGetLastError();
}

// One block per image: max of the partials, then the power-of-two scale.
__global__ __launch_bounds__(256) void k_pad_scale(const double* __restrict__ partial, int nblk,
                                                   float* __restrict__ scale) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    double m = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) m = fmax(m, partial[(size_t)b * nblk + k]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        float s = 1.f;
        if (mx > 0.0 && isfinite(mx)) {
            int e;
            frexp(mx, &e);                                 // mx = f 2^e, f in [0.5, 1)
            s = ldexpf(1.f, min(max(14 - e, -126), 126));  // mx * s in [2^13, 2^14)
        }
        scale[b] = s;
    }
}

hipError_t launch_pad_scale(const double* partial, int nblk, int batch, float* scale, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_scale, dim3(batch), dim3(256), 0, s, partial, nblk, scale);
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
// The interpolation weights of a sample are f and 1 - f, f = frac(t) rounded to
// float32.  The kernels use them scaled by 2^32: W = 2^32 f (the fraction word
// converted to float32) and G = 2^32 - W = 2^32 (1 - f), rounded.  Scaling by a
// power of two changes no rounding of the weights, their products or the sums
// of those, so each kernel multiplies its result by 2^-32 once, exactly, and
// gets the same bits as with f and 1 - f (for magnitudes that neither overflow
// nor fall to subnormals when scaled: |values| below about 2^90).
__device__ __forceinline__ float fx_wfrac(int64_t t) { return (float)(uint32_t)t; }
constexpr float kFxOne = 0x1p32f;
// intercept at driving index a: tc + 2 (a - c0) m, as one 32x32->64 multiply and one shift-add
__device__ __forceinline__ int64_t fx_at(const RayEntry& e, int a_minus_c0) {
    int64_t prod = (int64_t)a_minus_c0 * (int64_t)e.m;
    asm volatile("" : "+v"(prod));      // keep the product 32x32 (no reassociation with the shift)
    return e.tc + prod * 2;
}

// the same as one 32x32->64 multiply-add: a2 = 2 (a - c0)
__device__ __forceinline__ int64_t fx_at2(const RayEntry& e, int a2) { return e.tc + (int64_t)a2 * (int64_t)e.m; }

// Index of the first of the two samples in a padded line of n + 4: clamping
// into [0, n + 2] only ever moves samples onto the zero padding, so an
// out-of-range step contributes exactly zero (no range test needed).
__device__ __forceinline__ int fx_clamped_index(int64_t t, int n) { return min(max(fx_index(t), 0), n + 2); }
// The same as one unsigned minimum: a negative index wraps above n + 2 and so
// lands on the two zero samples at the far end of the line instead of the near
// end; either way the step contributes exactly zero.
__device__ __forceinline__ uint32_t fx_clamped_index_u(int64_t t, int n) {
    return min((uint32_t)fx_index(t), (uint32_t)(n + 2));
}

// Raw buffer loads of a group's padded copies: a buffer descriptor for the
// group (uniform), this lane's byte offset (its line set and sample index) and
// the step's row offset, uniform over the wavefront, as the scalar offset.
// Offsets are 32-bit, so the buffer path serves groups below 2 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t group_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <int BYTES>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, uint32_t (&w)[BYTES / 4]) {
    if constexpr (BYTES == 16) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
        w[0] = u[0]; w[1] = u[1]; w[2] = u[2]; w[3] = u[3];
    } else if constexpr (BYTES == 8) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
        w[0] = u[0]; w[1] = u[1];
    } else {
        w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
    }
}

// Block -> (view, chunk of 256 bins).  Blocks go to the eight XCDs round-robin
// (block L to XCD L mod 8); XCDs 0-3 take the views whose rays are mostly
// x-driven and XCDs 4-7 the mostly y-driven ones, so each XCD's L2 holds one of
// the two line sets of the padded copies instead of both.  Returns false for a
// padding slot (no view).
__device__ __forceinline__ bool proj_block(const KGeom& g, int chunks, int& v, int& chunk) {
    const int L = blockIdx.x, r = L & 7;
    const int idx = (L >> 3) * 4 + (r & 3);
    v = g.vorder[(r >> 2) * g.v_half + idx / chunks];
    chunk = idx % chunks;
    return v >= 0;
}

typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef float float4_a8 __attribute__((ext_vector_type(4), aligned(8)));

template <int P, bool BUF>
__global__ __launch_bounds__(kProjBlock) void k_project(KGeom g, const float* __restrict__ pad,
                                                         float* __restrict__ y, int chunks, int batch) {
    static_assert(P == 1 || P == 2, "images per thread");
    int v, chunk;
    if (!proj_block(g, chunks, v, chunk)) return;
    const int k = chunk * kProjBlock + threadIdx.x;
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
    if constexpr (BUF) {
        // the same samples through a buffer descriptor: one unsigned minimum and
        // one shift-add per step instead of two clamps, an add and a 64-bit address
        constexpr uint32_t SB = P * 4;             // bytes per sample
        const uint32_t set_bytes = (uint32_t)g.n * (uint32_t)line * SB;
        const __amdgpu_buffer_rsrc_t rs = group_rsrc(pad + (size_t)blockIdx.y * 2 * g.n * line * P, 2 * set_bytes);
        const uint32_t lane_base = axis ? set_bytes : 0u;
        uint32_t row_bytes = (uint32_t)a_lo * (uint32_t)line * SB;
#pragma unroll 4
        for (int a = a_lo; a <= a_hi; a++, t += m, row_bytes += (uint32_t)line * SB) {
            const float wf = fx_wfrac(t), wg = kFxOne - wf;
            uint32_t w[2 * P];
            buf_load<2 * SB>(rs, fx_clamped_index_u(t, g.n) * SB + lane_base, row_bytes, w);
            if constexpr (P == 1) {
                acc[0] = fmaf(wg, __uint_as_float(w[0]), acc[0]);
                acc[0] = fmaf(wf, __uint_as_float(w[1]), acc[0]);
            } else {                                   // [j][0..1], [j + 1][0..1]
                acc[0] = fmaf(wg, __uint_as_float(w[0]), acc[0]);
                acc[0] = fmaf(wf, __uint_as_float(w[2]), acc[0]);
                acc[1] = fmaf(wg, __uint_as_float(w[1]), acc[1]);
                acc[1] = fmaf(wf, __uint_as_float(w[3]), acc[1]);
            }
        }
    }
    if constexpr (!BUF) {
        uint32_t row = (uint32_t)(a_lo * line);
#pragma unroll 4
        for (int a = a_lo; a <= a_hi; a++, t += m, row += line) {
            const float wf = fx_wfrac(t), wg = kFxOne - wf;
            const float* p = lines + (size_t)((row + (uint32_t)fx_clamped_index(t, g.n)) * (uint32_t)P);
            if constexpr (P == 1) {
                const float2_a4 u = *reinterpret_cast<const float2_a4*>(p);
                acc[0] = fmaf(wg, u.x, acc[0]);
                acc[0] = fmaf(wf, u.y, acc[0]);
            } else {
                const float4_a8 u = *reinterpret_cast<const float4_a8*>(p);    // [j][0..1], [j + 1][0..1]
                acc[0] = fmaf(wg, u.x, acc[0]);
                acc[0] = fmaf(wf, u.z, acc[0]);
                acc[1] = fmaf(wg, u.y, acc[1]);
                acc[1] = fmaf(wf, u.w, acc[1]);
            }
        }
    }
    if (k >= g.ds) return;
    const float sv = ray ? g.step[(size_t)v * g.ds + k] * 0x1p-32f : 0.f;     // (weights scaled by 2^32)
#pragma unroll
    for (int q = 0; q < P; q++) {
        if (b0 + q >= batch) break;
        float out = 0.f;
        if (ray) out = acc[q] * sv;
        y[((size_t)(b0 + q) * g.n_views + v) * g.ds + k] = out;
    }
}

// The same projector over float16 copies (mixed-precision plans): groups of
// P <= 4 images per sample, converted to float32 before the multiply-adds, sums
// divided by the images' power-of-two scales.
// Samples j (s0) and j + 1 (s1) of P float16 images from the words of one load.
template <int P>
__device__ __forceinline__ void unpack_half_pair(const uint32_t* w, float (&s0)[P], float (&s1)[P]) {
    auto h = [&](int idx) {      // half number idx of the loaded words
        const uint32_t x = w[idx >> 1];
        return __half2float(__ushort_as_half((unsigned short)((idx & 1) ? x >> 16 : x & 0xffff)));
    };
#pragma unroll
    for (int q = 0; q < P; q++) {
        s0[q] = h(q);
        s1[q] = h(P + q);
    }
}

template <int P>
__device__ __forceinline__ void load_half_pair(const uint16_t* p, float (&s0)[P], float (&s1)[P]) {
    if constexpr (P == 4) {
        const float4_a8 u = *reinterpret_cast<const float4_a8*>(p);     // [j][0..3], [j + 1][0..3]
        const uint32_t w[4] = {__float_as_uint(u.x), __float_as_uint(u.y), __float_as_uint(u.z), __float_as_uint(u.w)};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t a = w[q >> 1], c = w[2 + (q >> 1)];
            s0[q] = __half2float(__ushort_as_half((unsigned short)((q & 1) ? a >> 16 : a & 0xffff)));
            s1[q] = __half2float(__ushort_as_half((unsigned short)((q & 1) ? c >> 16 : c & 0xffff)));
        }
    } else if constexpr (P == 2) {
        const float2_a4 u = *reinterpret_cast<const float2_a4*>(p);     // [j][0..1], [j + 1][0..1]
        const uint32_t a = __float_as_uint(u.x), c = __float_as_uint(u.y);
        s0[0] = __half2float(__ushort_as_half((unsigned short)(a & 0xffff)));
        s0[1] = __half2float(__ushort_as_half((unsigned short)(a >> 16)));
        s1[0] = __half2float(__ushort_as_half((unsigned short)(c & 0xffff)));
        s1[1] = __half2float(__ushort_as_half((unsigned short)(c >> 16)));
    } else {
        s0[0] = __half2float(__ushort_as_half(p[0]));
        s1[0] = __half2float(__ushort_as_half(p[1]));
    }
}

template <int P, bool BUF>
__global__ __launch_bounds__(kProjBlock) void k_project16(KGeom g, const uint16_t* __restrict__ pad,
                                                           const float* __restrict__ scale, float* __restrict__ y,
                                                           int chunks, int batch) {
    int v, chunk;
    if (!proj_block(g, chunks, v, chunk)) return;
    const int k = chunk * kProjBlock + threadIdx.x;
    const int b0 = blockIdx.y * P;
    const bool ray = k < g.n_bins;
    RayEntry e;
    e.tc = 0;
    e.m = 0;
    e.meta = 0;
    if (ray) e = g.rays[(size_t)v * g.n_bins + k];
    const bool hits = ray && ray_hi(e.meta) >= ray_lo(e.meta);
    const int lo = hits ? ray_lo(e.meta) : 0x7fffffff;
    const int hi = hits ? ray_hi(e.meta) : -1;
    const int axis = ray_axis(e.meta);
    const int a_lo = max(0, __builtin_amdgcn_readfirstlane(wave_min_i(lo)) - 1);
    const int a_hi = min(g.n - 1, __builtin_amdgcn_readfirstlane(wave_max_i(hi)) + 1);
    const int line = g.line;
    const uint16_t* lines = pad + ((size_t)blockIdx.y * 2 + axis) * g.n * line * P;
    float acc[P];
#pragma unroll
    for (int q = 0; q < P; q++) acc[q] = 0.f;
    int64_t t = fx_at(e, a_lo - g.c0);
    const int64_t m = (int64_t)e.m * 2;
    if constexpr (BUF) {
        constexpr uint32_t SB = P * 2;             // bytes per sample
        const uint32_t set_bytes = (uint32_t)g.n * (uint32_t)line * SB;
        const __amdgpu_buffer_rsrc_t rs = group_rsrc(pad + (size_t)blockIdx.y * 2 * g.n * line * P, 2 * set_bytes);
        const uint32_t lane_base = axis ? set_bytes : 0u;
        uint32_t row_bytes = (uint32_t)a_lo * (uint32_t)line * SB;
#pragma unroll 4
        for (int a = a_lo; a <= a_hi; a++, t += m, row_bytes += (uint32_t)line * SB) {
            const float wf = fx_wfrac(t), wg = kFxOne - wf;
            uint32_t w[(2 * SB + 3) / 4];
            buf_load<(2 * SB + 3) / 4 * 4>(rs, fx_clamped_index_u(t, g.n) * SB + lane_base,
                                           row_bytes, w);
            float s0[P], s1[P];
            unpack_half_pair<P>(w, s0, s1);
#pragma unroll
            for (int q = 0; q < P; q++) {
                acc[q] = fmaf(wg, s0[q], acc[q]);
                acc[q] = fmaf(wf, s1[q], acc[q]);
            }
        }
    }
    if constexpr (!BUF) {
        uint32_t row = (uint32_t)(a_lo * line);
#pragma unroll 4
        for (int a = a_lo; a <= a_hi; a++, t += m, row += line) {
            const float wf = fx_wfrac(t), wg = kFxOne - wf;
            float s0[P], s1[P];
            load_half_pair<P>(lines + (size_t)((row + (uint32_t)fx_clamped_index(t, g.n)) * (uint32_t)P), s0, s1);
#pragma unroll
            for (int q = 0; q < P; q++) {
                acc[q] = fmaf(wg, s0[q], acc[q]);
                acc[q] = fmaf(wf, s1[q], acc[q]);
            }
        }
    }
    if (k >= g.ds) return;
    const float sv = ray ? g.step[(size_t)v * g.ds + k] * 0x1p-32f : 0.f;     // (weights scaled by 2^32)
#pragma unroll
    for (int q = 0; q < P; q++) {
        const int b = b0 + q;
        if (b >= batch) break;
        float out = 0.f;
        if (ray) out = acc[q] * sv / scale[b];    // exact: scale is a power of two
        y[((size_t)b * g.n_views + v) * g.ds + k] = out;
    }
}

static void launch_project_g(const KGeom& g, PadBuf pad, float* y, int batch, hipStream_t s) {
    // buffer addressing while a group's two line sets stay below 2 GiB (32-bit offsets)
    const auto fits = [&](int sample_bytes) { return 2.0 * g.n * g.line * sample_bytes < 2147483648.0; };
    const int chunks = (g.ds + kProjBlock - 1) / kProjBlock;
    if (pad.half) {
        const int pg = pad_group16(batch);
        dim3 grid(2 * g.v_half * chunks, (batch + pg - 1) / pg), block(kProjBlock);
        const bool buf = fits(2 * pg);
        if (pg == 4 && buf)
            hipLaunchKernelGGL((k_project16<4, true>), grid, block, 0, s, g, pad.half, pad.scale, y, chunks, batch);
        else if (pg == 4)
            hipLaunchKernelGGL((k_project16<4, false>), grid, block, 0, s, g, pad.half, pad.scale, y, chunks, batch);
        else if (pg == 2 && buf)
            hipLaunchKernelGGL((k_project16<2, true>), grid, block, 0, s, g, pad.half, pad.scale, y, chunks, batch);
        else if (pg == 2)
            hipLaunchKernelGGL((k_project16<2, false>), grid, block, 0, s, g, pad.half, pad.scale, y, chunks, batch);
        else    // (a single image's two float16 samples are not dword aligned: pointer loads)
            hipLaunchKernelGGL((k_project16<1, false>), grid, block, 0, s, g, pad.half, pad.scale, y, chunks, batch);
        return;
    }
    const int pg = pad_group(batch);
    dim3 grid(2 * g.v_half * chunks, (batch + pg - 1) / pg), block(kProjBlock);
    const bool buf = fits(4 * pg);
    if (pg == 2 && buf) hipLaunchKernelGGL((k_project<2, true>), grid, block, 0, s, g, pad.base, y, chunks, batch);
    else if (pg == 2) hipLaunchKernelGGL((k_project<2, false>), grid, block, 0, s, g, pad.base, y, chunks, batch);
    else if (buf) hipLaunchKernelGGL((k_project<1, true>), grid, block, 0, s, g, pad.base, y, chunks, batch);
    else hipLaunchKernelGGL((k_project<1, false>), grid, block, 0, s, g, pad.base, y, chunks, batch);
}

hipError_t launch_project(const KGeom& g, PadBuf pad, float* y, int batch, hipStream_t s) {
    launch_project_g(g, pad, y, batch, s);
    return hipGetLastError();
}

// out[b / grp][v][k][b % grp] = y[b][v][k] * step[v][k]  (S y).
__global__ __launch_bounds__(256) void k_scale(KGeom g, const float* __restrict__ y, float* __restrict__ out,
                                               size_t count, int grp) {
    const size_t per_batch = (size_t)g.n_views * g.ds;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
        const size_t b = i / per_batch, vk = i - b * per_batch;
        const float sv = g.step[vk];
        const size_t gi = b / grp;
        out[(gi * per_batch + vk) * grp + (b - gi * grp)] = y[i] * sv;
    }
}

hipError_t launch_scale(const KGeom& g, const float* y, float* out, int batch, int grp, hipStream_t s) {
    const size_t count = (size_t)batch * g.n_views * g.ds;
    const size_t blocks = (count + 255) / 256 < 8192 ? (count + 255) / 256 : 8192;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, s, g, y, out, count, grp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- adjoint J^T
// One thread per column of PIX vertically adjacent pixels (i, j .. j + PIX - 1)
// and up to BT images; 16 x 16 PIX pixels per block.  PIX = 2 throughout: four
// pixels per thread share more intercept work but halve the wavefronts (1.24
// against 0.82 ms at 512^2 and 8 images), one pixel doubles them but also the
// LDS reads per pixel (1.38 against 0.99 ms at 16 images).  For every view the
// thread takes the bins whose rays can give any of its pixels a non-zero Joseph
// weight: any sample that touches a pixel lies in the diamond |dx| + |dy| < pixel
// around its centre, so its ray meets the detector within hw bins of the
// centre's own projection, and the centres lie within e bins of the projection
// km of their midpoint, so the thread takes the bins within hw + e + 0.01 of km.
// hw and e are bounded over the whole tile, once per plan (k_bp_windows, which
// also fixes the bins the tile stages for each view and whether their rays are
// x- or y-driven).  For each candidate the thread re-evaluates the forward
// projector's own fixed-point intercept and float32 weights, so the result is
// the exact transpose of J (k_project before its step scaling) up to summation
// order.  An x-driven ray crosses all PIX pixels at the same intercept, so one
// evaluation gives every weight; a y-driven ray needs its own intercept (one
// multiply-add) per pixel.  A larger window only adds candidates of weight
// exactly zero, so every pixel gets the same bits whatever PIX and BT.
//
// Views are processed eight at a time.  Per view, the tile's bins (at most 32
// PIX per pass) and their sinogram values are staged in shared memory by one
// wavefront (two views each); the window records and the view directions are
// uniform over the block and read with scalar loads.  The terms of a pass are
// summed in float32, across passes in float64.  No atomics.

// Loads from addresses that are uniform over the wavefront, through the scalar
// cache (for data the kernel only reads).
typedef const __attribute__((address_space(4))) uint32_t uniform_word;
__device__ __forceinline__ uint32_t uniform_u32(const void* p, int k) { return ((uniform_word*)p)[k]; }
__device__ __forceinline__ BpWin uniform_win(const BpWin* p) {
    BpWin r;
    r.kb0 = (int32_t)uniform_u32(p, 0);
    r.meta = (int32_t)uniform_u32(p, 1);
    r.lo = __uint_as_float(uniform_u32(p, 2));
    r.hi = __uint_as_float(uniform_u32(p, 3));
    return r;
}
__device__ __forceinline__ float2 uniform_f2(const float2* p) {
    return make_float2(__uint_as_float(uniform_u32(p, 0)), __uint_as_float(uniform_u32(p, 1)));
}

// Continuous detector bin of the projection of point (px, py) in view (c, s),
// in float32 (k_bp_windows bounds its rounding); BEAM: 0 parallel, 1 fan.
// floor(x) as an int in one instruction (x finite, within the int range).
__device__ __forceinline__ int floor_i32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

template <int BEAM>
__device__ __forceinline__ float bin_of(const KGeom& g, float px, float py, float c, float s) {
    if constexpr (BEAM == 0) return fmaf(fmaf(px, c, py * s), g.inv_bin, g.half_d);
    const float ap = fmaf(py, c, -px * s);
    const float bp = fmaf(-px, c, fmaf(-py, s, g.sod));
    return fmaf(ap * __builtin_amdgcn_rcpf(bp), g.kdet, g.half_d);
}

// Float32 value not below x.
__device__ __forceinline__ float float_up(double x) {
    const float f = (float)x;
    return (double)f < x ? nextafterf(f, INFINITY) : f;
}

// One thread per (tile, view), in float64.  The rectangle R of pixel centres the
// tile's threads project spans the tile's in-image pixels and the in-image
// stand-ins of those past the edge (pairs are clamped to n - PIX).  Over R:
// hw bounds the projected half-width of a pixel's diamond (parallel beam
// pixel m / bin with m = max(|c|, |s|); fan beam: a vertex moves ap and bp by at
// most pixel m, so |du| <= sdd pixel m (bp + |ap|) / (bp (bp - pixel m)) / bin,
// which grows with |ap| and falls with bp); the tile stages the bins within
// hw + 1/2 of the corners' projections.  A pair's centres lie within
// e = (PIX - 1) pixel / 2 max |du/dy| of its midpoint's projection (|du/dx| for
// horizontal pairs).  Parallel beam: u = (x c + y s) / bin + half_d, so
// |du/dy| = |s| / bin.  Fan beam: u = (sdd / bin) ap / bp + half_d with
// ap = y c - x s and bp = sod - x c - y s, so du/dy = (sdd / bin) (c bp + s ap)
// / bp^2 and du/dx = (sdd / bin) (c ap - s bp) / bp^2; both numerators are
// linear in (x, y), so their largest magnitudes over R are at its corners, as
// is the smallest bp.  The 0.01 bin added to the half-widths covers the float32
// rounding of the kernel's projections.
template <int PIX>
__global__ __launch_bounds__(256) void k_bp_windows(KGeom g, BpWin* __restrict__ win, float2* __restrict__ winx) {
    constexpr int TW = kBpTileW, TH = kBpTileH;
    static_assert(TH == 16 * PIX && TW == 16, "backprojector tiles");
    const int n = g.n, tiles_x = (n + TW - 1) / TW;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= bp_window_count(n, g.n_views)) return;
    const int v = (int)(idx % g.n_views), tile = (int)(idx / g.n_views);
    const int i0 = (tile % tiles_x) * TW, j0 = (tile / tiles_x) * TH;
    const int ia = min(i0, max(n - PIX, 0)), ja = min(j0, max(n - PIX, 0));
    const int ib = max(min(i0 + TW - 1, n - 1), ia + PIX - 1), jb = max(min(j0 + TH - 1, n - 1), ja + PIX - 1);
    const double pixel = g.pixel, hn = g.half_n, inv_bin = g.inv_bin, hd = g.half_d;
    const double x[2] = {(ia - hn) * pixel, (ib - hn) * pixel}, y[2] = {(ja - hn) * pixel, (jb - hn) * pixel};
    const double c = g.views[v].x, s = g.views[v].y;
    double k_lo = INFINITY, k_hi = -INFINITY, bp_min = INFINITY, ap_max = 0.0, ny = 0.0, nx = 0.0;
    for (int q = 0; q < 4; q++) {
        const double qx = x[q & 1], qy = y[q >> 1];
        double u;
        if (g.beam == 0) {
            u = (qx * c + qy * s) * inv_bin + hd;
        } else {
            const double ap = qy * c - qx * s, bp = (double)g.sod - (qx * c + qy * s);
            u = (double)g.sdd * ap / bp * inv_bin + hd;
            bp_min = fmin(bp_min, bp);
            ap_max = fmax(ap_max, fabs(ap));
            ny = fmax(ny, fabs(c * bp + s * ap));
            nx = fmax(nx, fabs(c * ap - s * bp));
        }
        k_lo = fmin(k_lo, u);
        k_hi = fmax(k_hi, u);
    }
    const double dm = pixel * fmax(fabs(c), fabs(s));
    double hw, dy, dx;
    if (g.beam == 0) {
        hw = dm * inv_bin;
        dy = fabs(s) * inv_bin;
        dx = fabs(c) * inv_bin;
    } else {
        const double k = (double)g.sdd * inv_bin;
        hw = k * dm * (bp_min + ap_max) / (bp_min * (bp_min - dm));
        dy = k * ny / (bp_min * bp_min);
        dx = k * nx / (bp_min * bp_min);
    }
    const int kb0 = max(0, (int)floor(k_lo - hw - 0.5));
    const int kb1 = min(g.n_bins - 1, (int)ceil(k_hi + hw + 0.5));
    int any_x = 0, any_y = 0;
    const RayEntry* rays = g.rays + (size_t)v * g.n_bins;
    for (int k = kb0; k <= kb1; k++) {
        if (ray_axis(rays[k].meta)) any_y = 1;
        else any_x = 1;
    }
    const double e = 0.5 * (PIX - 1) * pixel;
    const double hy = hw + e * dy + 0.01, hx = hw + e * dx + 0.01;
    BpWin r;
    r.kb0 = kb0;
    r.meta = max(0, kb1 - kb0 + 1) | (any_x << 16) | (any_y << 17);
    r.lo = float_up(kb0 + hy);
    r.hi = float_up(hy - kb0);
    win[idx] = r;
    winx[idx] = make_float2(float_up(kb0 + hx), float_up(hx - kb0));
}

hipError_t launch_bp_windows(const KGeom& g, BpWin* win, float2* winx, hipStream_t s) {
    const size_t count = bp_window_count(g.n, g.n_views);
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bp_windows<2>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, g, win, winx);
    return hipGetLastError();
}

// Weights of ray e for the pixels (i, j + q), q < PIX (scaled by 2^32, see
// fx_wfrac): exactly zero for a ray that samples none of them.
// AX: 0 = the ray is x-driven, 1 = y-driven, 2 = either (read from the
// table).  A pixel takes G if the first sample of the pair is the pixel's own
// (in its interpolated index) and W if it is the one before.  Only
// a sample with -1 <= j0 < n can match an in-image pixel: exactly the samples
// the forward projector weights, so no range test is needed.
template <int AX, int PIX>
__device__ __forceinline__ void joseph_column(const RayEntry& e, int i, int j, int c0, float (&w)[PIX]) {
    // (the first sample's padded index s is compared with the pixels' own,
    // which are constants of the thread)
    if constexpr (AX == 0) {
        // all pixels sit on the column the ray samples at i: one intercept
        const int64_t t = fx_at2(e, 2 * (i - c0));
        const float wf = fx_wfrac(t), wg = kFxOne - wf;
        const int s = fx_index(t);
        bool at[PIX + 1];     // at[k]: the first sample is on row j + k - 1
#pragma unroll
        for (int k = 0; k <= PIX; k++) at[k] = s == j + kPad + k - 1;
#pragma unroll
        for (int q = 0; q < PIX; q++) w[q] = at[q + 1] ? wg : (at[q] ? wf : 0.f);
    } else {
        // y-driven (AX == 1, or AX == 2 and the table says so): driving row
        // j + q, interpolated index i; x-driven: driving column i, index j + q
        const bool ydrv = AX == 1 || ray_axis(e.meta);
#pragma unroll
        for (int q = 0; q < PIX; q++) {
            const int64_t t = fx_at2(e, 2 * ((ydrv ? j + q : i) - c0));
            const float wf = fx_wfrac(t);
            float wg = kFxOne - wf;
            asm volatile("" : "+v"(wg));    // keep the selection branch-free (G is not sunk into a branch)
            const int s = fx_index(t);
            const int o = (ydrv ? i : j + q) + kPad;
            w[q] = s == o ? wg : (s == o - 1 ? wf : 0.f);
        }
    }
}

// Accumulate the candidates [wlo, whi] (the staged slots of one view, SF floats
// each: the bin's ray entry, then its BT values) into the pixels, two at a
// time.  The second of the last pair may be slot whi + 1: a ray outside the
// window (the window holds every ray that samples the pair, so this one samples
// neither pixel and its weights are exactly zero), a zero-filled slot past the
// staged bins or the spare slot (a zero ray entry samples index 0, which no
// pixel's index matches).  Its values are finite, so it adds exactly nothing
// (0 * y + acc = acc).
__device__ __forceinline__ RayEntry slot_ray(const float* p) { return *reinterpret_cast<const RayEntry*>(p); }
template <int AX, int BT, int PIX, int SF>
__device__ __forceinline__ void bp_candidates(const float* slots, int wlo, int whi, int i, int j, int c0,
                                              float (&acc)[PIX][BT]) {
    for (int w = wlo; w <= whi; w += 2) {
        const float* p0 = slots + w * SF;
        const RayEntry e0 = slot_ray(p0), e1 = slot_ray(p0 + SF);
        float y0[BT], y1[BT];
        load_group<BT>(p0 + 4, y0);
        load_group<BT>(p0 + SF + 4, y1);
        float wt0[PIX], wt1[PIX];
        joseph_column<AX, PIX>(e0, i, j, c0, wt0);
        joseph_column<AX, PIX>(e1, i, j, c0, wt1);
#pragma unroll
        for (int r = 0; r < PIX; r++)
#pragma unroll
            for (int q = 0; q < BT; q++) acc[r][q] = fmaf(wt1[r], y1[q], fmaf(wt0[r], y0[q], acc[r][q]));
    }
}

// The same with the axis choice (uniform over the block) inside the candidate
// loop: one loop, so the accumulators keep one set of registers across views
// (the per-axis loops make the compiler move them between register sets at
// every view).  Used from 8-image groups: it needs far fewer registers than
// the per-axis loops (at 8 images it fits five wavefronts per SIMD), which
// leaves room on each CU for the kernels of the other sub-batch stream of a
// split solve (8-image halves of a 16-image batch), though on its own the
// 8-image kernel is slower than the per-axis loops; with 16 images it is
// faster alone too, with 4 or fewer the per-axis loops win either way.  Both
// perform the same operations in the same order.
constexpr int kBpInLoopMin = 8;
template <int PIX>
__device__ __forceinline__ void joseph_pair(int axes, const RayEntry& e0, const RayEntry& e1, int i, int j, int c0,
                                            float (&wt0)[PIX], float (&wt1)[PIX]) {
    if (axes == 0) {
        joseph_column<0, PIX>(e0, i, j, c0, wt0);
        joseph_column<0, PIX>(e1, i, j, c0, wt1);
    } else if (axes == 1) {
        joseph_column<1, PIX>(e0, i, j, c0, wt0);
        joseph_column<1, PIX>(e1, i, j, c0, wt1);
    } else {
        joseph_column<2, PIX>(e0, i, j, c0, wt0);
        joseph_column<2, PIX>(e1, i, j, c0, wt1);
    }
}
template <int BT, int PIX, int SF>
__device__ __forceinline__ void bp_candidates_any(int axes, const float* slots, int wlo, int whi, int i, int j,
                                                  int c0, float (&acc)[PIX][BT]) {
    const float* const last = slots + whi * SF;
    for (const float* p = slots + wlo * SF; p <= last; p += 2 * SF) {
        const RayEntry e0 = slot_ray(p), e1 = slot_ray(p + SF);
        float y0[BT], y1[BT];
        load_group<BT>(p + 4, y0);
        load_group<BT>(p + SF + 4, y1);
        float wt0[PIX], wt1[PIX];
        joseph_pair<PIX>(axes, e0, e1, i, j, c0, wt0, wt1);
#pragma unroll
        for (int r = 0; r < PIX; r++)
#pragma unroll
            for (int q = 0; q < BT; q++) acc[r][q] = fmaf(wt1[r], y1[q], fmaf(wt0[r], y0[q], acc[r][q]));
    }
}

// Pixels per backprojector thread (see k_backproject).
static int bp_pix(int) { return 2; }
int bp_blocks(int n, int batch) { return ((n + 15) / 16) * ((n + 16 * bp_pix(batch) - 1) / (16 * bp_pix(batch))); }

// The beam type is a template parameter: as a run-time test it cost three
// uniform branches per view (about 5% of the launch).
template <int MODE, bool REDUCE, int BT, int PIX, int BEAM>
__global__ __launch_bounds__(256, BT == 8 ? 5 : (BT < 8 ? 4 : 3)) void k_backproject(KGeom g, const float* __restrict__ y, BpArgs a, int batch) {
    constexpr int NV = 8;                  // views per pass (the same for every group size)
    constexpr int VW = NV / 4;             // views staged per wavefront
    constexpr int BINS = 32 * PIX;         // staged bins per view and pass
    constexpr int TH = 16 * PIX;           // tile height
    static_assert(TH == kBpTileH && kBpTileW == 16, "tiles of the window table");
    static_assert(BINS % kWave == 0, "whole wavefronts stage a view");
    // one spare slot past the staged bins, read by the second candidate of a pair
    constexpr int SLOTS = BINS + 1;
    // a slot is its bin's ray entry (4 words) followed by its BT values, 8
    // words at least (so that entries stay 16-byte aligned): 12 words at 8
    // images, 20 at 16, strides at which the 16-byte reads of 8 consecutive
    // slots fall in distinct LDS banks; one address per candidate serves both
    constexpr int SF = BT >= 4 ? 4 + BT : 8;
    __shared__ __align__(16) float s_slot[NV][SLOTS * SF];
    // A group of views whose staged rays are all x-driven runs one loop
    // with no axis test.  One whose rays are all y-driven runs the same
    // loop over horizontal pixel tuples instead, which then share each
    // intercept as vertical ones do for x-driven rays; the tuple sums
    // reach the vertical owners through LDS.  Every pixel takes the same
    // terms in the same order either way.  Groups of both kinds, and
    // windows wider than one pass, take the per-view axis test.  Only
    // up to 4 images: the extra loops cost 8- and 16-image groups about 40
    // VGPRs (measured when the totals were float64 and rays and values sat
    // in separate arrays: 127 -> 165 and 195 -> 243), and the halves of a
    // two-stream solve (8 or 16 images) then leave less room for the
    // other stream's kernels (slower overall, though an 8-image launch
    // alone was 13% faster).
    constexpr bool kModes = BT <= 4;
    static_assert(!kModes || BT < kBpInLoopMin, "single-axis groups use the per-axis loop");
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    // tiles -> XCDs: blocks go to the eight XCDs round-robin; when the tile grid
    // splits into eight equal rectangles, each XCD gets one of them, so the
    // tiles sharing an L2 are neighbours and stage overlapping windows
    int bx = blockIdx.x, by = blockIdx.y;
    {
        const int gx = gridDim.x, gy = gridDim.y;
        if (gx % 4 == 0 && gy % 2 == 0) {
            const int L = by * gx + bx, T = gx * gy;
            const int t = (L % 8) * (T / 8) + L / 8;
            const int rw = gx / 4, rh = gy / 2, r = t / (rw * rh), u = t % (rw * rh);
            bx = (r % 4) * rw + u % rw;
            by = (r / 4) * rh + u / rw;
        }
    }
    const int i0 = bx * 16, j0 = by * TH;
    const int i = i0 + tx, j = j0 + PIX * ty;      // pixels (i, j + r), r < PIX
    const int b0 = blockIdx.z * BT;
    const int n = g.n;
    // the tile's window records, one per view
    const size_t wrow = (size_t)(by * gridDim.x + bx) * g.n_views;
    const BpWin* wt = g.bpwin + wrow;
    const float2* wtx = g.bpwinx + wrow;
    // midpoint of the thread's pixel column (pixels past the image edge take an
    // in-image neighbour's window; their sums are dropped)
    const float px = ((float)min(i, n - 1) - g.half_n) * g.pixel;
    const float pym = ((float)min(j, max(n - PIX, 0)) - g.half_n + 0.5f * (PIX - 1)) * g.pixel;
    // the same thread's horizontal tuple (ih + q, jh), q < PIX, used for view
    // groups whose rays are all y-driven (kModes), and its midpoint
    const int ih = i0 + PIX * (threadIdx.x % (16 / PIX)), jh = j0 + threadIdx.x / (16 / PIX);
    const float pxhm = ((float)min(ih, max(n - PIX, 0)) - g.half_n + 0.5f * (PIX - 1)) * g.pixel;
    const float pyh = ((float)min(jh, n - 1) - g.half_n) * g.pixel;
    // group-interleaved input [group][v][k][BT]: this thread's BT images are
    // contiguous and 4 * BT-byte aligned
    const float* yg = y + (size_t)blockIdx.z * g.n_views * g.ds * BT;
    float tot[PIX][BT];
#pragma unroll
    for (int r = 0; r < PIX; r++)
#pragma unroll
        for (int q = 0; q < BT; q++) tot[r][q] = 0.f;
    for (int v0 = 0; v0 < g.n_views; v0 += NV) {
        // staging passes over the widest window of the eight views, and the
        // union of their axis bits (bit 0: some ray x-driven, bit 1: some y-driven)
        int passes = 0, axes_any = 0;
#pragma unroll
        for (int s = 0; s < NV; s++) {
            if (v0 + s < g.n_views) {
                const int m = (int)uniform_u32(&wt[v0 + s], 1);
                passes = max(passes, ((m & 0xFFFF) + BINS - 1) / BINS);
                axes_any |= m >> 16;
            }
        }
        int mode = 0;    // 1: all rays x-driven, 2: all y-driven (one pass, up to 4 images)
        if (kModes && passes == 1) mode = (axes_any & 2) == 0 ? 1 : ((axes_any & 1) == 0 ? 2 : 0);
        float acc[PIX][BT];
#pragma unroll
        for (int r = 0; r < PIX; r++)
#pragma unroll
            for (int q = 0; q < BT; q++) acc[r][q] = 0.f;
        for (int p = 0; p < passes; p++) {
            // stage: wavefront w loads bins kb0 + p * BINS + (lane, lane + 64, ...)
            // of views w and w + 4 of the pass; slots past the window get zeros
#pragma unroll
            for (int hh = 0; hh < VW; hh++) {
                const int sv = wave + 4 * hh, v = v0 + sv;
                int kb0 = 0, nb = 0;
                if (v < g.n_views) {
                    const BpWin r = uniform_win(&wt[v]);
                    kb0 = r.kb0;
                    nb = r.meta & 0xFFFF;
                }
#pragma unroll
                for (int hb = 0; hb < BINS / kWave; hb++) {
                    const int slot = hb * kWave + lane;
                    const int w = p * BINS + slot;
                    int4 e = make_int4(0, 0, 0, 0);     // a RayEntry
                    float t[BT];
#pragma unroll
                    for (int q = 0; q < BT; q++) t[q] = 0.f;
                    if (w < nb) {
                        const int k = kb0 + w;
                        e = reinterpret_cast<const int4*>(g.rays)[(size_t)v * g.n_bins + k];
                        load_group<BT>(yg + ((size_t)v * g.ds + k) * BT, t);
                    }
                    float* sl = &s_slot[sv][slot * SF];
                    *reinterpret_cast<int4*>(sl) = e;
                    store_group<BT>(sl + 4, t);
                }
                // the spare slot: a zero ray entry and zero values (staged with
                // every pass: the horizontal tuples' exchange reuses this memory)
                if (lane == 0) {
                    float* sl = &s_slot[sv][BINS * SF];
                    float z[BT];
#pragma unroll
                    for (int q = 0; q < BT; q++) z[q] = 0.f;
                    *reinterpret_cast<int4*>(sl) = make_int4(0, 0, 0, 0);
                    store_group<BT>(sl + 4, z);
                }
            }
            __syncthreads();
            // the staged slots [wlo, whi] within the window of a pixel pair whose
            // midpoint projects to km
            const int base = p * BINS;
            // (ceil(km - lo) = -floor(lo - km): one rounding convert each)
            auto window = [&](float km, float lo, float hi, int meta, int& wlo, int& whi) {
                wlo = max(-floor_i32(lo - km) - base, 0);
                whi = min(floor_i32(km + hi) - base, min((meta & 0xFFFF) - 1 - base, BINS - 1));
            };
            if (mode == 1) {
#pragma unroll
                for (int s = 0; s < NV; s++) {
                    const int v = v0 + s;
                    if (v >= g.n_views) continue;
                    const BpWin r = uniform_win(&wt[v]);
                    const float2 cs = uniform_f2(&g.views[v]);
                    int wlo, whi;
                    window(bin_of<BEAM>(g, px, pym, cs.x, cs.y), r.lo, r.hi, r.meta, wlo, whi);
                    bp_candidates<0, BT, PIX, SF>(s_slot[s], wlo, whi, i, j, g.c0, acc);
                }
                __syncthreads();
                continue;
            }
            if (mode == 2) {
                // acc (still zero: first and only pass) first holds the tuple sums
#pragma unroll
                for (int s = 0; s < NV; s++) {
                    const int v = v0 + s;
                    if (v >= g.n_views) continue;
                    const int meta = (int)uniform_u32(&wt[v], 1);
                    const float2 lh = uniform_f2(&wtx[v]);
                    const float2 cs = uniform_f2(&g.views[v]);
                    int wlo, whi;
                    window(bin_of<BEAM>(g, pxhm, pyh, cs.x, cs.y), lh.x, lh.y, meta, wlo, whi);
                    // the x-driven loop with the roles of rows and columns exchanged
                    bp_candidates<0, BT, PIX, SF>(s_slot[s], wlo, whi, jh, ih, g.c0, acc);
                }
                __syncthreads();
                // tuple sums -> [row][column][image] in the value buffer -> vertical owners
                float* xb = &s_slot[0][0];
                static_assert(NV * SLOTS * SF >= 16 * TH * BT, "exchange fits the slot buffer");
#pragma unroll
                for (int q = 0; q < PIX; q++) store_group<BT>(xb + ((jh - j0) * 16 + (ih - i0) + q) * BT, acc[q]);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < PIX; r++) load_group<BT>(xb + ((j - j0 + r) * 16 + (i - i0)) * BT, acc[r]);
                __syncthreads();
                continue;
            }
#pragma unroll
            for (int s = 0; s < NV; s++) {
                const int v = v0 + s;
                if (v >= g.n_views) continue;
                const BpWin r = uniform_win(&wt[v]);
                const float2 cs = uniform_f2(&g.views[v]);
                int wlo, whi;
                window(bin_of<BEAM>(g, px, pym, cs.x, cs.y), r.lo, r.hi, r.meta, wlo, whi);
                // staged rays all x-driven (0), all y-driven (1) or both (2)
                const int am = (r.meta >> 16) & 3;
                const int axes = am == 1 ? 0 : (am == 2 ? 1 : 2);
                if constexpr (BT >= kBpInLoopMin)
                    bp_candidates_any<BT, PIX, SF>(axes, s_slot[s], wlo, whi, i, j, g.c0, acc);
                else if (axes == 0)
                    bp_candidates<0, BT, PIX, SF>(s_slot[s], wlo, whi, i, j, g.c0, acc);
                else if (axes == 1)
                    bp_candidates<1, BT, PIX, SF>(s_slot[s], wlo, whi, i, j, g.c0, acc);
                else
                    bp_candidates<2, BT, PIX, SF>(s_slot[s], wlo, whi, i, j, g.c0, acc);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < PIX; r++)
#pragma unroll
            for (int q = 0; q < BT; q++) tot[r][q] += acc[r][q];
    }
#pragma unroll
    for (int r = 0; r < PIX; r++)
#pragma unroll
        for (int q = 0; q < BT; q++) tot[r][q] *= 0x1p-32;     // (weights scaled by 2^32: exact)
    const int nblk = gridDim.x * gridDim.y;
    const int blk = by * gridDim.x + bx;
    float res[PIX][BT];     // RESIDUAL: r of every pixel and image (0 outside the image or batch)
#pragma unroll
    for (int q = 0; q < BT; q++) {
#pragma unroll
        for (int r = 0; r < PIX; r++) res[r][q] = 0.f;
        const int b = b0 + q;
        if (b >= batch) continue;     // uniform across the block
        double part = 0.0;
#pragma unroll
        for (int r = 0; r < PIX; r++) {
            if (i >= n || j + r >= n) continue;
            const size_t idx = (size_t)b * n * n + (size_t)(j + r) * n + i;
            if (MODE == BP_PLAIN) {
                a.out[idx] = tot[r][q];
            } else if (MODE == BP_MATVEC) {
                const float pv = a.aux[idx];
                const float qv = (float)fma((double)a.mu, (double)pv, (double)tot[r][q]);
                a.out[idx] = qv;
                part += (double)pv * (double)qv;
            } else if (MODE == BP_STEP) {
                a.out[idx] = (float)fma((double)a.mu, (double)a.rhs[idx] - (double)tot[r][q], (double)a.aux[idx]);
            } else {  // BP_RESIDUAL
                const float rv = (float)((double)a.out[idx] - fma((double)a.mu, (double)a.aux[idx], (double)tot[r][q]));
                a.out[idx] = rv;
                a.p_out[idx] = rv;
                res[r][q] = rv;
                part += (double)rv * (double)rv;
            }
        }
        if (REDUCE) block_partial<256>(part, a.partial + (size_t)b * nblk + blk);
    }
    if (MODE == BP_RESIDUAL && a.pad_out.base) {    // (float16 copies are built separately)
        constexpr int P = BT < 2 ? BT : 2;    // pad_group(batch)
        store_padded_column<BT, P, PIX>(a.pad_out.base + (size_t)b0 * 2 * n * g.line, n, g.line, i0, j0, tx, ty, res);
    }
}

template <int MODE, bool REDUCE, int BEAM>
static void launch_bp_beam(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s) {
    const int bt = image_group(batch), pix = bp_pix(batch);
    dim3 grid((g.n + 15) / 16, (g.n + 16 * pix - 1) / (16 * pix), (batch + bt - 1) / bt), block(256);
    if (bt == 16) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 16, 2, BEAM>), grid, block, 0, s, g, y, a, batch);
    else if (bt == 8) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 8, 2, BEAM>), grid, block, 0, s, g, y, a, batch);
    else if (bt == 4) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 4, 2, BEAM>), grid, block, 0, s, g, y, a, batch);
    else if (bt == 2) hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 2, 2, BEAM>), grid, block, 0, s, g, y, a, batch);
    else hipLaunchKernelGGL((k_backproject<MODE, REDUCE, 1, 2, BEAM>), grid, block, 0, s, g, y, a, batch);
}

template <int MODE, bool REDUCE>
static void launch_bp_mode(const KGeom& g, const float* y, const BpArgs& a, int batch, hipStream_t s) {
    if (g.beam == 0) launch_bp_beam<MODE, REDUCE, 0>(g, y, a, batch, s);
    else launch_bp_beam<MODE, REDUCE, 1>(g, y, a, batch, s);
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
    case BP_STEP:
        launch_bp_mode<BP_STEP, false>(g, y, a, batch, s);
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
