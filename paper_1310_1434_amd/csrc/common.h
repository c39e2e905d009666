// Device helpers shared by the AIR kernels (gfx950, wave64).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "air_internal.h"

namespace air {

constexpr int kWave = 64;

// RayEntry::meta fields (see geometry.h)
__device__ __forceinline__ int ray_lo(int32_t meta) { return meta & 0x7FFF; }
__device__ __forceinline__ int ray_hi(int32_t meta) { return ((meta >> 15) & 0x7FFF) - 1; }
__device__ __forceinline__ int ray_axis(int32_t meta) { return (meta >> 30) & 1; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}

// Block sum of one float64 per thread with a fixed tree (wave shuffles, then
// the waves in order); thread 0 stores it to *slot.  The partials of all
// blocks are summed by k_finalize in index order, so a reduction gives the
// same bits whatever the batch size or the order in which blocks run.
template <int BLOCK>
__device__ __forceinline__ void block_partial(double v, double* slot) {
    __shared__ double sh[BLOCK / kWave];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    v = wave_sum(v);
    if (tid % kWave == 0) sh[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / kWave; w++) s += sh[w];
        *slot = s;
    }
    __syncthreads();
}

// Block maximum of one non-negative float per thread (fmaxf: a NaN is passed
// over unless every value is NaN); thread 0 stores it to *slot.  A maximum
// takes no rounding, so any order of reduction gives the same value.
template <int BLOCK>
__device__ __forceinline__ void block_max(float v, float* slot) {
    __shared__ float sh[BLOCK / kWave];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    if (tid % kWave == 0) sh[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        float m = sh[0];
#pragma unroll
        for (int w = 1; w < BLOCK / kWave; w++) m = fmaxf(m, sh[w]);
        *slot = m;
    }
    __syncthreads();
}

// G contiguous floats at p, aligned to min(4 G, 16) bytes.
template <int G>
__device__ __forceinline__ void load_group(const float* p, float (&v)[G]) {
    if constexpr (G % 4 == 0) {
#pragma unroll
        for (int q = 0; q < G; q += 4) {
            const float4 t = *reinterpret_cast<const float4*>(p + q);
            v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
        }
    } else if constexpr (G == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
        for (int q = 0; q < G; q++) v[q] = p[q];
    }
}
template <int G>
__device__ __forceinline__ void store_group(float* p, const float (&v)[G]) {
    if constexpr (G % 4 == 0) {
#pragma unroll
        for (int q = 0; q < G; q += 4) *reinterpret_cast<float4*>(p + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
    } else if constexpr (G == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int q = 0; q < G; q++) p[q] = v[q];
    }
}
template <int G>
__device__ __forceinline__ void store_zero_group(float* p) {
    float z[G];
#pragma unroll
    for (int q = 0; q < G; q++) z[q] = 0.f;
    store_group<G>(p, z);
}

// float16 samples of P <= 4 images, one aligned 2 P-byte store (round to nearest).
template <int P>
__device__ __forceinline__ void store_half_group(uint16_t* p, const float (&v)[P]) {
    uint16_t h[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < P; q++) h[q] = __half_as_ushort(__float2half_rn(v[q]));
    if constexpr (P == 4) *reinterpret_cast<uint2*>(p) = make_uint2(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16);
    else if constexpr (P == 2) *reinterpret_cast<uint32_t*>(p) = h[0] | (uint32_t)h[1] << 16;
    else p[0] = h[0];
}
// A sample group of a padded line set, float32 or float16.
template <int P>
__device__ __forceinline__ void put_group(float* p, const float (&v)[P]) { store_group<P>(p, v); }
template <int P>
__device__ __forceinline__ void put_group(uint16_t* p, const float (&v)[P]) { store_half_group<P>(p, v); }
template <int P, typename T>
__device__ __forceinline__ void put_zero_group(T* p) {
    float z[P];
#pragma unroll
    for (int q = 0; q < P; q++) z[q] = 0.f;
    put_group<P>(p, z);
}

// Write one 16x16 tile of a group of G images into its padded line sets,
// which hold the images in consecutive pairs (or singles) of P (see PadBuf;
// pad points at the first of the G / P sub-groups): rows (line set 1,
// [j][kPad + i][q]) and columns (line set 0, [i][kPad + j][q]), plus the zero
// samples at both ends of every line the tile touches at the border.  The
// column copy goes through shared memory so that both copies are written as
// contiguous runs.  lds holds 16 * 17 * G floats; all 256 threads of the
// block must call this.  T: float, or uint16_t for float16 copies (v already
// scaled).
template <int G, int P, typename T = float>
__device__ __forceinline__ void store_padded_group(T* pad, int n, int line, int i0, int j0, int tx, int ty,
                                                   const float (&v)[G], float* lds) {
    static_assert(G % P == 0, "sub-groups must tile the group");
    const size_t sub = (size_t)2 * n * line * P;     // samples per sub-group
    const int i = i0 + tx, j = j0 + ty;
#pragma unroll
    for (int s = 0; s < G / P; s++) {
        T* rows = pad + s * sub + (size_t)n * line * P;
        float u[P];
#pragma unroll
        for (int q = 0; q < P; q++) u[q] = v[s * P + q];
        if (i < n && j < n) put_group<P>(rows + ((size_t)j * line + kPad + i) * P, u);
        if (j < n && tx < kPad) {
            if (i0 == 0) put_zero_group<P>(rows + ((size_t)j * line + tx) * P);
            if (i0 + 16 >= n) put_zero_group<P>(rows + ((size_t)j * line + kPad + n + tx) * P);
        }
    }
#pragma unroll
    for (int q = 0; q < G; q++) lds[(ty * 17 + tx) * G + q] = v[q];
    __syncthreads();
    const int ic = i0 + ty, jc = j0 + tx;   // column line ic, sample jc
#pragma unroll
    for (int s = 0; s < G / P; s++) {
        T* cols = pad + s * sub;
        float w[P];
#pragma unroll
        for (int q = 0; q < P; q++) w[q] = lds[(tx * 17 + ty) * G + s * P + q];
        if (ic < n && jc < n) put_group<P>(cols + ((size_t)ic * line + kPad + jc) * P, w);
        if (ic < n && tx < kPad) {
            if (j0 == 0) put_zero_group<P>(cols + ((size_t)ic * line + tx) * P);
            if (j0 + 16 >= n) put_zero_group<P>(cols + ((size_t)ic * line + kPad + n + tx) * P);
        }
    }
}

// Write one 16 x (16 PIX) tile of a group of G images, held as vertical pixel
// columns (thread (tx, ty) holds (i0 + tx, j0 + PIX ty + r), r < PIX, in v[r]),
// into its padded line sets (sub-groups of P as in store_padded_group).  The
// pixels of a column are adjacent samples of one column line, so both copies
// are written as contiguous runs without a transpose.
template <int G, int P, int PIX>
__device__ __forceinline__ void store_padded_column(float* pad, int n, int line, int i0, int j0, int tx, int ty,
                                                    const float (&v)[PIX][G]) {
    static_assert(G % P == 0, "sub-groups must tile the group");
    const size_t sub = (size_t)2 * n * line * P;     // floats per sub-group
    const int i = i0 + tx, j = j0 + PIX * ty;
#pragma unroll
    for (int s = 0; s < G / P; s++) {
        float* cols = pad + s * sub;
        float* rows = cols + (size_t)n * line * P;
#pragma unroll
        for (int r = 0; r < PIX; r++) {
            float u[P];
#pragma unroll
            for (int q = 0; q < P; q++) u[q] = v[r][s * P + q];
            const int jr = j + r;
            if (jr >= n) break;
            if (i < n) {
                store_group<P>(rows + ((size_t)jr * line + kPad + i) * P, u);        // row jr, sample i
                store_group<P>(cols + ((size_t)i * line + kPad + jr) * P, u);        // column i, sample jr
            }
            if (tx < kPad) {
                if (i0 == 0) store_zero_group<P>(rows + ((size_t)jr * line + tx) * P);
                if (i0 + 16 >= n) store_zero_group<P>(rows + ((size_t)jr * line + kPad + n + tx) * P);
            }
        }
        if (i < n && ty < kPad) {
            if (j0 == 0) store_zero_group<P>(cols + ((size_t)i * line + ty) * P);
            if (j0 + 16 * PIX >= n) store_zero_group<P>(cols + ((size_t)i * line + kPad + n + ty) * P);
        }
    }
}

}  // namespace air
