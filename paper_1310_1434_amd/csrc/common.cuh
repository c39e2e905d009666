// Device helpers shared by the AIR kernels (gfx950, wave64).
#pragma once

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

// Write one 16x16 tile of an image into its two padded line sets: rows (line
// set 1, pad[j][kPad + i]) and columns (line set 0, pad[i][kPad + j]), plus the
// zero samples at both ends of every line the tile touches at the border.
// tile is 16 x 17 shared floats; all 256 threads of the block must call this.
__device__ __forceinline__ void store_padded_tile(float* pad_b, int n, int line, int i0, int j0, int tx,
                                                  int ty, float v, float (*tile)[17]) {
    float* cols = pad_b;
    float* rows = pad_b + (size_t)n * line;
    const int i = i0 + tx, j = j0 + ty;
    if (i < n && j < n) rows[(size_t)j * line + kPad + i] = v;
    if (j < n && tx < kPad) {
        if (i0 == 0) rows[(size_t)j * line + tx] = 0.f;
        if (i0 + 16 >= n) rows[(size_t)j * line + kPad + n + tx] = 0.f;
    }
    tile[ty][tx] = v;
    __syncthreads();
    const int ic = i0 + ty, jc = j0 + tx;   // column line ic, sample jc
    if (ic < n && jc < n) cols[(size_t)ic * line + kPad + jc] = tile[tx][ty];
    if (ic < n && tx < kPad) {
        if (j0 == 0) cols[(size_t)ic * line + tx] = 0.f;
        if (j0 + 16 >= n) cols[(size_t)ic * line + kPad + n + tx] = 0.f;
    }
}

}  // namespace air
