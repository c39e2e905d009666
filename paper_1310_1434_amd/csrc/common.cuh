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

// Deterministic block reduction of one float64 per thread.  Every block writes
// its partial to partial[blk]; the block that arrives last (device-scope
// counter) sums all partials in index order with a fixed tree and writes *out,
// then re-arms the counter.  The result does not depend on which block is last
// or on how many batch items share the launch.
template <int BLOCK>
__device__ __forceinline__ void block_reduce_last(double v, double* partial, unsigned* count, double* out,
                                                  int nblk, int blk) {
    __shared__ double sh[BLOCK / kWave];
    __shared__ bool last;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid % kWave, wid = tid / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / kWave; w++) s += sh[w];
        partial[blk] = s;
        __threadfence();
        const unsigned prev = atomicAdd(count, 1u);
        last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double s = 0.0;
    for (int i = tid; i < nblk; i += BLOCK) s += __hip_atomic_load(partial + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / kWave; w++) t += sh[w];
        *out = t;
        atomicExch(count, 0u);
    }
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
