// Ramp filtration y' = C y as a dense Toeplitz GEMM on the matrix cores.
//
// Rows of the sinogram batch (batch x views) form M, detector bins form K and
// N: Y'[m][n] = sum_k Y[m][k] T(k - n), T(d) = kappa r(|d|) for |d| < n_bins.
// The Toeplitz operand is never stored as a matrix: the float32 kernel reads
// it from a copy of the taps in LDS, the 16-bit kernels from precomputed MFMA
// fragments, one per diagonal offset k0 - n0.
//
// Tiles: a block of 4 waves covers 64 rows x 32 columns; each wave owns 16
// rows and two 16x16 accumulator tiles.  When the output is group-interleaved
// (the backprojector's input, [group][v][k][G]) the tile rows run over
// (group, view, image in group), so the G images of one view are rows of the
// same wave and every G-float output chunk is completed by one block.  Blocks
// go to the eight XCDs round-robin; the column tiles of one row tile are kept
// on one XCD, so each sinogram row is fetched into that XCD's L2 once.  Rows have stride ds (n_bins rounded
// up to 32, zero-filled), so the K loop needs no bounds tests.  Within one
// MFMA the assignment of actual k to the instruction's k slots is free as
// long as both operands agree; it is chosen so that each lane reads
// contiguous sinogram values (one 16-byte load per lane per 16 k for f32,
// two per 32 k for the 16-bit kernels).
#include "common.cuh"

namespace air {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------- tiles
// Tile row m -> image b and view v.  grp == 0: m = b * n_views + v (the input
// layout).  grp > 0: m = (gi * n_views + v) * grp + bl, b = gi * grp + bl; rows of
// images past the batch are padding.
struct RampRow {
    int b, v;
    size_t out;       // output offset of column 0 (add col * (grp ? grp : 1))
    bool valid;
};
__device__ __forceinline__ RampRow ramp_row(int m, int batch, int n_views, int ds, int grp) {
    RampRow r;
    if (grp == 0) {
        r.b = m / n_views;
        r.v = m - r.b * n_views;
        r.out = (size_t)m * ds;
    } else {
        const int per = n_views * grp;
        const int gi = m / per, rem = m - gi * per;
        r.v = rem / grp;
        const int bl = rem - r.v * grp;
        r.b = gi * grp + bl;
        r.out = ((size_t)gi * n_views + r.v) * ds * grp + bl;
    }
    r.valid = r.b < batch;
    return r;
}

// Tile rows of a launch and the block -> (row tile, column tile) map.
__host__ __device__ inline int ramp_tile_rows(int batch, int n_views, int grp) {
    return (grp == 0 ? batch : (batch + grp - 1) / grp * grp) * n_views;
}
__device__ __forceinline__ bool ramp_block(int row_tiles, int col_tiles, int& rt, int& ct) {
    const int L = blockIdx.x, q = L >> 3;
    const int j = q / col_tiles;
    ct = q - j * col_tiles;
    rt = j * 8 + (L & 7);
    return rt < row_tiles;
}

// ---------------------------------------------------------------------------- float32

template <int SCALE>
__global__ __launch_bounds__(256) void k_ramp_f32(const float* __restrict__ y, float* __restrict__ yf,
                                                  const float* __restrict__ taps, const float* __restrict__ step,
                                                  const float* __restrict__ wsq, int n_views, int rows, int ds,
                                                  int grp) {
    extern __shared__ float T[];   // [2 ds]: T[d + ds] = kappa r(|d|)
    const int batch = rows / n_views, mrows = ramp_tile_rows(batch, n_views, grp);
    int rt, ct;
    if (!ramp_block((mrows + 63) / 64, ds / 32, rt, ct)) return;   // (uniform over the block)
    for (int i = threadIdx.x; i < 2 * ds; i += 256) T[i] = taps[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = rt * 64 + w * 16 + (lane & 15);   // A row of this lane
    const int slot = lane >> 4;                     // k slot 0..3
    const int n0 = ct * 32;
    const int ncol = n0 + (lane & 15);
    const RampRow ar = ramp_row(m, batch, n_views, ds, grp);
    const bool mvalid = m < mrows && ar.valid;
    const float* arow = y + (mvalid ? ((size_t)ar.b * n_views + ar.v) * ds : 0);
    f4_t acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < ds; k0 += 16) {
        float4 av = *reinterpret_cast<const float4*>(arow + k0 + 4 * slot);
        if (wsq) {      // cosine-weighted C: D^(1/2) before R
            const float4 wv = *reinterpret_cast<const float4*>(wsq + k0 + 4 * slot);
            av.x *= wv.x;
            av.y *= wv.y;
            av.z *= wv.z;
            av.w *= wv.w;
        }
        if (!mvalid) av = make_float4(0.f, 0.f, 0.f, 0.f);
        // MFMA #q uses actual k = k0 + 4 slot + q in this lane's slot
        const int d = k0 + 4 * slot - ncol + ds;
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, T[d + 0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, T[d + 0 - 16], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, T[d + 1], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, T[d + 1 - 16], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, T[d + 2], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, T[d + 2 - 16], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, T[d + 3], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, T[d + 3 - 16], acc1, 0, 0, 0);
    }
    // accumulator layout: lane holds C[4 (lane/16) + r][lane % 16]
    const int rbase = rt * 64 + w * 16 + 4 * (lane >> 4);
    const int cs = grp ? grp : 1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int row = rbase + r;
        const RampRow orow = ramp_row(row, batch, n_views, ds, grp);
        if (row < mrows && orow.valid) {
            float o0 = acc0[r], o1 = acc1[r];
            if (wsq) {      // and D^(1/2) after
                o0 *= wsq[ncol];
                o1 *= wsq[ncol + 16];
            }
            if (SCALE & RAMP_POST) {
                const float* so = step + (size_t)orow.v * ds;
                o0 *= so[ncol];
                o1 *= so[ncol + 16];
            }
            yf[orow.out + (size_t)ncol * cs] = o0;
            yf[orow.out + (size_t)(ncol + 16) * cs] = o1;
        }
    }
}

// ---------------------------------------------------------------------------- 16-bit splits
// Fragment f of a split term holds, for lane l, the 8 values T16(delta + 8 (l/16) + i - l%16),
// i = 0..7, with delta = dmin + 16 f (delta = k0 - n0 of the tile).
template <int PREC, int SCALE>
__global__ __launch_bounds__(256) void k_ramp_split(const float* __restrict__ y, float* __restrict__ yf,
                                                    RampTables t, int rows, int ds, int grp) {
    const int batch = rows / t.n_views, mrows = ramp_tile_rows(batch, t.n_views, grp);
    int rt, ct;
    if (!ramp_block((mrows + 63) / 64, ds / 32, rt, ct)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = rt * 64 + w * 16 + (lane & 15);
    const int slot = lane >> 4;                 // k slots 8 slot .. 8 slot + 7
    const int n0 = ct * 32;
    const RampRow ar = ramp_row(m, batch, t.n_views, ds, grp);
    const bool mvalid = m < mrows && ar.valid;
    const float* arow = y + (mvalid ? ((size_t)ar.b * t.n_views + ar.v) * ds : 0);
    f4_t accA0 = {0.f, 0.f, 0.f, 0.f}, accA1 = accA0, accB0 = accA0, accB1 = accA0;
    for (int k0 = 0; k0 < ds; k0 += 32) {
        float4 a0 = *reinterpret_cast<const float4*>(arow + k0 + 8 * slot);
        float4 a1 = *reinterpret_cast<const float4*>(arow + k0 + 8 * slot + 4);
        if (t.wsq) {    // cosine-weighted C: D^(1/2) before R
            const float4 w0 = *reinterpret_cast<const float4*>(t.wsq + k0 + 8 * slot);
            const float4 w1 = *reinterpret_cast<const float4*>(t.wsq + k0 + 8 * slot + 4);
            a0.x *= w0.x; a0.y *= w0.y; a0.z *= w0.z; a0.w *= w0.w;
            a1.x *= w1.x; a1.y *= w1.y; a1.z *= w1.z; a1.w *= w1.w;
        }
        if (!mvalid) {
            a0 = make_float4(0.f, 0.f, 0.f, 0.f);
            a1 = a0;
        }
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const int f0 = (k0 - n0 - t.dmin) >> 4;      // fragment of the first n tile
        const int f1 = f0 - 1;                        // n0 + 16: delta - 16
        if (PREC == AIR_MIXED_F16) {
            h8_t hi, lo;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const _Float16 h = (_Float16)av[i];
                hi[i] = h;
                lo[i] = (_Float16)((av[i] - (float)h) * 2048.f);
            }
            const uint4 bh0 = t.frag_a[(size_t)f0 * 64 + lane], bl0 = t.frag_b[(size_t)f0 * 64 + lane];
            const uint4 bh1 = t.frag_a[(size_t)f1 * 64 + lane], bl1 = t.frag_b[(size_t)f1 * 64 + lane];
            const h8_t Bh0 = __builtin_bit_cast(h8_t, bh0), Bl0 = __builtin_bit_cast(h8_t, bl0);
            const h8_t Bh1 = __builtin_bit_cast(h8_t, bh1), Bl1 = __builtin_bit_cast(h8_t, bl1);
            accA0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, Bh0, accA0, 0, 0, 0);
            accA1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, Bh1, accA1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, Bl0, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, Bl1, accB1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, Bh0, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, Bh1, accB1, 0, 0, 0);
        } else {
            b8_t s1, s2, s3;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const __bf16 c1 = (__bf16)av[i];
                const float r1 = av[i] - (float)c1;
                const __bf16 c2 = (__bf16)r1;
                const __bf16 c3 = (__bf16)(r1 - (float)c2);
                s1[i] = c1; s2[i] = c2; s3[i] = c3;
            }
            const b8_t B10 = __builtin_bit_cast(b8_t, t.frag_a[(size_t)f0 * 64 + lane]);
            const b8_t B20 = __builtin_bit_cast(b8_t, t.frag_b[(size_t)f0 * 64 + lane]);
            const b8_t B30 = __builtin_bit_cast(b8_t, t.frag_c[(size_t)f0 * 64 + lane]);
            const b8_t B11 = __builtin_bit_cast(b8_t, t.frag_a[(size_t)f1 * 64 + lane]);
            const b8_t B21 = __builtin_bit_cast(b8_t, t.frag_b[(size_t)f1 * 64 + lane]);
            const b8_t B31 = __builtin_bit_cast(b8_t, t.frag_c[(size_t)f1 * 64 + lane]);
            accA0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B10, accA0, 0, 0, 0);
            accA1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B11, accA1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B20, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B21, accB1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s2, B10, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s2, B11, accB1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B30, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s1, B31, accB1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s2, B20, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s2, B21, accB1, 0, 0, 0);
            accB0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s3, B10, accB0, 0, 0, 0);
            accB1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s3, B11, accB1, 0, 0, 0);
        }
    }
    const float cross = (PREC == AIR_MIXED_F16) ? (1.f / 2048.f) : 1.f;
    const int rbase = rt * 64 + w * 16 + 4 * (lane >> 4);
    const int ncol = n0 + (lane & 15);
    const int cs = grp ? grp : 1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int row = rbase + r;
        const RampRow orow = ramp_row(row, batch, t.n_views, ds, grp);
        if (row < mrows && orow.valid) {
            float o0 = t.out_scale * fmaf(accB0[r], cross, accA0[r]);
            float o1 = t.out_scale * fmaf(accB1[r], cross, accA1[r]);
            if (t.wsq) {    // and D^(1/2) after
                o0 *= t.wsq[ncol];
                o1 *= t.wsq[ncol + 16];
            }
            if (SCALE & RAMP_POST) {
                const float* so = t.step + (size_t)orow.v * ds;
                o0 *= so[ncol];
                o1 *= so[ncol + 16];
            }
            yf[orow.out + (size_t)ncol * cs] = o0;
            yf[orow.out + (size_t)(ncol + 16) * cs] = o1;
        }
    }
}

template <int SCALE>
static hipError_t launch_ramp_scaled(int prec, const RampTables& t, const float* y, float* yf, int rows, int ds,
                                     int grp, hipStream_t s) {
    const int n_views = t.n_views;
    const int row_tiles = (ramp_tile_rows(rows / n_views, n_views, grp) + 63) / 64;
    dim3 grid(8 * ((row_tiles + 7) / 8) * (ds / 32)), block(256);
    if (prec == AIR_FP32) {
        hipLaunchKernelGGL(k_ramp_f32<SCALE>, grid, block, 2 * ds * sizeof(float), s, y, yf, t.taps32, t.step,
                           t.wsq, t.n_views, rows, ds, grp);
    } else if (prec == AIR_MIXED_F16) {
        hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_F16, SCALE>), grid, block, 0, s, y, yf, t, rows, ds, grp);
    } else if (prec == AIR_MIXED_BF16) {
        hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_BF16, SCALE>), grid, block, 0, s, y, yf, t, rows, ds, grp);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ramp(int prec, const RampTables& t, const float* y, float* yf, int rows, int ds, int scale,
                       int grp, hipStream_t s) {
    switch (scale) {
    case 0: return launch_ramp_scaled<0>(prec, t, y, yf, rows, ds, grp, s);
    case RAMP_POST: return launch_ramp_scaled<RAMP_POST>(prec, t, y, yf, rows, ds, grp, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace air
