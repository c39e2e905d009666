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
#include "common.h"

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

// ---------------------------------------------------------------------------- row scales
// One wavefront per row of stride ds: scale[row] = 2^(14 - e) for the row's
// max |y| = f 2^e (f in [0.5, 1)), so that the scaled row's largest value lies
// in [2^13, 2^14); 1 for a zero or non-finite row.  The float16 split of a
// scaled value then neither overflows (float16 max 65504) nor falls into the
// float16 subnormal range unless it is 2^27 times smaller than the row's
// largest value, and dividing the filtered row by the scale is exact.
__global__ __launch_bounds__(256) void k_row_scale(const float* __restrict__ y, float* __restrict__ scale, int rows,
                                                   int ds) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= rows) return;     // (uniform over the wavefront)
    const float* r = y + (size_t)row * ds;
    float m = 0.f;
    for (int k = 4 * lane; k < ds; k += 4 * kWave) {      // ds is a multiple of 32
        const float4 v = *reinterpret_cast<const float4*>(r + k);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    // (fmaxf drops a NaN operand; a NaN row keeps the max of its other values)
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if (lane == 0) {
        float s = 1.f;
        if (m > 0.f && isfinite(m)) {
            int e;
            frexpf(m, &e);
            s = ldexpf(1.f, min(max(14 - e, -126), 126));
        }
        scale[row] = s;
    }
}

// ---------------------------------------------------------------------------- 16-bit splits
// v_mfma_f32_16x16x16 (f16 / bf16): lane l supplies row (or column) l % 16 at
// k slots 4 (l / 16) + i, i < 4, mapped to the actual k = k0 + 4 (l / 16) + i,
// so its sinogram operand is one contiguous float4.  Its Toeplitz operand,
// T(k - n) for those four k, is four consecutive values of a split-term
// table, read from LDS as one 8-byte entry of the table copy shifted by
// (first index) mod 4.  For each chunk of KC k the block stages the part of
// the tables its columns need (all terms, all shifts: a few KB, so any
// detector size fits); NG 16-column tiles per wavefront let each sinogram load
// feed 3 NG (f16) or 6 NG (bf16) MFMAs.
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

template <int PREC, int SCALE, int NG>
__global__ __launch_bounds__(256) void k_ramp_split(const float* __restrict__ y, float* __restrict__ yf,
                                                    RampTables t, int rows, int ds, int grp) {
    constexpr int NT = PREC == AIR_MIXED_F16 ? 2 : 3;
    constexpr int KC = 512;                         // k per staged chunk
    constexpr int JW = (KC + 16 * NG) / 4 + 2;      // table entries per shift and chunk
    static_assert(kRampZero >= 16 * NG, "zero margin covers a partial column tile");
    __shared__ uint2 tab[NT * 4 * JW];              // [term][shift][entry]
    const int batch = rows / t.n_views, mrows = ramp_tile_rows(batch, t.n_views, grp);
    int rt, ct;
    if (!ramp_block((mrows + 63) / 64, (ds + 16 * NG - 1) / (16 * NG), rt, ct)) return;   // (uniform)
    const int tj = t.tab_j;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = rt * 64 + w * 16 + (lane & 15);
    const int slot = lane >> 4;                 // k slots 4 slot .. 4 slot + 3
    const int n0 = ct * 16 * NG;
    const int ng = min(NG, (ds - n0) / 16);     // column tiles inside ds (uniform)
    const int ncol = n0 + (lane & 15);
    const RampRow ar = ramp_row(m, batch, t.n_views, ds, grp);
    const bool mvalid = m < mrows && ar.valid;
    const float* arow = y + (mvalid ? ((size_t)ar.b * t.n_views + ar.v) * ds : 0);
    // the row's power-of-two scale (float16 split), applied before the split
    const float rs = (t.rscale && mvalid) ? t.rscale[(size_t)ar.b * t.n_views + ar.v] : 1.f;
    f4_t accA[NG], accB[NG];
#pragma unroll
    for (int c = 0; c < NG; c++) {
        accA[c] = (f4_t){0.f, 0.f, 0.f, 0.f};
        accB[c] = accA[c];
    }
    float4 an = *reinterpret_cast<const float4*>(arow + 4 * slot);
    for (int kc = 0; kc < ds; kc += KC) {
        // entries j_lo .. j_lo + JW - 1 hold every table index x = k - n + ds + kRampZero
        // (plus 3) of k in [kc, kc + KC) and n in [n0, n0 + 16 NG); past the tables'
        // end the last entry is repeated (only for k beyond ds, never used)
        const int j_lo = (kc - n0 - 16 * NG + ds + kRampZero) >> 2;
        __syncthreads();                        // the previous chunk's reads are done
        for (int e0 = 0; e0 < NT * 4 * JW; e0 += 4 * 256) {
            uint2 u[4];
#pragma unroll
            for (int h = 0; h < 4; h++) {
                const int e = min(e0 + h * 256 + (int)threadIdx.x, NT * 4 * JW - 1);
                const int us = e / JW, jj = e - us * JW;     // us = term * 4 + shift
                u[h] = t.tab16[(size_t)us * tj + min(j_lo + jj, tj - 1)];
            }
#pragma unroll
            for (int h = 0; h < 4; h++) tab[min(e0 + h * 256 + (int)threadIdx.x, NT * 4 * JW - 1)] = u[h];
        }
        __syncthreads();
        const int kend = min(kc + KC, ds);
        for (int k0 = kc; k0 < kend; k0 += 16) {
            float4 a = an;
            if (k0 + 16 < ds) an = *reinterpret_cast<const float4*>(arow + k0 + 16 + 4 * slot);
            if (t.wsq) {    // cosine-weighted C: D^(1/2) before R
                const float4 wv = *reinterpret_cast<const float4*>(t.wsq + k0 + 4 * slot);
                a.x *= wv.x; a.y *= wv.y; a.z *= wv.z; a.w *= wv.w;
            }
            if (!mvalid) a = make_float4(0.f, 0.f, 0.f, 0.f);
            const float av[4] = {a.x * rs, a.y * rs, a.z * rs, a.w * rs};
            // staged entry of T(k0 + 4 slot - ncol) for column tile 0; tile c is 16 lower
            const int x0 = k0 + 4 * slot - ncol + ds + kRampZero - 4 * j_lo;
            if constexpr (PREC == AIR_MIXED_F16) {
                h4_t hi, lo;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const _Float16 h = (_Float16)av[i];
                    hi[i] = h;
                    lo[i] = (_Float16)((av[i] - (float)h) * 2048.f);
                }
#pragma unroll
                for (int c = 0; c < NG; c++) {
                    const int x = x0 - 16 * c, e = (x & 3) * JW + (x >> 2);
                    const h4_t Bh = __builtin_bit_cast(h4_t, tab[e]);
                    const h4_t Bl = __builtin_bit_cast(h4_t, tab[4 * JW + e]);
                    accA[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(hi, Bh, accA[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(hi, Bl, accB[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(lo, Bh, accB[c], 0, 0, 0);
                }
            } else {
                s4_t s1, s2, s3;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const __bf16 c1 = (__bf16)av[i];
                    const float r1 = av[i] - (float)c1;
                    const __bf16 c2 = (__bf16)r1;
                    const __bf16 c3 = (__bf16)(r1 - (float)c2);
                    s1[i] = __builtin_bit_cast(short, c1);
                    s2[i] = __builtin_bit_cast(short, c2);
                    s3[i] = __builtin_bit_cast(short, c3);
                }
#pragma unroll
                for (int c = 0; c < NG; c++) {
                    const int x = x0 - 16 * c, e = (x & 3) * JW + (x >> 2);
                    const s4_t B1 = __builtin_bit_cast(s4_t, tab[e]);
                    const s4_t B2 = __builtin_bit_cast(s4_t, tab[4 * JW + e]);
                    const s4_t B3 = __builtin_bit_cast(s4_t, tab[8 * JW + e]);
                    accA[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s1, B1, accA[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s1, B2, accB[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s2, B1, accB[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s1, B3, accB[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s2, B2, accB[c], 0, 0, 0);
                    accB[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s3, B1, accB[c], 0, 0, 0);
                }
            }
        }
    }
    const float cross = (PREC == AIR_MIXED_F16) ? (1.f / 2048.f) : 1.f;
    const int rbase = rt * 64 + w * 16 + 4 * (lane >> 4);
    const int cs = grp ? grp : 1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int row = rbase + r;
        const RampRow orow = ramp_row(row, batch, t.n_views, ds, grp);
        if (row < mrows && orow.valid) {
            const float* so = t.step + (size_t)orow.v * ds;
            // undo the row's power-of-two scale exactly
            const float osc = t.rscale ? t.out_scale / t.rscale[(size_t)orow.b * t.n_views + orow.v] : t.out_scale;
#pragma unroll
            for (int c = 0; c < NG; c++) {
                if (c >= ng) break;
                const int col = ncol + 16 * c;
                float o = osc * fmaf(accB[c][r], cross, accA[c][r]);
                if (t.wsq) o *= t.wsq[col];     // and D^(1/2) after
                if (SCALE & RAMP_POST) o *= so[col];
                yf[orow.out + (size_t)col * cs] = o;
            }
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
    } else if (prec == AIR_MIXED_F16 || prec == AIR_MIXED_BF16) {
        if (t.rscale) {
            hipLaunchKernelGGL(k_row_scale, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, y, t.rscale, rows, ds);
            if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
        }
        // widest column tiles (up to 128 columns) that still give at least three blocks per CU
        const int rt8 = 8 * ((row_tiles + 7) / 8);
        const size_t lds = 0;
        const int ng = rt8 * ((ds + 127) / 128) >= 768 ? 8 : rt8 * ((ds + 63) / 64) >= 768 ? 4 : 2;
        const dim3 g2(rt8 * ((ds + 16 * ng - 1) / (16 * ng)));
        if (prec == AIR_MIXED_F16) {
            if (ng == 8) hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_F16, SCALE, 8>), g2, block, lds, s, y, yf, t, rows, ds, grp);
            else if (ng == 4) hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_F16, SCALE, 4>), g2, block, lds, s, y, yf, t, rows, ds, grp);
            else hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_F16, SCALE, 2>), g2, block, lds, s, y, yf, t, rows, ds, grp);
        } else {
            if (ng == 8) hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_BF16, SCALE, 8>), g2, block, lds, s, y, yf, t, rows, ds, grp);
            else if (ng == 4) hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_BF16, SCALE, 4>), g2, block, lds, s, y, yf, t, rows, ds, grp);
            else hipLaunchKernelGGL((k_ramp_split<AIR_MIXED_BF16, SCALE, 2>), g2, block, lds, s, y, yf, t, rows, ds, grp);
        }
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
