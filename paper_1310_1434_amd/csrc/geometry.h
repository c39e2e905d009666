// Host-side scan geometry and the per-ray Joseph tables (float64, built once
// per plan).  This translation unit is compiled without floating-point
// contraction so every intercept is evaluated exactly as written.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace air {

// One Joseph ray, as the GPU kernels read it (16 bytes, one load).
//   T(a) = tc + (a - c0) * 2m   intercept at driving index a in fixed point with
//                               kFrac = 32 fractional bits (m has 31), shifted
//                               by kPad, so that the high word of T is the
//                               sample's index in a padded line
//   meta = lo | (hi + 1) << 15 | axis << 30
// The path length per driving step, s = pixel |d| / |d_drive|, is kept in a
// separate per-ray array: A = S J with J the bare interpolation weights, and
// the normal operator A^T C A = J^T (S C S) J applies the first S in the
// projector's epilogue and the second in the ramp's.
// Integer arithmetic makes the intercept exact and associative: the forward
// projector advances it by 2m per step and the backprojector evaluates it
// directly, and both get the same bits.  Resolution 2^-32 pixel (the slope's
// rounding adds at most n/2 * 2^-32); a float32 intercept (error ~3e-5 pixel
// at n = 512) alone would move A^T C y by ~1e-5 relative, since the
// ramp-filtered sinogram is high-pass.  The interpolation weights are float32.
constexpr int kFrac = 32;      // fractional bits of tc and T
constexpr int kSlopeFrac = 31; // fractional bits of m (|m| <= 1 fits int32)
struct RayEntry {
    int64_t tc;
    int32_t m;
    int32_t meta;
};
static_assert(sizeof(RayEntry) == 16, "RayEntry must be 16 bytes");

inline int meta_lo(int32_t meta) { return meta & 0x7FFF; }
inline int meta_hi(int32_t meta) { return ((meta >> 15) & 0x7FFF) - 1; }
inline int meta_axis(int32_t meta) { return (meta >> 30) & 1; }

constexpr int kMaxN = 16384;
constexpr int kMaxBins = 8192;
constexpr int kPad = 2;          // zero samples at each end of a padded image line

// Host-side geometry (float64, caller's view tables copied).
struct GeomHost {
    int beam = 0;
    int n = 0, n_views = 0, n_bins = 0;
    double pixel = 0, bin = 0, sod = 0, sdd = 0;
    std::vector<double> cosv, sinv;
};

// Builds the per-ray tables (float64 on the host, no FMA contraction).
// Returns an empty string on success, else an error message.
// step[v * n_bins + k] receives s of each ray.
std::string build_ray_tables(const GeomHost& g, std::vector<RayEntry>& rays, std::vector<float>& step,
                             std::vector<int8_t>& axis, std::vector<int32_t>& lo, std::vector<int32_t>& hi);

// Taps r(0..n_bins-1) of the ramp window, float64, dimensionless (the
// detector pitch and the view count enter through kappa):
//   0 Ram-Lak      r(0) = 1/4, r(odd m) = -1/(pi m)^2, r(even m != 0) = 0
//   1 Shepp-Logan  r(m) = -2 / (pi^2 (4 m^2 - 1))
//   2 Hann         Ram-Lak times (1 + cos w) / 2 in frequency: r/2 + (r(m-1) + r(m+1))/4
void ramp_taps64(int n_bins, int window, std::vector<double>& r);

}  // namespace air
