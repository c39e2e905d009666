// Host-side scan geometry and the per-ray Joseph tables (float64, built once
// per plan).  This translation unit is compiled without floating-point
// contraction so every intercept is evaluated exactly as written.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace air {

// One Joseph ray, as the GPU kernels read it (32 bytes, two 16-byte loads).
//   t(a) = fma((double)(a - c0), m, tc)   intercept at driving index a (pixel units, float64)
//   s    = pixel |d| / |d_drive|           path length per driving step
//   meta = lo | (hi + 1) << 15 | axis << 30
// The intercept is float64 because the ramp-filtered sinogram is high-pass:
// a float32 intercept (error ~3e-5 pixel at n = 512) alone moves A^T C y by
// ~1e-5 relative.  The interpolation weights themselves are float32.
struct RayEntry {
    double tc;
    double m;
    float s;
    int32_t meta;
    int32_t unused[2];
};
static_assert(sizeof(RayEntry) == 32, "RayEntry must be 32 bytes");

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
std::string build_ray_tables(const GeomHost& g, std::vector<RayEntry>& rays, std::vector<int8_t>& axis,
                             std::vector<int32_t>& lo, std::vector<int32_t>& hi);

// Ram-Lak taps r(0..n_bins-1), float64.
void ramp_taps64(int n_bins, std::vector<double>& r);

}  // namespace air
