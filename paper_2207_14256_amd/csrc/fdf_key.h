// Spatial sort key of a particle, shared by the sort's rank pass and the
// push that writes the keys for the next step's re-sort (gfx950).
#pragma once
#include "fdf_device.h"

namespace fdf {
namespace sort_key {

__device__ __forceinline__ uint32_t part1by2(uint32_t v) {   // spread 10 bits to every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton index of the coarse tile of cell c (the counting-sort bucket) above
// the Morton index of the cell inside the tile (fine_bits = log2 tile side).
__device__ __forceinline__ uint32_t morton_key(const uint32_t (&c)[3], int fine_bits) {
  const int fb = fine_bits;
  const uint32_t fm = (1u << fb) - 1u;
  const uint32_t coarse = (part1by2(c[0] >> fb) << 2) | (part1by2(c[1] >> fb) << 1) | part1by2(c[2] >> fb);
  const uint32_t fine = (part1by2(c[0] & fm) << 2) | (part1by2(c[1] & fm) << 1) | part1by2(c[2] & fm);
  return (coarse << (3 * fb)) | fine;
}

// Key of an FP32 particle at fixed-point position xin and momentum q: the
// position extrapolated by tau_scaled = predict_tau 2^32 / L along its
// velocity q / sqrt(q^2 + (m a)^2) (when predict), wrapping with the box.
__device__ __forceinline__ uint32_t key_f32(const uint32_t (&xin)[3], const float (&q)[3], float ma,
                                            float tau_scaled, bool predict, int cell_shift, int fine_bits) {
  uint32_t x[3] = {xin[0], xin[1], xin[2]};
  if (predict) {
    const float f = tau_scaled / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + ma * ma);
    for (int d = 0; d < 3; ++d) x[d] += (uint32_t)__float2int_rn(q[d] * f);
  }
  uint32_t c[3];
  for (int d = 0; d < 3; ++d) c[d] = x[d] >> cell_shift;
  return morton_key(c, fine_bits);
}

}  // namespace sort_key
}  // namespace fdf
