// Device-side helpers shared by the HIP kernels of the FastDF push (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdf {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): four 64-bit counter
// words mixed with a two-word key through ten rounds; the key advances by the
// Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ u64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2,
                                           uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  u64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Stream tags of the method's draws (key word 1).
constexpr uint64_t kStreamField = 0x46, kStreamPosition = 0x50,
                   kStreamMomentum = 0x51, kStreamDirection = 0x44;

// uint64 -> (0,1): (floor(w/2^12) + 1/2) 2^-52, exact in binary64.
__device__ __forceinline__ double unit_open(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// bfloat16 storage (round to nearest even; inputs are finite)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename R> struct cplx { R x, y; };

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }

// Canonical momentum of particle id (sec. 2.1 sampling): |q| with pdf
// proportional to q^2 fbar(q), drawn by a Gamma(3, T) proposal
// q = -T ln(u0 u1 u2) kept when u3 (1 + e^{-q/T}) < 1 (first kept trial of at
// most 64), times an isotropic direction (mu = 2u - 1, phi = 2 pi u'); each
// component computed in binary64 and rounded once to binary32.
__device__ __forceinline__ void sample_momentum(uint64_t seed, uint64_t id, double T, float* qf) {
  const u64x4 wd = philox4x64(id, 0, 0, 0, seed, kStreamDirection);
  const double mu = 2.0 * unit_open(wd.v[0]) - 1.0;
  const double ph = 2.0 * 3.14159265358979323846 * unit_open(wd.v[1]);
  const double st = sqrt(1.0 - mu * mu);
  const double nh[3] = {st * cos(ph), st * sin(ph), mu};
  double q = 0.0;
  for (int trial = 0; trial < 64; ++trial) {
    const u64x4 w = philox4x64(id, (uint64_t)trial, 0, 0, seed, kStreamMomentum);
    const double u0 = unit_open(w.v[0]), u1 = unit_open(w.v[1]);
    const double u2 = unit_open(w.v[2]), u3 = unit_open(w.v[3]);
    const double prop = -T * log(u0 * u1 * u2);
    q = prop;
    if (u3 * (1.0 + exp(-prop / T)) < 1.0) break;
  }
  for (int d = 0; d < 3; ++d) qf[d] = (float)(q * nh[d]);
}

}  // namespace fdf
