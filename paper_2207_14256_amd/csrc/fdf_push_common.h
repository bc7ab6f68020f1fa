// Pieces shared by the push kernels: block size, the XCD-aware chunk order,
// segment lookup and non-temporal particle-state access.
#pragma once
#include "fdf_device.h"
#include "fdf_internal.h"

namespace fdf {
namespace push_detail {

constexpr int kBlock = 256;

// Consecutive block ids are dealt round-robin to the 8 XCDs; remap so each
// XCD (own L2) walks a contiguous range of chunks, i.e. a compact region of
// sorted particles.
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t nb) {
  const int64_t full = nb - nb % 8;
  if (b >= full) return b;
  const int64_t per = full / 8;
  return (b % 8) * per + b / 8;
}

// Several segments (species) in one launch: each XCD takes the same share of
// every segment, a contiguous eighth of its chunks, and walks its shares in
// segment order.  A contiguous eighth of the whole chunk range would give
// whole species to single XCDs, and species whose particles cost more (sparse
// seeds, whose gathers share few mesh lines) would hold the launch on those
// XCDs.  -1: a block past its XCD's share (the grid is 8 times the largest).
__device__ __forceinline__ int64_t xcd_segment_chunk(const PushArgs& a, int64_t b) {
  const int64_t x = b & 7;
  int64_t l = b >> 3;
  for (int s = 0; s < a.nseg; ++s) {
    const int64_t cb = a.seg[s].chunk_begin;
    const int64_t n = (s + 1 < a.nseg ? a.seg[s + 1].chunk_begin : a.total_chunks) - cb;
    const int64_t lo = n * x / 8, hi = n * (x + 1) / 8;
    if (l < hi - lo) return cb + lo + l;
    l -= hi - lo;
  }
  return -1;
}

// The chunk of this block in a non-persistent launch, or -1.
__device__ __forceinline__ int64_t launch_chunk(const PushArgs& a) {
  return a.xcd_blocks > 0 ? xcd_segment_chunk(a, blockIdx.x) : xcd_chunk(blockIdx.x, gridDim.x);
}

__device__ __forceinline__ int find_segment(const Segment* seg, int nseg, int64_t chunk) {
  int s = 0;
  while (s + 1 < nseg && seg[s + 1].chunk_begin <= chunk) ++s;
  return s;
}

// The segment of a chunk in the copy that holds its species' current state
// (both copies list the same chunk ranges); *skip: the species is left alone
// by this launch.
__device__ __forceinline__ const Segment& chunk_segment(const PushArgs& a, int64_t chunk, bool* skip) {
  const int s = find_segment(a.seg, a.nseg, chunk);
  const bool low = s < 64;
  *skip = low && ((a.skip_mask >> s) & 1ull);
  return (low && ((a.alt_mask >> s) & 1ull)) ? a.seg_alt[s] : a.seg[s];
}

// The state arrays live in device global memory.  Their pointers come from a
// device-side segment table, so the compiler cannot infer the address space
// and would emit flat instructions; naming the global space gives global
// loads/stores with a scalar base and a 32-bit lane offset.
// (The host pass parses device code too; HIP's vector classes cannot bind
// address-space-qualified references there, and no code is emitted for it.)
#if defined(__HIP_DEVICE_COMPILE__)
#define FDF_GLOBAL __attribute__((address_space(1)))
#else
#define FDF_GLOBAL
#endif
template <typename T> __device__ __forceinline__ const FDF_GLOBAL T* gptr(const T* p) {
  return (const FDF_GLOBAL T*)p;
}
template <typename T> __device__ __forceinline__ T ldnt(const T* p) { return __builtin_nontemporal_load(gptr(p)); }
template <typename T> __device__ __forceinline__ void stnt(T v, T* p) {
  __builtin_nontemporal_store(v, (FDF_GLOBAL T*)p);
}

// Interpolation stencil of the force: CIC (r = 1, 8 points) or TSC (r = 2,
// 27 points).  Every operation is explicit so that each copy of the code is
// instruction-identical (bitwise results whatever slot a particle lands in).
template <bool TSC> struct Stencil { static constexpr int N = TSC ? 27 : 8; };

// FP32 form: x is a 32-bit fixed-point fraction of the box per axis.
template <bool TSC, typename I>
__device__ __forceinline__ void stencil_u32(const uint32_t* xu, int shift, uint32_t gmask, float finv,
                                            I G, I* cell, float* w) {
#pragma clang fp contract(off)
  const uint32_t fmask = (1u << shift) - 1u;
  if constexpr (!TSC) {
    uint32_t i0[3], i1[3];
    float t[3], u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      i0[d] = xu[d] >> shift;
      i1[d] = (i0[d] + 1u) & gmask;
      t[d] = (float)(xu[d] & fmask) * finv;
      u[d] = 1.0f - t[d];
    }
    const I ax[2] = {(I)mesh_x(i0[0], (uint32_t)G), (I)mesh_x(i1[0], (uint32_t)G)};
    const I ay[2] = {(I)mesh_y(i0[1], (uint32_t)G), (I)mesh_y(i1[1], (uint32_t)G)};
    const I az[2] = {(I)mesh_z(i0[2]), (I)mesh_z(i1[2])};
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc >> 2, cy = (cc >> 1) & 1, cz = cc & 1;
      cell[cc] = ax[cx] + ay[cy] + az[cz];
      w[cc] = ((cx ? t[0] : u[0]) * (cy ? t[1] : u[1])) * (cz ? t[2] : u[2]);
    }
  } else {
    // nearest point i = floor(u + 1/2); f = u + 1/2 - i = d + 1/2 in [0, 1)
    uint32_t idx[3][3];
    float wt[3][3];
    const uint32_t half = 1u << (shift - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const uint32_t xs = xu[d] + half;                 // wraps with the box
      const uint32_t i = xs >> shift;
      const float f = (float)(xs & fmask) * finv;
      const float g = 1.0f - f, h = f - 0.5f;
      idx[d][0] = (i - 1u) & gmask;
      idx[d][1] = i;
      idx[d][2] = (i + 1u) & gmask;
      wt[d][0] = 0.5f * (g * g);                        // (1/2 - d)^2 / 2
      wt[d][1] = 0.75f - h * h;                         // 3/4 - d^2
      wt[d][2] = 0.5f * (f * f);                        // (1/2 + d)^2 / 2
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cell[9 * a + 3 * b + c] =
              (I)mesh_x(idx[0][a], (uint32_t)G) + (I)mesh_y(idx[1][b], (uint32_t)G) + (I)mesh_z(idx[2][c]);
          w[9 * a + 3 * b + c] = (wt[0][a] * wt[1][b]) * wt[2][c];
        }
  }
}

// CIC stencil of the FP32 form as byte offsets into a mesh of CB-byte cells
// (the same corners and weights as stencil_u32<false>): the per-axis terms
// of the brick layout scaled by CB with 24-bit multiplies and shifts (full
// rate), instead of a 32-bit multiplication of every corner's cell index.
template <uint32_t CB>
__device__ __forceinline__ void stencil_u32_bytes(const uint32_t* xu, int shift, uint32_t gmask, float finv,
                                                  uint32_t lg, uint32_t* off, float* w) {
#pragma clang fp contract(off)
  const uint32_t fmask = (1u << shift) - 1u;
  uint32_t i0[3], i1[3];
  float t[3], u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    i0[d] = xu[d] >> shift;
    i1[d] = (i0[d] + 1u) & gmask;
    t[d] = (float)(xu[d] & fmask) * finv;
    u[d] = 1.0f - t[d];
  }
  // bytes of mesh_x(i) * CB, mesh_y(i) * CB, mesh_z(i) * CB
  auto mul24 = [](uint32_t a, uint32_t b) { return (uint32_t)__umul24(a, b); };
  auto bx = [&](uint32_t i) { return (mul24(i >> 2, CB) << (2u * lg + 2u)) + mul24(i & 3u, 16u * CB); };
  auto by = [&](uint32_t i) { return (mul24(i >> 2, CB) << (lg + 4u)) + mul24(i & 3u, 4u * CB); };
  auto bz = [&](uint32_t i) { return mul24(i >> 2, 64u * CB) + mul24(i & 3u, CB); };
  const uint32_t ax[2] = {bx(i0[0]), bx(i1[0])};
  const uint32_t ay[2] = {by(i0[1]), by(i1[1])};
  const uint32_t az[2] = {bz(i0[2]), bz(i1[2])};
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int cx = cc >> 2, cy = (cc >> 1) & 1, cz = cc & 1;
    off[cc] = ax[cx] + ay[cy] + az[cz];
    w[cc] = ((cx ? t[0] : u[0]) * (cy ? t[1] : u[1])) * (cz ? t[2] : u[2]);
  }
}

// FP64 form: x in [0, L) Mpc.
template <bool TSC, typename I>
__device__ __forceinline__ void stencil_f64(const double* x, double ginv, int gm, I G,
                                            I* cell, double* w) {
#pragma clang fp contract(off)
  if constexpr (!TSC) {
    int i0[3], i1[3];
    double t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = x[d] * ginv;
      const double fl = floor(u);
      t[d] = u - fl;
      i0[d] = ((int)fl) & gm;
      i1[d] = (i0[d] + 1) & gm;
    }
    const I ax[2] = {(I)mesh_x((uint32_t)i0[0], (uint32_t)G), (I)mesh_x((uint32_t)i1[0], (uint32_t)G)};
    const I ay[2] = {(I)mesh_y((uint32_t)i0[1], (uint32_t)G), (I)mesh_y((uint32_t)i1[1], (uint32_t)G)};
    const I az[2] = {(I)mesh_z((uint32_t)i0[2]), (I)mesh_z((uint32_t)i1[2])};
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc >> 2, cy = (cc >> 1) & 1, cz = cc & 1;
      cell[cc] = ax[cx] + ay[cy] + az[cz];
      w[cc] = ((cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1])) * (cz ? t[2] : 1.0 - t[2]);
    }
  } else {
    int idx[3][3];
    double wt[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = x[d] * ginv;
      const double fl = floor(u + 0.5);
      const double dd = u - fl;                         // in [-1/2, 1/2)
      const int i = ((int)fl) & gm;
      idx[d][0] = (i - 1) & gm;
      idx[d][1] = i;
      idx[d][2] = (i + 1) & gm;
      wt[d][0] = 0.5 * ((0.5 - dd) * (0.5 - dd));
      wt[d][1] = 0.75 - dd * dd;
      wt[d][2] = 0.5 * ((0.5 + dd) * (0.5 + dd));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cell[9 * a + 3 * b + c] = (I)mesh_x((uint32_t)idx[0][a], (uint32_t)G) +
                                    (I)mesh_y((uint32_t)idx[1][b], (uint32_t)G) + (I)mesh_z((uint32_t)idx[2][c]);
          w[9 * a + 3 * b + c] = (wt[0][a] * wt[1][b]) * wt[2][c];
        }
  }
}

}  // namespace push_detail
}  // namespace fdf
