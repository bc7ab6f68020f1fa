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

__device__ __forceinline__ int find_segment(const Segment* seg, int nseg, int64_t chunk) {
  int s = 0;
  while (s + 1 < nseg && seg[s + 1].chunk_begin <= chunk) ++s;
  return s;
}

template <typename T> __device__ __forceinline__ T ldnt(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void stnt(T v, T* p) { __builtin_nontemporal_store(v, p); }

}  // namespace push_detail
}  // namespace fdf
