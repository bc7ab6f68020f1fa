// Spatial bucket sort of the particle state (gfx950).
//
// Key = Morton index of the T^3-cell tile holding the particle, taken from the
// top bits of the position.  A counting sort: count particles per key, an
// exclusive scan of the counts, then a scatter of every state array into the
// other buffer copy.  Both atomic passes aggregate runs of equal keys within a
// 64-lane wavefront (nearly sorted input has long runs), so one lane per run
// issues the atomic.  The order inside a tile is arbitrary; the push is per
// particle, so results do not depend on it.  Particles keep their id.
#include "fdf_device.h"
#include "fdf_internal.h"

namespace fdf {
namespace {

__device__ __forceinline__ uint32_t part1by2(uint32_t v) {   // spread 10 bits to every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t tile_key(const SortArgs& a, int64_t i) {
  uint32_t t[3];
  if (a.fp64) {
    const double s = (double)a.tiles / a.box;
    for (int d = 0; d < 3; ++d) t[d] = (uint32_t)(int64_t)floor(a.seg.xd[d][i] * s) & (uint32_t)(a.tiles - 1);
  } else {
    for (int d = 0; d < 3; ++d) t[d] = a.seg.xu[d][i] >> a.shift;
  }
  return (part1by2(t[0]) << 2) | (part1by2(t[1]) << 1) | part1by2(t[2]);
}

struct WaveRun {
  int leader;   // lane that starts this lane's run
  int len;      // run length (valid on leaders)
};

// Runs of equal keys among the active lanes of a wavefront.
__device__ __forceinline__ WaveRun wave_runs(uint32_t key, bool active) {
  const int lane = threadIdx.x & 63;
  const uint32_t kprev = (uint32_t)__shfl_up((int)key, 1, 64);
  const bool start = active && (lane == 0 || kprev != key);
  const uint64_t smask = __ballot(start);
  const uint64_t bmask = __ballot(start || !active);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t above = bmask & ~upto;
  const int end = above ? __ffsll((unsigned long long)above) - 1 : 64;
  WaveRun r;
  r.len = end - lane;
  const uint64_t below = smask & upto;
  r.leader = below ? 63 - __clzll(below) : lane;
  return r;
}

__global__ void k_sort_count(SortArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < a.seg.n;
  const uint32_t key = active ? tile_key(a, i) : 0xFFFFFFFFu;
  const WaveRun r = wave_runs(key, active);
  if (active && r.leader == (int)(threadIdx.x & 63)) atomicAdd(&a.count[key], (uint32_t)r.len);
}

template <typename T>
__device__ __forceinline__ void move(const T* src, T* dst, int64_t i, uint32_t pos) { dst[pos] = src[i]; }

__global__ void k_sort_scatter(SortArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < a.seg.n;
  const uint32_t key = active ? tile_key(a, i) : 0xFFFFFFFFu;
  const WaveRun r = wave_runs(key, active);
  const int lane = threadIdx.x & 63;
  uint32_t base = 0;
  if (active && r.leader == lane) base = atomicAdd(&a.offset[key], (uint32_t)r.len);
  base = (uint32_t)__shfl((int)base, r.leader, 64);
  if (!active) return;
  const uint32_t pos = base + (uint32_t)(lane - r.leader);
  const Segment& s = a.seg;
  const Segment& d = a.dst;
  for (int k = 0; k < 3; ++k) {
    if (a.fp64) {
      move(s.xd[k], d.xd[k], i, pos);
      move(s.qd[k], d.qd[k], i, pos);
      move(s.q0d[k], d.q0d[k], i, pos);
    } else {
      move(s.xu[k], d.xu[k], i, pos);
      move(s.qf[k], d.qf[k], i, pos);
      move(s.cf[k], d.cf[k], i, pos);
      move(s.q0f[k], d.q0f[k], i, pos);
    }
  }
  move(s.id, d.id, i, pos);
}

// ------------------------------------------------- exclusive scan (uint32) --
constexpr int kScanBlock = 1024;   // threads
constexpr int kScanItems = 4;      // items per thread

// Exclusive scan of each block's 4096 items in place; block totals to sums.
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(uint32_t* data, int64_t n, uint32_t* sums) {
  __shared__ uint32_t warp_tot[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems], tot = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? data[base + k] : 0u;
    tot += v[k];
  }
  // inclusive scan of thread totals across the wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = tot;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) warp_tot[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < kScanBlock / 64 ? warp_tot[lane] : 0u;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)w, off, 64);
      if (lane >= off) w += y;
    }
    if (lane < kScanBlock / 64) warp_tot[lane] = w;   // inclusive over waves
  }
  __syncthreads();
  uint32_t run = inc - tot + (wid ? warp_tot[wid - 1] : 0u);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) data[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1 && sums) sums[blockIdx.x] = run;
}

__global__ void k_scan_add(uint32_t* data, int64_t n, const uint32_t* sums) {
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) data[i] += sums[i / per];
}

void scan_exclusive(uint32_t* data, int64_t n, uint32_t* scratch, hipStream_t s) {
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  const int64_t nb = (n + per - 1) / per;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, data, n, (uint32_t*)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanBlock), 0, s, data, n, scratch);
  scan_exclusive(scratch, nb, scratch + nb, s);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, data, n, scratch);
}

}  // namespace

size_t sort_scan_scratch_words(int64_t nkeys) {
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  size_t words = 0;
  for (int64_t n = nkeys; n > 1; n = (n + per - 1) / per) words += (size_t)((n + per - 1) / per) + 1;
  return words + 16;
}

void launch_sort(const SortArgs& a, hipStream_t s) {
  const int64_t n = a.seg.n;
  const unsigned grid = (unsigned)((n + 255) / 256);
  launch_fill_zero(a.count, ((size_t)a.nkeys * 4 + 15) / 16 * 16, s);
  hipLaunchKernelGGL(k_sort_count, dim3(grid), dim3(256), 0, s, a);
  scan_exclusive(a.count, a.nkeys, a.scan_scratch, s);
  SortArgs b = a;
  b.offset = a.count;   // the scanned counts are the bucket starts
  hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(256), 0, s, b);
}

}  // namespace fdf
