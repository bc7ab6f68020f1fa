// Spatial bucket sort of the particle state (gfx950).
//
// Order = Morton index of the coarse T^3-cell tile holding the particle (the
// bucket of a counting sort), then the Morton index of its cell inside the
// tile.  Rank pass: each block of 1024 particles sorts itself by that key in
// LDS and reserves one contiguous range per bucket it touches (one atomic per
// block and bucket).  Scan: bucket counts become bucket starts.  Move pass:
// every state array goes to start + rank in the other buffer copy (in the
// FP32 separable form the push of the step does this instead, writing its
// updated state in sorted order: k_push_sort_f32).  Within a
// bucket the fragments of different blocks follow each other in arbitrary
// order, each sorted by cell.  The push is per particle, so results do not
// depend on the order.  Particles keep their id.
#include "fdf_device.h"
#include "fdf_internal.h"
#include "fdf_key.h"

namespace fdf {
namespace {

using namespace sort_key;

// The species a rank block belongs to: its state arrays, prediction and
// outputs (one species, or one job of a batched re-sort).
struct RankView {
  const uint32_t* xu[3];
  const float* q0f[3];
  const float* dqf[3];
  const double* xd[3];
  const double* qd[3];
  int64_t n;
  double tau, ma;
  const uint32_t* keys;    // precomputed keys of the species' particles, or null
  uint32_t* count;
  uint32_t* rank;
  uint32_t* bucket;
  uint32_t* src;
};

__device__ __forceinline__ RankView view_of(const Segment& g, double tau, double ma, const uint32_t* keys,
                                            uint32_t* count, uint32_t* rank, uint32_t* bucket, uint32_t* src) {
  RankView v;
  v.keys = keys;
  for (int d = 0; d < 3; ++d) {
    v.xu[d] = g.xu[d]; v.q0f[d] = g.q0f[d]; v.dqf[d] = g.dqf[d]; v.xd[d] = g.xd[d]; v.qd[d] = g.qd[d];
  }
  v.n = g.n;
  v.tau = tau;
  v.ma = ma;
  v.count = count;
  v.rank = rank;
  v.bucket = bucket;
  v.src = src;
  return v;
}

// Full key of particle i: Morton index of its coarse tile (the counting-sort
// bucket) above the Morton index of its cell inside the tile.  The position
// is extrapolated along the particle's current velocity to the middle of the
// interval until the next re-sort: neighbours in that order stay within half
// an interval's drift of each other over the whole interval, instead of a
// whole interval's drift by its end.
__device__ __forceinline__ uint32_t full_key(const SortArgs& a, const RankView& g, int64_t i) {
  if (g.keys) return g.keys[i];   // written by the push before this re-sort
  if (a.fp64) {
    uint32_t c[3];
    const double s = (double)a.grid_n / a.box;
    double v[3] = {0.0, 0.0, 0.0};
    if (g.tau != 0.0) {
      const double q[3] = {g.qd[0][i], g.qd[1][i], g.qd[2][i]};
      const double f = g.tau / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + g.ma * g.ma);
      for (int d = 0; d < 3; ++d) v[d] = q[d] * f;
    }
    for (int d = 0; d < 3; ++d)
      c[d] = (uint32_t)(int64_t)floor((g.xd[d][i] + v[d]) * s) & (uint32_t)(a.grid_n - 1);
    return morton_key(c, a.fine_bits);
  }
  const uint32_t x[3] = {g.xu[0][i], g.xu[1][i], g.xu[2][i]};
  float q[3] = {0.0f, 0.0f, 0.0f};
  if (g.tau != 0.0)
    for (int d = 0; d < 3; ++d) q[d] = g.q0f[d][i] + g.dqf[d][i];
  return key_f32(x, q, (float)g.ma, (float)(g.tau * 4294967296.0 / a.box), g.tau != 0.0, a.cell_shift,
                 a.fine_bits);
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so each XCD (own
// L2) takes a contiguous range of particles: the bucket fragments written by
// neighbouring blocks then merge into whole lines in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t full = nb - nb % 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

constexpr int kRankThreads = 256;
constexpr int kRankBlock = kSortBlock;    // particles per block
constexpr uint64_t kIdxMask = kRankBlock - 1;
constexpr uint64_t kNoKey = 0xFFFFFFFFull;      // sorts after every key (at most 30 bits)



__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Value of lane (this lane xor mask).  The network's masks are compile-time
// constants after unrolling: 1 and 2 are quad permutations and 4 and 8 two row
// shifts and a select, all DPP moves on the vector ALU; 16 is a swizzle inside
// 32 lanes; only 32 goes through the LDS crossbar (bpermute).  Row shifts: lane
// i of row_shl:n reads lane i + n of its row of 16, row_shr:n lane i - n.
__device__ __forceinline__ uint32_t shfl_xor_word(uint32_t v, int mask) {
  const int x = (int)v;
  if (mask == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  if (mask == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  if (mask == 4) {
    const int up = __builtin_amdgcn_mov_dpp(x, 0x104, 0xF, 0xF, false);   // row_shl:4
    const int dn = __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, false);   // row_shr:4
    return (uint32_t)((__lane_id() & 4) ? dn : up);
  }
  if (mask == 8) {
    const int up = __builtin_amdgcn_mov_dpp(x, 0x108, 0xF, 0xF, false);   // row_shl:8
    const int dn = __builtin_amdgcn_mov_dpp(x, 0x118, 0xF, 0xF, false);   // row_shr:8
    return (uint32_t)((__lane_id() & 8) ? dn : up);
  }
  if (mask == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);   // and 0x1f, xor 0x10
  return (uint32_t)__shfl_xor(x, mask, 64);
}
__device__ __forceinline__ uint64_t shfl_xor_word(uint64_t v, int mask) {
  return ((uint64_t)shfl_xor_word((uint32_t)(v >> 32), mask) << 32) | shfl_xor_word((uint32_t)v, mask);
}

// Bitonic sort of the block's 1024 words, thread t holding sorted positions
// 4t .. 4t + 3 in registers.  Element e = 4 tid + r keeps the smaller of its
// pair exactly when it is the lower index of an ascending pair or the upper
// index of a descending one.  Real words are unique (the slot is in the low
// bits; equal padding words are interchangeable), so one comparison decides:
// take the partner's word when (partner < own) == keep_min.  For partners 4
// or more apart, both bits of e that decide keep_min are bits of tid, so the
// direction is one per thread and stage.  Partners within a thread swap in
// registers, partners within a wave meet through lane shuffles, and only the
// three stages that cross waves go through LDS (lds: kRankBlock words).
template <typename W>
__device__ __forceinline__ void bitonic_block(W (&v)[4], W* lds, int tid) {
#pragma unroll
  for (int k = 2; k <= kRankBlock; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 4) {
        const bool upper = (tid & (j >> 2)) != 0;
        const bool desc = k < kRankBlock && (tid & (k >> 2)) != 0;
        const bool keep_min = upper == desc;
        if (j >= 4 * 64) {               // partner in another wave
          __syncthreads();
#pragma unroll
          for (int r = 0; r < 4; ++r) lds[4 * tid + r] = v[r];
          __syncthreads();
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const W w = lds[(4 * tid + r) ^ j];
            v[r] = ((w < v[r]) == keep_min) ? w : v[r];
          }
        } else {                         // partner in another lane of the wave
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const W w = shfl_xor_word(v[r], j >> 2);
            v[r] = ((w < v[r]) == keep_min) ? w : v[r];
          }
        }
      } else {                           // partner in this thread
        // bit k of e: a bit of r for k < 4, of tid above (none for the last merge)
        const bool up = k == kRankBlock || (tid & (k >> 2)) == 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r & j) continue;
          const bool asc = k < 4 ? (r & k) == 0 : up;
          const W x = v[r], y = v[r + j];
          if ((x > y) == asc) { v[r] = y; v[r + j] = x; }
        }
      }
    }
  }
}

// Rank pass.  A block sorts its 1024 particles by (full key, slot) (bitonic,
// above), cuts the sorted run into segments of equal bucket, and reserves one
// contiguous range per segment with a single atomicAdd on the bucket count.
// For each element of the block's sorted run its source slot, bucket and rank
// inside the bucket are written at its sorted position.  The fragment a block
// writes into a bucket is therefore contiguous and ordered by cell.
// When the block's keys span less than 2^22 (spatially compact blocks, the
// common case once sorted), the network runs on 32-bit words of (key - the
// block's smallest key, slot), half the work of the 64-bit words.
__device__ __forceinline__ void rank_block(const SortArgs& a, const RankView& g, int64_t blk) {
  static_assert(kRankBlock == 4 * kRankThreads, "four elements per thread");
  __shared__ uint64_t kv[kRankBlock];
  __shared__ uint32_t seg_start[kRankBlock];
  __shared__ uint32_t seg_base[kRankBlock];
  __shared__ uint32_t wave_max[kRankThreads / 64];
  __shared__ uint64_t wave_kmin[kRankThreads / 64], wave_kmax[kRankThreads / 64];
  const int64_t i0 = blk * kRankBlock;
  const int cnt = (int)min<int64_t>(kRankBlock, g.n - i0);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  // keys read coalesced (element tid + 256 r)
  uint64_t key[4];
  uint64_t kmin = ~0ull, kmax = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = tid + kRankThreads * r;
    key[r] = e < cnt ? (uint64_t)full_key(a, g, i0 + e) : kNoKey;
    if (e < cnt) { kmin = min(kmin, key[r]); kmax = max(kmax, key[r]); }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    kmin = min(kmin, shfl_xor_u64(kmin, off));
    kmax = max(kmax, shfl_xor_u64(kmax, off));
  }
  if (lane == 0) { wave_kmin[wid] = kmin; wave_kmax[wid] = kmax; }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kRankThreads / 64; ++w) { kmin = min(kmin, wave_kmin[w]); kmax = max(kmax, wave_kmax[w]); }
  if (kmax - kmin < (1ull << 22)) {      // block-uniform (cnt >= 1, so kmin <= kmax)
    uint32_t* kw = (uint32_t*)kv;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + kRankThreads * r;
      kw[e] = e < cnt ? ((uint32_t)(key[r] - kmin) << 10) | (uint32_t)e : 0xFFFFFFFFu;
    }
    __syncthreads();
    uint32_t v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = kw[4 * tid + r];
    bitonic_block(v, kw, tid);
    __syncthreads();
    // back to (key, slot) words; the padding sorts to positions >= cnt
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 4 * tid + r;
      kv[pos] = pos < cnt ? ((kmin + (v[r] >> 10)) << 10) | (uint64_t)(v[r] & (uint32_t)kIdxMask)
                          : (kNoKey << 10) | (uint64_t)pos;
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + kRankThreads * r;
      kv[e] = (key[r] << 10) | (uint64_t)e;
    }
    __syncthreads();
    uint64_t v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = kv[4 * tid + r];
    bitonic_block(v, kv, tid);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) kv[4 * tid + r] = v[r];
    __syncthreads();
  }
  // segment starts: inclusive max-scan of head positions over the sorted run;
  // thread tid owns sorted elements 4 tid .. 4 tid + 3
  const int sh = 10 + 3 * a.fine_bits;   // key bits below the bucket index
  uint32_t loc[4];
  uint32_t m = 0;
  for (int r = 0; r < 4; ++r) {
    const int e = 4 * tid + r;
    const bool head = e == 0 || (kv[e] >> sh) != (kv[e - 1] >> sh);
    m = head ? (uint32_t)e : m;
    loc[r] = m;
  }
  uint32_t inc = m;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
    if (lane >= off) inc = max(inc, y);
  }
  if (lane == 63) wave_max[wid] = inc;
  __syncthreads();
  uint32_t carry = (uint32_t)__shfl_up((int)inc, 1, 64);
  if (lane == 0) carry = 0;
  for (int w = 0; w < wid; ++w) carry = max(carry, wave_max[w]);
  for (int r = 0; r < 4; ++r) {
    const uint32_t st = max(loc[r], carry);
    seg_start[4 * tid + r] = st;
    carry = max(carry, loc[r]);
  }
  __syncthreads();
  // the last element of each segment reserves the segment's range
  for (int r = 0; r < 4; ++r) {
    const int e = 4 * tid + r;
    const uint64_t key = kv[e] >> 10;
    const bool last = e == kRankBlock - 1 || (kv[e + 1] >> sh) != (kv[e] >> sh);
    if (last && key != kNoKey) {
      const uint32_t st = seg_start[e];
      seg_base[st] = atomicAdd(&g.count[(uint32_t)(key >> (3 * a.fine_bits))], (uint32_t)(e - st + 1));
    }
  }
  __syncthreads();
  // outputs in sorted order: source slot, bucket and rank of sorted element e
  for (int r = 0; r < 4; ++r) {
    const int e = 4 * tid + r;
    const uint64_t key = kv[e] >> 10;
    const int64_t o = i0 + e;
    if (o >= g.n) continue;   // sentinels sort last: e < n - i0 holds real particles
    const uint32_t st = seg_start[e];
    g.src[o] = (uint32_t)(kv[e] & kIdxMask);
    g.rank[o] = seg_base[st] + (uint32_t)(e - st);
    g.bucket[o] = (uint32_t)(key >> (3 * a.fine_bits));
  }
}

// One species (batch.njobs == 0), or one block of a batched re-sort.
__global__ void __launch_bounds__(kRankThreads) k_sort_rank(SortArgs a) {
  if (a.batch.njobs == 0) {
    rank_block(a, view_of(a.seg, a.predict_tau, a.ma, a.keys, a.count, a.rank, a.bucket, a.src),
               xcd_block(blockIdx.x, gridDim.x));
    return;
  }
  int64_t local;
  const int j = batch_block(a.batch, blockIdx.x, &local);
  if (j < 0) return;
  const SortBatch& b = a.batch;
  const Segment& g = b.tables[b.job_cur[j]][b.job_species[j]];
  const int64_t base = b.job_base[j];
  rank_block(a, view_of(g, b.job_tau[j], b.job_ma[j], a.keys ? a.keys + base : nullptr, a.count + j * a.nkeys,
                        a.rank + base, a.bucket + base, a.src + base), local);
}

// Move pass, one 1024-block at a time and one state array at a time: the
// block's window of the array is read once, coalesced, into LDS; element e of
// the sorted order then takes source slot src[e] from LDS and is written to
// start[bucket] + rank, so consecutive threads write consecutive addresses
// inside each bucket fragment.
template <typename T>
__device__ __forceinline__ void move_array(const T* __restrict__ src, T* __restrict__ dst, T* lds,
                                           int64_t i0, int cnt, const int* sidx, const uint32_t* pos) {
  for (int e = threadIdx.x; e < cnt; e += 256) lds[e] = src[i0 + e];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRankBlock / 256; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < cnt) dst[pos[r]] = lds[sidx[r]];
  }
  __syncthreads();
}

// Two 4-byte arrays per LDS round (the same 8 KB as one 8-byte array).
__device__ __forceinline__ void move_pair(const uint32_t* __restrict__ s0, uint32_t* __restrict__ d0,
                                          const uint32_t* __restrict__ s1, uint32_t* __restrict__ d1,
                                          uint32_t* lds, int64_t i0, int cnt, const int* sidx,
                                          const uint32_t* pos) {
  for (int e = threadIdx.x; e < cnt; e += 256) {
    lds[e] = s0[i0 + e];
    lds[kRankBlock + e] = s1[i0 + e];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRankBlock / 256; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < cnt) {
      d0[pos[r]] = lds[sidx[r]];
      d1[pos[r]] = lds[kRankBlock + sidx[r]];
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_sort_move(SortArgs a) {
  __shared__ uint64_t lds_raw[kRankBlock];
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i0 = blk * kRankBlock;
  const int cnt = (int)min<int64_t>(kRankBlock, a.seg.n - i0);
  int sidx[kRankBlock / 256];
  uint32_t pos[kRankBlock / 256];
#pragma unroll
  for (int r = 0; r < kRankBlock / 256; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < cnt) {
      const int64_t o = i0 + e;
      sidx[r] = (int)a.src[o];
      pos[r] = a.count[a.bucket[o]] + a.rank[o];
    }
  }
  const Segment& s = a.seg;
  const Segment& d = a.dst;
  if (a.id_only) {
    move_array(s.id, d.id, (uint32_t*)lds_raw, i0, cnt, sidx, pos);
  } else if (a.fp64) {
    double* l = (double*)lds_raw;
    for (int k = 0; k < 3; ++k) {
      move_array(s.xd[k], d.xd[k], l, i0, cnt, sidx, pos);
      move_array(s.qd[k], d.qd[k], l, i0, cnt, sidx, pos);
      move_array(s.q0d[k], d.q0d[k], l, i0, cnt, sidx, pos);
    }
    move_array(s.id, d.id, (uint32_t*)lds_raw, i0, cnt, sidx, pos);
  } else {
    uint32_t* l = (uint32_t*)lds_raw;
    const uint32_t* sa[10] = {s.xu[0], s.xu[1], s.xu[2],
                              (const uint32_t*)s.q0f[0], (const uint32_t*)s.q0f[1], (const uint32_t*)s.q0f[2],
                              (const uint32_t*)s.dqf[0], (const uint32_t*)s.dqf[1], (const uint32_t*)s.dqf[2], s.id};
    uint32_t* da[10] = {d.xu[0], d.xu[1], d.xu[2], (uint32_t*)d.q0f[0], (uint32_t*)d.q0f[1],
                        (uint32_t*)d.q0f[2], (uint32_t*)d.dqf[0], (uint32_t*)d.dqf[1], (uint32_t*)d.dqf[2], d.id};
#pragma unroll
    for (int k = 0; k < 10; k += 2) move_pair(sa[k], da[k], sa[k + 1], da[k + 1], l, i0, cnt, sidx, pos);
  }
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

void launch_sort_rank(const SortArgs& a, hipStream_t s) {
  const int64_t n = a.seg.n;
  launch_fill_zero(a.count, ((size_t)a.nkeys * 4 + 15) / 16 * 16, s);
  hipLaunchKernelGGL(k_sort_rank, dim3((unsigned)((n + kRankBlock - 1) / kRankBlock)), dim3(kRankThreads), 0, s, a);
  scan_exclusive(a.count, a.nkeys, a.scan_scratch, s);   // bucket counts -> bucket starts
}

// Batched rank pass: counts of every job cleared, ranked, scanned together.
void launch_sort_rank_batch(const SortArgs& a, hipStream_t s) {
  const int64_t keys = a.nkeys * a.batch.njobs;
  launch_fill_zero(a.count, ((size_t)keys * 4 + 15) / 16 * 16, s);
  hipLaunchKernelGGL(k_sort_rank, dim3((unsigned)batch_grid(a.batch)), dim3(kRankThreads), 0, s, a);
  scan_exclusive(a.count, keys, a.scan_scratch, s);
}

void launch_sort(const SortArgs& a, hipStream_t s) {
  const int64_t n = a.seg.n;
  launch_sort_rank(a, s);
  hipLaunchKernelGGL(k_sort_move, dim3((unsigned)((n + kRankBlock - 1) / kRankBlock)), dim3(256), 0, s, a);
}

}  // namespace fdf
