// Gather + kick-drift-kick push of the neutrino tracers (sec. 3.3), gfx950.
//
// One launch advances every species by one leapfrog step: the kick of the
// closing half of step k-1 and the opening half of step k are evaluated at the
// same (x_k, a_k), so they are applied as one kick with the summed Delta tau;
// then the drift.  The last launch of a call is a kick alone, leaving q at a
// schedule point.
//
// Per particle: CIC (trilinear; or TSC, 27 points, when PushArgs::tsc is set)
// interpolation of the gradient grids at x,
//   F = -eps0 grad psi - (q0^2/eps0) grad phi + q0 (q0 . grad phi)/eps0 + q0 phidot
//   (eq. releq_approx, eps0 = sqrt(q0^2 + m^2 a^2)),
//   q += kick * F,  x += drift * q / sqrt(q^2 + m^2 a_{k+1/2}^2)   (eq. discrete_drift).
//
// FP32 form: x is a uint32 fixed-point fraction of the box per axis, so the
// periodic wrap is integer overflow and the cell index is the top log2(G)
// bits; the momentum is q = q0 + dq with the accumulated kicks dq in binary32
// (the kicks only ever add to dq, whose rounding is relative to dq, not q);
// grids are bfloat16 with 8, 6 or 4 slots = one 16-, 12- or 8-byte load per
// CIC corner.
// FP64 form: everything binary64; 8 slots = four 16-byte loads per corner.
//
// Blocks take contiguous chunks of one species, in an XCD-aware order (with
// several species, every XCD takes an eighth of each).  On a step that begins
// with a re-sort, k_push_sort_f32 pushes the species due (one launch for all
// of them) and writes their updated state straight to their sorted slots; the
// plain push of the step before can also write their sort keys.
//
// The separable form is the one implemented here; the other equations of
// motion (fdf_push_eom.hip) take over when PushArgs::eom is set.
#include "fdf_push_common.h"
#include "fdf_key.h"

namespace fdf {
namespace {

using namespace push_detail;

// Gather of the slots from a bfloat16 grid: 8-slot cells hold gpsi[3],
// gphi[3], phidot and a pad (16 bytes), 6-slot cells gpsi[3], gphi[3] with
// phidot = 0 (12 bytes), 4-slot cells gpsi[3], phidot with phi = psi (8 bytes).
struct Cell12 { uint32_t x, y, z; };
template <int NSLOT> struct CellType { using T = uint4; };
template <> struct CellType<6> { using T = Cell12; };
template <> struct CellType<4> { using T = uint2; };

// OFF32: the mesh spans less than 4 GiB, so a corner is addressed as a
// uniform base plus a 32-bit byte offset (one VGPR per corner instead of a
// 64-bit address).
template <typename V, bool OFF32>
__device__ __forceinline__ V load_cell(const void* grid, uint32_t cell) {
  if constexpr (OFF32) {
    const char FDF_GLOBAL* b = (const char FDF_GLOBAL*)grid;
    return *(const FDF_GLOBAL V*)(b + cell * (uint32_t)sizeof(V));
  } else {
    return ((const FDF_GLOBAL V*)grid)[(size_t)cell];
  }
}

// g += w * (the slots of one cell), slot by slot.
template <int NSLOT, typename V>
__device__ __forceinline__ void accum_cell_bf16(float w, const V& v, float* g) {
#pragma clang fp contract(off)
  if constexpr (NSLOT == 8) {
    g[0] = fmaf(w, bf16_lo(v.x), g[0]); g[1] = fmaf(w, bf16_hi(v.x), g[1]);
    g[2] = fmaf(w, bf16_lo(v.y), g[2]); g[3] = fmaf(w, bf16_hi(v.y), g[3]);
    g[4] = fmaf(w, bf16_lo(v.z), g[4]); g[5] = fmaf(w, bf16_hi(v.z), g[5]);
    g[6] = fmaf(w, bf16_lo(v.w), g[6]);
  } else if constexpr (NSLOT == 6) {
    g[0] = fmaf(w, bf16_lo(v.x), g[0]); g[1] = fmaf(w, bf16_hi(v.x), g[1]);
    g[2] = fmaf(w, bf16_lo(v.y), g[2]); g[3] = fmaf(w, bf16_hi(v.y), g[3]);
    g[4] = fmaf(w, bf16_lo(v.z), g[4]); g[5] = fmaf(w, bf16_hi(v.z), g[5]);
  } else {
    g[0] = fmaf(w, bf16_lo(v.x), g[0]); g[1] = fmaf(w, bf16_hi(v.x), g[1]);
    g[2] = fmaf(w, bf16_lo(v.y), g[2]); g[6] = fmaf(w, bf16_hi(v.y), g[6]);
  }
}

template <int NSLOT, int NPT, bool OFF32>
__device__ __forceinline__ void gather_bf16(const void* grid, const uint32_t* cell, const float* w,
                                            float* g /* 7, accumulated */) {
  using V = typename CellType<NSLOT>::T;
  V v[NPT];
#pragma unroll
  for (int c = 0; c < NPT; ++c) v[c] = load_cell<V, OFF32>(grid, cell[c]);
#pragma unroll
  for (int c = 0; c < NPT; ++c) accum_cell_bf16<NSLOT>(w[c], v[c], g);
}

// Gather over a whole stencil: CIC in one batch of 8 loads, TSC in three
// batches of 9 (one x-plane of the 27 points each).
template <int NSLOT, bool TSC, bool OFF32>
__device__ __forceinline__ void gather_stencil_bf16(const void* grid, const uint32_t* cell, const float* w, float* g) {
  if constexpr (TSC) {
#pragma unroll
    for (int b = 0; b < 3; ++b) gather_bf16<NSLOT, 9, OFF32>(grid, cell + 9 * b, w + 9 * b, g);
  } else {
    gather_bf16<NSLOT, 8, OFF32>(grid, cell, w, g);
  }
}

// Launch constants of the FP32 update of one segment.
struct ConstF32 {
  int shift;
  uint32_t gmask, G;
  float finv, kick, ma2, mah2, dscale, ta, tb;
  const void* gridA;
  const void* gridB;
};

template <bool BLEND>
__device__ __forceinline__ ConstF32 const_f32(const PushArgs& a, const Segment& sg) {
  ConstF32 k;
  k.shift = 32 - a.log2g;
  k.gmask = (uint32_t)a.G - 1u;
  k.G = (uint32_t)a.G;
  k.finv = __uint_as_float((uint32_t)(127 - k.shift) << 23);   // 2^-shift
  k.kick = (float)a.kick;
  const float ma = (float)(sg.m * a.a_kick);
  const float mah = (float)(sg.m * a.a_drift);
  k.ma2 = ma * ma;
  k.mah2 = mah * mah;
  k.dscale = (float)(a.drift * 4294967296.0 / a.box);
  k.gridA = (BLEND && a.grid_sel) ? sg.grid2 : sg.grid;
  k.gridB = (BLEND && a.grid_sel) ? sg.grid : sg.grid2;
  k.tb = (float)a.blend_t;
  k.ta = 1.0f - k.tb;
  return k;
}

// The kick and drift of one particle from its interpolated mesh values g.
template <int NSLOT>
__device__ __forceinline__ void kick_drift_f32(const ConstF32& k, bool drift, float* g, uint32_t* xu,
                                               const float* q0, float* dq) {
#pragma clang fp contract(off)
  if (NSLOT == 4) { g[3] = g[0]; g[4] = g[1]; g[5] = g[2]; }
  // separable force of eq. releq_approx
  // 1/eps from the hardware reciprocal square root (about 1 ulp; the bf16
  // mesh dominates the error budget of this form by four orders of magnitude)
  const float q0sq = fmaf(q0[0], q0[0], fmaf(q0[1], q0[1], q0[2] * q0[2]));
  const float e02 = q0sq + k.ma2;
  const float ie0 = __builtin_amdgcn_rsqf(e02);
  const float e0 = e02 * ie0;
  const float q0g = fmaf(q0[0], g[3], fmaf(q0[1], g[4], q0[2] * g[5]));
  const float qg = fmaf(q0g, ie0, g[6]);          // (q0 . grad phi)/eps0 + phidot
  const float cphi = q0sq * ie0;                    // q0^2 / eps0
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float F = fmaf(q0[d], qg, fmaf(-cphi, g[3 + d], -(e0 * g[d])));
    dq[d] = fmaf(k.kick, F, dq[d]);
  }
  if (drift) {
    float q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) q[d] = q0[d] + dq[d];
    const float qq = fmaf(q[0], q[0], fmaf(q[1], q[1], q[2] * q[2]));
    const float ie = __builtin_amdgcn_rsqf(qq + k.mah2);
#pragma unroll
    for (int d = 0; d < 3; ++d) xu[d] += (uint32_t)__float2int_rn(k.dscale * (q[d] * ie));
  }
}

// The FP32 update of one particle: gather, separable kick into dq, drift of
// the fixed-point position.  Every floating-point operation is written out
// (explicit fmaf, no contraction) so that every copy of this code is
// instruction-identical: a particle gets bit-identical results in whichever
// slot of whichever block, and whichever kernel, it is updated.
template <int NSLOT, bool BLEND, bool TSC, bool OFF32>
__device__ __forceinline__ void update_f32(const ConstF32& k, bool drift, uint32_t* xu, const float* q0,
                                           float* dq) {
#pragma clang fp contract(off)
  constexpr int NP = Stencil<TSC>::N;
  uint32_t cell[NP];
  float w[NP];
  stencil_u32<TSC>(xu, k.shift, k.gmask, k.finv, k.G, cell, w);
  float g[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (BLEND) {   // super-steps: (1 - t) G_A + t G_B folded into the weights
    float wa[NP], wb[NP];
#pragma unroll
    for (int cc = 0; cc < NP; ++cc) { wa[cc] = k.ta * w[cc]; wb[cc] = k.tb * w[cc]; }
    gather_stencil_bf16<NSLOT, TSC, OFF32>(k.gridA, cell, wa, g);
    gather_stencil_bf16<NSLOT, TSC, OFF32>(k.gridB, cell, wb, g);
  } else {
    gather_stencil_bf16<NSLOT, TSC, OFF32>(k.gridA, cell, w, g);
  }
  kick_drift_f32<NSLOT>(k, drift, g, xu, q0, dq);
}

// The CIC update of GRP particles at once: all their gathers are issued
// before any is consumed, so GRP corner sets are in flight together instead
// of one particle's at a time.  Each particle's arithmetic is the same, in the
// same order, as update_f32's.
template <int NSLOT, int GRP, bool OFF32>
__device__ __forceinline__ void update_group_f32(const ConstF32& k, bool drift, uint32_t (*xu)[3],
                                                 const float (*q0)[3], float (*dq)[3]) {
#pragma clang fp contract(off)
  using V = typename CellType<NSLOT>::T;
  uint32_t cell[GRP][8];
  float w[GRP][8];
  V v[GRP][8];
  if constexpr (OFF32) {   // byte offsets straight from the stencil
    const uint32_t lg = 32u - (uint32_t)k.shift;
#pragma unroll
    for (int p = 0; p < GRP; ++p)
      stencil_u32_bytes<(uint32_t)sizeof(V)>(xu[p], k.shift, k.gmask, k.finv, lg, cell[p], w[p]);
    const char FDF_GLOBAL* b = (const char FDF_GLOBAL*)k.gridA;
#pragma unroll
    for (int p = 0; p < GRP; ++p)
#pragma unroll
      for (int c = 0; c < 8; ++c) v[p][c] = *(const FDF_GLOBAL V*)(b + cell[p][c]);
  } else {
#pragma unroll
    for (int p = 0; p < GRP; ++p) stencil_u32<false>(xu[p], k.shift, k.gmask, k.finv, k.G, cell[p], w[p]);
#pragma unroll
    for (int p = 0; p < GRP; ++p)
#pragma unroll
      for (int c = 0; c < 8; ++c) v[p][c] = load_cell<V, OFF32>(k.gridA, cell[p][c]);
  }
#pragma unroll
  for (int p = 0; p < GRP; ++p) {
    float g[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) accum_cell_bf16<NSLOT>(w[p][c], v[p][c], g);
    kick_drift_f32<NSLOT>(k, drift, g, xu[p], q0[p], dq[p]);
  }
}

// Particles per gather group of a PPT-particle thread.
template <int PPT> struct GatherGroup { static constexpr int N = PPT < 4 ? PPT : 4; };

template <int NSLOT, int PPT, bool BLEND, bool TSC, bool OFF32, bool KEY>
__device__ __forceinline__ void push_chunk_f32(const PushArgs& a, int64_t chunk) {
  bool skip;
  const Segment& sg = chunk_segment(a, chunk, &skip);
  if (skip) return;
  const int64_t first = (chunk - sg.chunk_begin) * (int64_t)(kBlock * PPT) + threadIdx.x;
  // chunk-relative arrays: a uniform base and a 32-bit lane index
  const int64_t c0 = first - threadIdx.x;
  const int64_t left = sg.n - c0;
  uint32_t* X[3];
  const float* Q0[3];
  float* DQ[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { X[d] = sg.xu[d] + c0; Q0[d] = sg.q0f[d] + c0; DQ[d] = sg.dqf[d] + c0; }

  // three phases, so that the loads of all PPT particles are in flight
  // together (a store between them would pin the next loads behind it).
  // Slots past the end of the species load its last particle and are not
  // stored, so the loads and updates are straight-line code.
  const ConstF32 k = const_f32<BLEND>(a, sg);
  uint32_t xu[PPT][3];
  float dq[PPT][3], q0[PPT][3];
  const uint32_t last = (uint32_t)min<int64_t>(left - 1, (int64_t)(PPT * kBlock - 1));
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const uint32_t i = min(threadIdx.x + (uint32_t)(p * kBlock), last);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xu[p][d] = ldnt(&X[d][i]);
      q0[p][d] = ldnt(&Q0[d][i]);
      dq[p][d] = ldnt(&DQ[d][i]);
    }
  }
  if constexpr (!BLEND && !TSC) {
    constexpr int GRP = GatherGroup<PPT>::N;
#pragma unroll
    for (int p = 0; p < PPT; p += GRP)
      update_group_f32<NSLOT, GRP, OFF32>(k, a.do_drift != 0, xu + p, q0 + p, dq + p);
  } else {
#pragma unroll
    for (int p = 0; p < PPT; ++p) update_f32<NSLOT, BLEND, TSC, OFF32>(k, a.do_drift != 0, xu[p], q0[p], dq[p]);
  }
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const uint32_t i = threadIdx.x + (uint32_t)(p * kBlock);
    if ((int64_t)i >= left) break;
    if (a.do_drift) {
#pragma unroll
      for (int d = 0; d < 3; ++d) stnt(xu[p][d], &X[d][i]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) stnt(dq[p][d], &DQ[d][i]);
  }
  if constexpr (KEY) {   // sort keys of the next step's re-sort, from the state just stored
    const float ma = (float)a.key_ma, ts = (float)(a.key_tau * 4294967296.0 / a.box);
    uint32_t* K = a.key_out + c0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const uint32_t i = threadIdx.x + (uint32_t)(p * kBlock);
      if ((int64_t)i >= left) break;
      const float q[3] = {q0[p][0] + dq[p][0], q0[p][1] + dq[p][1], q0[p][2] + dq[p][2]};
      K[i] = sort_key::key_f32(xu[p], q, ma, ts, a.key_tau != 0.0, k.shift, a.key_fine_bits);
    }
  }
}

// A push that also performs the re-sort of the species whose rank pass has
// run (one, or the jobs of a batch): one block per rank block of kSortBlock
// particles.  The block reads its
// particles in place (coalesced), updates them, stages the whole new state in
// LDS and writes it out in sorted order, element e of the sorted run to
// start[bucket[e]] + rank[e] of the other buffer copy, so consecutive threads
// write consecutive slots of a bucket fragment.  The re-sort then costs the
// push the writes of q0 and id and the index reads, instead of a pass of its
// own over the whole state.
// PER particles per thread: kSortBlock / PER threads per block.
template <int NSLOT, bool BLEND, bool TSC, bool OFF32, int PER>
__global__ void __launch_bounds__(kSortBlock / PER) k_push_sort_f32(PushArgs a) {
  constexpr int kPer = PER;
  constexpr int kFusedThreads = kSortBlock / PER;
  __shared__ uint32_t st[10][kSortBlock];
  // one species (sort_batch.njobs == 0: seg and dseg point at its entries),
  // or one job of a batched re-sort (seg and seg_alt are the two tables)
  const SortBatch& sb = a.sort_batch;
  int64_t blk = xcd_chunk(blockIdx.x, gridDim.x), base = 0;
  const Segment* sgp = a.seg;
  const Segment* dsp = a.dseg;
  const uint32_t* start = a.sort_start;
  if (sb.njobs > 0) {
    const int j = batch_block(sb, blockIdx.x, &blk);
    if (j < 0) return;
    const int cur = sb.job_cur[j], sp = sb.job_species[j];
    sgp = (cur ? a.seg_alt : a.seg) + sp;
    dsp = (cur ? a.seg : a.seg_alt) + sp;
    base = sb.job_base[j];
    start = a.sort_start + j * a.sort_nkeys;
  }
  const Segment& sg = *sgp;
  const Segment& ds = *dsp;
  const uint32_t* sort_src = a.sort_src + base;
  const uint32_t* sort_bucket = a.sort_bucket + base;
  const uint32_t* sort_rank = a.sort_rank + base;
  const int64_t i0 = blk * (int64_t)kSortBlock;
  const int cnt = (int)min<int64_t>(kSortBlock, sg.n - i0);
  // the sort outputs and ids first: their latency (bucket, then its start)
  // overlaps the state loads and the gathers.  Elements past the end of the
  // species load its last one and are neither staged nor stored, so the
  // loads and updates are straight-line code.
  uint32_t src[kPer], bucket[kPer], rank[kPer], id[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int e = min((int)threadIdx.x + r * kFusedThreads, cnt - 1);
    const int64_t o = i0 + e;                  // element e of the sorted order; slot e of the block
    src[r] = ldnt(&sort_src[o]);
    bucket[r] = ldnt(&sort_bucket[o]);
    rank[r] = ldnt(&sort_rank[o]);
    id[r] = ldnt(&sg.id[o]);
  }
  uint32_t xu[kPer][3];
  float dq[kPer][3], q0[kPer][3];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int64_t i = i0 + min((int)threadIdx.x + r * kFusedThreads, cnt - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xu[r][d] = ldnt(&sg.xu[d][i]);
      q0[r][d] = ldnt(&sg.q0f[d][i]);
      dq[r][d] = ldnt(&sg.dqf[d][i]);
    }
  }
  int64_t dst[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) dst[r] = (int64_t)start[bucket[r]] - base + rank[r];
  const ConstF32 k = const_f32<BLEND>(a, sg);
  if constexpr (!BLEND && !TSC) {
    update_group_f32<NSLOT, kPer, OFF32>(k, true, xu, q0, dq);
  } else {
#pragma unroll
    for (int r = 0; r < kPer; ++r) update_f32<NSLOT, BLEND, TSC, OFF32>(k, true, xu[r], q0[r], dq[r]);
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int e = threadIdx.x + r * kFusedThreads;
    if (e >= cnt) break;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      st[d][e] = xu[r][d];
      st[3 + d][e] = __float_as_uint(q0[r][d]);
      st[6 + d][e] = __float_as_uint(dq[r][d]);
    }
    st[9][e] = id[r];
  }
  __syncthreads();
  // one array at a time, with cached stores: the fragments that neighbouring
  // blocks write into a bucket merge into whole lines in L2
  uint32_t* out[10] = {ds.xu[0], ds.xu[1], ds.xu[2], (uint32_t*)ds.q0f[0], (uint32_t*)ds.q0f[1],
                       (uint32_t*)ds.q0f[2], (uint32_t*)ds.dqf[0], (uint32_t*)ds.dqf[1], (uint32_t*)ds.dqf[2], ds.id};
#pragma unroll
  for (int k = 0; k < 10; ++k) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int e = threadIdx.x + r * kFusedThreads;
      if (e < cnt) out[k][dst[r]] = st[k][src[r]];
    }
  }
}

// 16-byte piece j of the NSLOT-double cell `cell`.
template <int NSLOT, bool OFF32>
__device__ __forceinline__ double2 load_piece_f64(const void* grid, uint32_t cell, int j) {
  if constexpr (OFF32) {
    const char FDF_GLOBAL* b = (const char FDF_GLOBAL*)grid;
    return *(const FDF_GLOBAL double2*)(b + cell * (uint32_t)(8 * NSLOT) + 16 * j);
  } else {
    return ((const FDF_GLOBAL double2*)grid)[(size_t)cell * (NSLOT / 2) + j];
  }
}

template <int NSLOT, int NPT, bool OFF32>
__device__ __forceinline__ void gather_f64(const void* grid, const uint32_t* cell, const double* w,
                                           double* g /* 7, accumulated */) {
#pragma clang fp contract(off)
#pragma unroll
  for (int c = 0; c < NPT; ++c) {
    if constexpr (NSLOT == 6) {
      const double2 v0 = load_piece_f64<6, OFF32>(grid, cell[c], 0);
      const double2 v1 = load_piece_f64<6, OFF32>(grid, cell[c], 1);
      const double2 v2 = load_piece_f64<6, OFF32>(grid, cell[c], 2);
      g[0] = fma(w[c], v0.x, g[0]); g[1] = fma(w[c], v0.y, g[1]); g[2] = fma(w[c], v1.x, g[2]);
      g[3] = fma(w[c], v1.y, g[3]); g[4] = fma(w[c], v2.x, g[4]); g[5] = fma(w[c], v2.y, g[5]);
    } else if constexpr (NSLOT == 8) {
      const double2 v0 = load_piece_f64<8, OFF32>(grid, cell[c], 0);
      const double2 v1 = load_piece_f64<8, OFF32>(grid, cell[c], 1);
      const double2 v2 = load_piece_f64<8, OFF32>(grid, cell[c], 2);
      const double2 v3 = load_piece_f64<8, OFF32>(grid, cell[c], 3);
      g[0] = fma(w[c], v0.x, g[0]); g[1] = fma(w[c], v0.y, g[1]); g[2] = fma(w[c], v1.x, g[2]);
      g[3] = fma(w[c], v1.y, g[3]); g[4] = fma(w[c], v2.x, g[4]); g[5] = fma(w[c], v2.y, g[5]);
      g[6] = fma(w[c], v3.x, g[6]);
    } else {
      const double2 v0 = load_piece_f64<4, OFF32>(grid, cell[c], 0);
      const double2 v1 = load_piece_f64<4, OFF32>(grid, cell[c], 1);
      g[0] = fma(w[c], v0.x, g[0]); g[1] = fma(w[c], v0.y, g[1]); g[2] = fma(w[c], v1.x, g[2]);
      g[6] = fma(w[c], v1.y, g[6]);
    }
  }
}

template <int NSLOT, bool TSC, bool OFF32>
__device__ __forceinline__ void gather_stencil_f64(const void* grid, const uint32_t* cell, const double* w, double* g) {
  if constexpr (TSC) {
#pragma unroll
    for (int b = 0; b < 3; ++b) gather_f64<NSLOT, 9, OFF32>(grid, cell + 9 * b, w + 9 * b, g);
  } else {
    gather_f64<NSLOT, 8, OFF32>(grid, cell, w, g);
  }
}

template <int NSLOT, int PPT, bool BLEND, bool TSC, bool OFF32>
__device__ __forceinline__ void push_chunk_f64(const PushArgs& a, int64_t chunk) {
#pragma clang fp contract(off)
  constexpr int NP = Stencil<TSC>::N;
  bool skip;
  const Segment& sg = chunk_segment(a, chunk, &skip);
  if (skip) return;
  const int64_t n = sg.n;
  const int64_t first = (chunk - sg.chunk_begin) * (int64_t)(kBlock * PPT) + threadIdx.x;
  const int gm = a.G - 1;
  const double ginv = (double)a.G / a.box;
  const double ma = sg.m * a.a_kick;
  const double mah = sg.m * a.a_drift;
  const uint32_t G = (uint32_t)a.G;
  const void* gridA = (BLEND && a.grid_sel) ? sg.grid2 : sg.grid;
  const void* gridB = (BLEND && a.grid_sel) ? sg.grid : sg.grid2;
  const double tb = a.blend_t, ta = 1.0 - tb;
  // chunk-relative arrays: a uniform base and a 32-bit lane index
  const int64_t c0 = first - threadIdx.x;
  const int64_t left = n - c0;
  double* X[3];
  double* Q[3];
  const double* Q0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { X[d] = sg.xd[d] + c0; Q[d] = sg.qd[d] + c0; Q0[d] = sg.q0d[d] + c0; }

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const uint32_t i = threadIdx.x + (uint32_t)(p * kBlock);
    if ((int64_t)i >= left) break;
    double x[3], q[3], q0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] = ldnt(&X[d][i]);
      q[d] = ldnt(&Q[d][i]);
      q0[d] = ldnt(&Q0[d][i]);
    }
    uint32_t cell[NP];
    double w[NP];
    stencil_f64<TSC>(x, ginv, gm, G, cell, w);
    double g[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (BLEND) {
      double wa[NP], wb[NP];
#pragma unroll
      for (int cc = 0; cc < NP; ++cc) { wa[cc] = ta * w[cc]; wb[cc] = tb * w[cc]; }
      gather_stencil_f64<NSLOT, TSC, OFF32>(gridA, cell, wa, g);
      gather_stencil_f64<NSLOT, TSC, OFF32>(gridB, cell, wb, g);
    } else {
      gather_stencil_f64<NSLOT, TSC, OFF32>(gridA, cell, w, g);
    }
    if (NSLOT == 4) { g[3] = g[0]; g[4] = g[1]; g[5] = g[2]; }
    const double q0sq = fma(q0[0], q0[0], fma(q0[1], q0[1], q0[2] * q0[2]));
    const double e0 = sqrt(q0sq + ma * ma);
    const double qg = fma(q0[0], g[3], fma(q0[1], g[4], q0[2] * g[5])) / e0 + g[6];
    const double cphi = q0sq / e0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double F = fma(q0[d], qg, fma(-cphi, g[3 + d], -(e0 * g[d])));
      q[d] = fma(a.kick, F, q[d]);
    }
    if (a.do_drift) {
      const double e = sqrt(fma(q[0], q[0], fma(q[1], q[1], q[2] * q[2])) + mah * mah);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double xn = fmod(fma(a.drift, q[d] / e, x[d]), a.box);   // floor-mod as numpy.mod
        if (xn < 0.0) xn += a.box;
        stnt(xn, &X[d][i]);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) stnt(q[d], &Q[d][i]);
  }
}

// Chunk loop.  One block per chunk, or (persistent) a fixed grid whose
// blocks stride over the chunks; either way each XCD (block id mod 8) walks a
// contiguous eighth of the chunk range.
template <int NSLOT, int PPT, bool BLEND, bool TSC, bool OFF32, bool KEY = false>
__global__ void __launch_bounds__(kBlock) k_push_f32(PushArgs a) {
  if (!a.persistent) {
    const int64_t c = launch_chunk(a);
    if (c >= 0) push_chunk_f32<NSLOT, PPT, BLEND, TSC, OFF32, KEY>(a, c);
    return;
  }
  const int64_t per = (a.total_chunks + 7) / 8, x = blockIdx.x % 8, stride = gridDim.x / 8;
  const int64_t end = min((x + 1) * per, a.total_chunks);
  for (int64_t c = x * per + blockIdx.x / 8; c < end; c += stride)
    push_chunk_f32<NSLOT, PPT, BLEND, TSC, OFF32, KEY>(a, c);
}

template <int NSLOT, int PPT, bool BLEND, bool TSC, bool OFF32>
__global__ void __launch_bounds__(kBlock) k_push_f64(PushArgs a) {
  if (!a.persistent) {
    const int64_t c = launch_chunk(a);
    if (c >= 0) push_chunk_f64<NSLOT, PPT, BLEND, TSC, OFF32>(a, c);
    return;
  }
  const int64_t per = (a.total_chunks + 7) / 8, x = blockIdx.x % 8, stride = gridDim.x / 8;
  const int64_t end = min((x + 1) * per, a.total_chunks);
  for (int64_t c = x * per + blockIdx.x / 8; c < end; c += stride) push_chunk_f64<NSLOT, PPT, BLEND, TSC, OFF32>(a, c);
}

template <int PPT, bool BLEND, bool TSC>
void push_launch(const PushArgs& a, hipStream_t s) {
  const int64_t grid_blocks = a.persistent ? a.persistent : (a.xcd_blocks > 0 ? a.xcd_blocks : a.total_chunks);
  const dim3 grid((unsigned)grid_blocks), block(kBlock);
  // byte offsets of the mesh fit 32 bits?
  const bool off32 = (uint64_t)a.G * a.G * a.G * (uint64_t)(a.nslot * (a.fp64 ? 8 : 2)) <= (1ull << 32);
  if (a.fp64) {
    if (off32) {
      if (a.nslot == 8) hipLaunchKernelGGL((k_push_f64<8, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
      else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f64<6, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
      else hipLaunchKernelGGL((k_push_f64<4, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
    } else {
      if (a.nslot == 8) hipLaunchKernelGGL((k_push_f64<8, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
      else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f64<6, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
      else hipLaunchKernelGGL((k_push_f64<4, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
    }
  } else {
    if constexpr (!BLEND && !TSC) {
      if (a.key_out) {   // this push also writes the sort keys of the next step's re-sort
        if (off32) {
          if (a.nslot == 8) hipLaunchKernelGGL((k_push_f32<8, PPT, false, false, true, true>), grid, block, a.lds_reserve, s, a);
          else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f32<6, PPT, false, false, true, true>), grid, block, a.lds_reserve, s, a);
          else hipLaunchKernelGGL((k_push_f32<4, PPT, false, false, true, true>), grid, block, a.lds_reserve, s, a);
        } else {
          if (a.nslot == 8) hipLaunchKernelGGL((k_push_f32<8, PPT, false, false, false, true>), grid, block, a.lds_reserve, s, a);
          else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f32<6, PPT, false, false, false, true>), grid, block, a.lds_reserve, s, a);
          else hipLaunchKernelGGL((k_push_f32<4, PPT, false, false, false, true>), grid, block, a.lds_reserve, s, a);
        }
        return;
      }
    }
    if (off32) {
      if (a.nslot == 8) hipLaunchKernelGGL((k_push_f32<8, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
      else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f32<6, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
      else hipLaunchKernelGGL((k_push_f32<4, PPT, BLEND, TSC, true>), grid, block, a.lds_reserve, s, a);
    } else {
      if (a.nslot == 8) hipLaunchKernelGGL((k_push_f32<8, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
      else if (a.nslot == 6) hipLaunchKernelGGL((k_push_f32<6, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
      else hipLaunchKernelGGL((k_push_f32<4, PPT, BLEND, TSC, false>), grid, block, a.lds_reserve, s, a);
    }
  }
}

template <bool BLEND, bool TSC, int PER>
void push_sort_launch_per(const PushArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.sort_batch.njobs > 0 ? batch_grid(a.sort_batch) : a.total_chunks)),
      block(kSortBlock / PER);
  const bool off32 = (uint64_t)a.G * a.G * a.G * (uint64_t)(a.nslot * 2) <= (1ull << 32);
  if (off32) {
    if (a.nslot == 8) hipLaunchKernelGGL((k_push_sort_f32<8, BLEND, TSC, true, PER>), grid, block, a.lds_reserve, s, a);
    else if (a.nslot == 6) hipLaunchKernelGGL((k_push_sort_f32<6, BLEND, TSC, true, PER>), grid, block, a.lds_reserve, s, a);
    else hipLaunchKernelGGL((k_push_sort_f32<4, BLEND, TSC, true, PER>), grid, block, a.lds_reserve, s, a);
  } else {
    if (a.nslot == 8) hipLaunchKernelGGL((k_push_sort_f32<8, BLEND, TSC, false, PER>), grid, block, a.lds_reserve, s, a);
    else if (a.nslot == 6) hipLaunchKernelGGL((k_push_sort_f32<6, BLEND, TSC, false, PER>), grid, block, a.lds_reserve, s, a);
    else hipLaunchKernelGGL((k_push_sort_f32<4, BLEND, TSC, false, PER>), grid, block, a.lds_reserve, s, a);
  }
}

template <bool BLEND, bool TSC>
void push_sort_launch(const PushArgs& a, hipStream_t s) {
  if (a.ppt == 1) push_sort_launch_per<BLEND, TSC, 1>(a, s);
  else if (a.ppt == 2) push_sort_launch_per<BLEND, TSC, 2>(a, s);
  else push_sort_launch_per<BLEND, TSC, 4>(a, s);
}

template <int PPT>
void push_ppt(const PushArgs& a, hipStream_t s) {
  if (a.tsc) {
    if (a.blend) push_launch<PPT, true, true>(a, s);
    else push_launch<PPT, false, true>(a, s);
  } else {
    if (a.blend) push_launch<PPT, true, false>(a, s);
    else push_launch<PPT, false, false>(a, s);
  }
}

}  // namespace

int push_chunk_particles(int ppt) { return kBlock * ppt; }

void launch_push_sort(const PushArgs& a, hipStream_t s) {
  if (a.tsc) {
    if (a.blend) push_sort_launch<true, true>(a, s);
    else push_sort_launch<false, true>(a, s);
  } else {
    if (a.blend) push_sort_launch<true, false>(a, s);
    else push_sort_launch<false, false>(a, s);
  }
}

void launch_push(const PushArgs& a, hipStream_t s) {
  if (a.eom != 0) { launch_push_eom(a, s); return; }
  switch (a.ppt) {
    case 1: push_ppt<1>(a, s); break;
    case 2: push_ppt<2>(a, s); break;
    case 4: push_ppt<4>(a, s); break;
    default: push_ppt<8>(a, s); break;
  }
}

}  // namespace fdf
