// Kick-drift-kick push for the non-separable equations of motion, gfx950.
//
// Forms (PushArgs::eom; fdf_config.eom):
//   EXACT     geodesic in q, eq. releq + eq. geodesic (sec. 3.1):
//               F = -eps grad psi - (q^2/eps) grad phi + q (q . grad phi)/eps + q phidot
//               v = (q/eps) (1 + phi + psi)
//   CANONICAL Lagrangian form in P, eq. releq_lag + eq. geodesic_lag (sec. 3.2):
//               F = -eps grad psi - (P^2/eps) grad phi
//               v = (P/eps) [1 + psi + (2 - P^2/eps^2) phi]
//   SR_NEWTON eq. p_eq (sec. 5):  F = -(2 P^2 + m^2 a^2)/eps grad psi,  v = P/eps
//   SIMPLE_Q  eq. q_eq (sec. 5):  F = -eps grad psi,                    v = q/eps
//   NEWTONIAN (sec. 5):           F = -m a grad psi,                    v = q/eps
// with eps = sqrt(q^2 + m^2 a^2) of the current momentum.
//
// The force depends on the momentum it acts on, so the two half-kicks that
// meet at a time point are not merged: a launch gathers the mesh once at x_k
// and applies the closing half-kick of step k-1 (coefficient `kick`) and then
// the opening half-kick of step k (`kick_open`), each with the momentum it
// starts from, then drifts with the metric factor sampled at x_k.
//
// Grid slots per cell: EXACT   gpsi[3] gphi[3] phidot (phi + psi)
//                      CANONICAL gpsi[3] gphi[3] psi phi
//                      others  gpsi[3] 0           (4 slots)
// Storage forms as in the separable push (fixed-point x and q = q0 + dq in FP32).
#include "fdf_push_common.h"

namespace fdf {
namespace {

using namespace push_detail;

enum : int32_t { EOM_EXACT = 1, EOM_CANONICAL = 2, EOM_SR_NEWTON = 3, EOM_SIMPLE_Q = 4, EOM_NEWTONIAN = 5 };

// All slots of a cell, accumulated with the stencil weights.
template <int NSLOT, int NPT>
__device__ __forceinline__ void gather_all_bf16(const void* grid, const size_t* cell, const float* w, float* g) {
#pragma clang fp contract(off)
  if constexpr (NSLOT == 8) {
    const FDF_GLOBAL uint4* gp = (const FDF_GLOBAL uint4*)grid;
    uint4 v[NPT];
#pragma unroll
    for (int c = 0; c < NPT; ++c) v[c] = gp[cell[c]];
#pragma unroll
    for (int c = 0; c < NPT; ++c) {
      const uint32_t u[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        g[2 * j] = fmaf(w[c], bf16_lo(u[j]), g[2 * j]);
        g[2 * j + 1] = fmaf(w[c], bf16_hi(u[j]), g[2 * j + 1]);
      }
    }
  } else {
    const FDF_GLOBAL uint2* gp = (const FDF_GLOBAL uint2*)grid;
    uint2 v[NPT];
#pragma unroll
    for (int c = 0; c < NPT; ++c) v[c] = gp[cell[c]];
#pragma unroll
    for (int c = 0; c < NPT; ++c) {
      g[0] = fmaf(w[c], bf16_lo(v[c].x), g[0]); g[1] = fmaf(w[c], bf16_hi(v[c].x), g[1]);
      g[2] = fmaf(w[c], bf16_lo(v[c].y), g[2]);
    }
  }
}

template <int NSLOT, int NPT>
__device__ __forceinline__ void gather_all_f64(const void* grid, const size_t* cell, const double* w, double* g) {
#pragma clang fp contract(off)
  const FDF_GLOBAL double2* gp = (const FDF_GLOBAL double2*)grid;
#pragma unroll
  for (int c = 0; c < NPT; ++c) {
#pragma unroll
    for (int j = 0; j < NSLOT / 2; ++j) {
      if (NSLOT == 4 && j == 1) {
        g[2] = fma(w[c], gp[2 * cell[c] + 1].x, g[2]);
      } else {
        const double2 v = gp[(NSLOT / 2) * cell[c] + j];
        g[2 * j] = fma(w[c], v.x, g[2 * j]);
        g[2 * j + 1] = fma(w[c], v.y, g[2 * j + 1]);
      }
    }
  }
}

// Whole stencil: CIC in one batch, TSC in three x-planes of 9 points.
template <int NSLOT, bool TSC, typename R>
__device__ __forceinline__ void gather_stencil(const void* grid, const size_t* cell, const R* w, R* g) {
  constexpr int B = TSC ? 3 : 1, NPT = TSC ? 9 : 8;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (sizeof(R) == 4) gather_all_bf16<NSLOT, NPT>(grid, cell + NPT * b, w + NPT * b, g);
    else gather_all_f64<NSLOT, NPT>(grid, cell + NPT * b, w + NPT * b, g);
  }
}

// Force of the selected form from gathered slots g and momentum q; ma2 = (m a)^2.
template <typename R>
__device__ __forceinline__ void eom_force(int eom, const R* q, const R* g, R ma, R ma2, R* F) {
#pragma clang fp contract(off)
  const R q2 = fma(q[0], q[0], fma(q[1], q[1], q[2] * q[2]));
  const R e = sqrt(q2 + ma2);
  if (eom == EOM_NEWTONIAN) {
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -(ma * g[d]);
    return;
  }
  const R ie = (R)1 / e;
  if (eom == EOM_SR_NEWTON) {
    const R s = fma((R)2, q2, ma2) * ie;
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -(s * g[d]);
    return;
  }
  if (eom == EOM_SIMPLE_Q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -(e * g[d]);
    return;
  }
  const R cphi = q2 * ie;
  R qg = (R)0;
  if (eom == EOM_EXACT) qg = fma(fma(q[0], g[3], fma(q[1], g[4], q[2] * g[5])), ie, g[6]);
#pragma unroll
  for (int d = 0; d < 3; ++d) F[d] = fma(q[d], qg, fma(-cphi, g[3 + d], -(e * g[d])));
}

// Metric factor s of the velocity v = (q/eps)(1 + s), eps at the drift time.
template <typename R>
__device__ __forceinline__ R eom_drift_factor(int eom, R q2, R ie2, const R* g) {
#pragma clang fp contract(off)
  if (eom == EOM_EXACT) return g[7];                                    // phi + psi
  if (eom == EOM_CANONICAL) return fma((R)2 - q2 * ie2, g[7], g[6]);    // psi + (2 - P^2/eps^2) phi
  return (R)0;
}

template <int NSLOT, int PPT, bool BLEND, bool TSC>
__device__ __forceinline__ void push_chunk_eom_f32(const PushArgs& a, int64_t chunk) {
#pragma clang fp contract(off)
  constexpr int NP = Stencil<TSC>::N;
  bool skip;
  const Segment& sg = chunk_segment(a, chunk, &skip);
  if (skip) return;
  const int64_t n = sg.n;
  const int64_t first = (chunk - sg.chunk_begin) * (int64_t)(kBlock * PPT) + threadIdx.x;
  const int shift = 32 - a.log2g;
  const uint32_t gmask = (uint32_t)a.G - 1u;
  const float finv = __uint_as_float((uint32_t)(127 - shift) << 23);   // 2^-shift
  const float kicks[2] = {(float)a.kick, (float)a.kick_open};
  const float ma = (float)(sg.m * a.a_kick);
  const float mah = (float)(sg.m * a.a_drift);
  const float ma2 = ma * ma, mah2 = mah * mah;
  const float dscale = (float)(a.drift * 4294967296.0 / a.box);
  const size_t G = (size_t)a.G;
  const void* gridA = (BLEND && a.grid_sel) ? sg.grid2 : sg.grid;
  const void* gridB = (BLEND && a.grid_sel) ? sg.grid : sg.grid2;
  const float tb = (float)a.blend_t, ta = 1.0f - tb;

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int64_t i = first + (int64_t)p * kBlock;
    if (i >= n) break;
    uint32_t xu[3];
    float q0[3], dq[3], q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xu[d] = ldnt(&sg.xu[d][i]);
      q0[d] = ldnt(&sg.q0f[d][i]);
      dq[d] = ldnt(&sg.dqf[d][i]);
      q[d] = q0[d] + dq[d];
    }
    size_t cell[NP];
    float w[NP];
    stencil_u32<TSC>(xu, shift, gmask, finv, G, cell, w);
    float g[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (BLEND) {
      float wa[NP], wb[NP];
#pragma unroll
      for (int cc = 0; cc < NP; ++cc) { wa[cc] = ta * w[cc]; wb[cc] = tb * w[cc]; }
      gather_stencil<NSLOT, TSC>(gridA, cell, wa, g);
      gather_stencil<NSLOT, TSC>(gridB, cell, wb, g);
    } else {
      gather_stencil<NSLOT, TSC>(gridA, cell, w, g);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (kicks[h] == 0.0f) continue;
      float F[3];
      eom_force<float>(a.eom, q, g, ma, ma2, F);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        dq[d] = fmaf(kicks[h], F[d], dq[d]);
        q[d] = q0[d] + dq[d];
      }
    }
    if (a.do_drift) {
      const float qq = fmaf(q[0], q[0], fmaf(q[1], q[1], q[2] * q[2]));
      const float e2 = qq + mah2;
      const float ie = 1.0f / sqrtf(e2);
      const float sf = eom_drift_factor<float>(a.eom, qq, 1.0f / e2, g);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float v = q[d] * ie;
        const int disp = __float2int_rn(dscale * fmaf(v, sf, v));
        stnt(xu[d] + (uint32_t)disp, &sg.xu[d][i]);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) stnt(dq[d], &sg.dqf[d][i]);
  }
}

template <int NSLOT, int PPT, bool BLEND, bool TSC>
__device__ __forceinline__ void push_chunk_eom_f64(const PushArgs& a, int64_t chunk) {
#pragma clang fp contract(off)
  constexpr int NP = Stencil<TSC>::N;
  bool skip;
  const Segment& sg = chunk_segment(a, chunk, &skip);
  if (skip) return;
  const int64_t n = sg.n;
  const int64_t first = (chunk - sg.chunk_begin) * (int64_t)(kBlock * PPT) + threadIdx.x;
  const int gm = a.G - 1;
  const double ginv = (double)a.G / a.box;
  const double kicks[2] = {a.kick, a.kick_open};
  const double ma = sg.m * a.a_kick;
  const double mah = sg.m * a.a_drift;
  const size_t G = (size_t)a.G;
  const void* gridA = (BLEND && a.grid_sel) ? sg.grid2 : sg.grid;
  const void* gridB = (BLEND && a.grid_sel) ? sg.grid : sg.grid2;
  const double tb = a.blend_t, ta = 1.0 - tb;

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int64_t i = first + (int64_t)p * kBlock;
    if (i >= n) break;
    double x[3], q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] = ldnt(&sg.xd[d][i]);
      q[d] = ldnt(&sg.qd[d][i]);
    }
    size_t cell[NP];
    double w[NP];
    stencil_f64<TSC>(x, ginv, gm, G, cell, w);
    double g[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (BLEND) {
      double wa[NP], wb[NP];
#pragma unroll
      for (int cc = 0; cc < NP; ++cc) { wa[cc] = ta * w[cc]; wb[cc] = tb * w[cc]; }
      gather_stencil<NSLOT, TSC>(gridA, cell, wa, g);
      gather_stencil<NSLOT, TSC>(gridB, cell, wb, g);
    } else {
      gather_stencil<NSLOT, TSC>(gridA, cell, w, g);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (kicks[h] == 0.0) continue;
      double F[3];
      eom_force<double>(a.eom, q, g, ma, ma * ma, F);
#pragma unroll
      for (int d = 0; d < 3; ++d) q[d] = fma(kicks[h], F[d], q[d]);
    }
    if (a.do_drift) {
      const double qq = fma(q[0], q[0], fma(q[1], q[1], q[2] * q[2]));
      const double e2 = qq + mah * mah;
      const double e = sqrt(e2);
      const double sf = eom_drift_factor<double>(a.eom, qq, 1.0 / e2, g);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double v = q[d] / e;
        double xn = fmod(fma(a.drift, fma(v, sf, v), x[d]), a.box);   // floor-mod as numpy.mod
        if (xn < 0.0) xn += a.box;
        stnt(xn, &sg.xd[d][i]);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) stnt(q[d], &sg.qd[d][i]);
  }
}

template <int NSLOT, int PPT, bool BLEND, bool TSC>
__global__ void __launch_bounds__(kBlock) k_push_eom_f32(PushArgs a) {
  if (!a.persistent) {
    const int64_t c = launch_chunk(a);
    if (c >= 0) push_chunk_eom_f32<NSLOT, PPT, BLEND, TSC>(a, c);
    return;
  }
  const int64_t per = (a.total_chunks + 7) / 8, x = blockIdx.x % 8, stride = gridDim.x / 8;
  const int64_t end = min((x + 1) * per, a.total_chunks);
  for (int64_t c = x * per + blockIdx.x / 8; c < end; c += stride) push_chunk_eom_f32<NSLOT, PPT, BLEND, TSC>(a, c);
}

template <int NSLOT, int PPT, bool BLEND, bool TSC>
__global__ void __launch_bounds__(kBlock) k_push_eom_f64(PushArgs a) {
  if (!a.persistent) {
    const int64_t c = launch_chunk(a);
    if (c >= 0) push_chunk_eom_f64<NSLOT, PPT, BLEND, TSC>(a, c);
    return;
  }
  const int64_t per = (a.total_chunks + 7) / 8, x = blockIdx.x % 8, stride = gridDim.x / 8;
  const int64_t end = min((x + 1) * per, a.total_chunks);
  for (int64_t c = x * per + blockIdx.x / 8; c < end; c += stride) push_chunk_eom_f64<NSLOT, PPT, BLEND, TSC>(a, c);
}

template <int PPT, bool BLEND, bool TSC>
void eom_launch(const PushArgs& a, hipStream_t s) {
  const int64_t grid_blocks = a.persistent ? a.persistent : (a.xcd_blocks > 0 ? a.xcd_blocks : a.total_chunks);
  const dim3 grid((unsigned)grid_blocks), block(kBlock);
  if (a.fp64) {
    if (a.nslot == 8) hipLaunchKernelGGL((k_push_eom_f64<8, PPT, BLEND, TSC>), grid, block, a.lds_reserve, s, a);
    else hipLaunchKernelGGL((k_push_eom_f64<4, PPT, BLEND, TSC>), grid, block, a.lds_reserve, s, a);
  } else {
    if (a.nslot == 8) hipLaunchKernelGGL((k_push_eom_f32<8, PPT, BLEND, TSC>), grid, block, a.lds_reserve, s, a);
    else hipLaunchKernelGGL((k_push_eom_f32<4, PPT, BLEND, TSC>), grid, block, a.lds_reserve, s, a);
  }
}

template <int PPT>
void eom_ppt(const PushArgs& a, hipStream_t s) {
  if (a.tsc) {
    if (a.blend) eom_launch<PPT, true, true>(a, s);
    else eom_launch<PPT, false, true>(a, s);
  } else {
    if (a.blend) eom_launch<PPT, true, false>(a, s);
    else eom_launch<PPT, false, false>(a, s);
  }
}

}  // namespace

void launch_push_eom(const PushArgs& a, hipStream_t s) {
  switch (a.ppt) {
    case 1: eom_ppt<1>(a, s); break;
    case 2: eom_ppt<2>(a, s); break;
    case 4: eom_ppt<4>(a, s); break;
    default: eom_ppt<8>(a, s); break;
  }
}

}  // namespace fdf
