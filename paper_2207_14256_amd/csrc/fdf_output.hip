// Outputs of the push: delta-f weights (sec. 2.2) and the energy-density
// deposit of eq. empirical_rho, gfx950.
#include <algorithm>

#include "fdf_device.h"
#include "fdf_internal.h"

namespace fdf {
namespace {

// Current momentum (binary64) and the sampled momentum p of particle i.
__device__ __forceinline__ void momenta(const OutputArgs& a, int64_t i, uint32_t id,
                                        double* q, double* p) {
  if (a.fp64) {
    for (int d = 0; d < 3; ++d) { q[d] = a.seg.qd[d][i]; p[d] = a.seg.q0d[d][i]; }
  } else {
    // q = q0 + dq, exact in binary64
    for (int d = 0; d < 3; ++d) {
      p[d] = (double)a.seg.q0f[d][i];
      q[d] = p[d] + (double)a.seg.dqf[d][i];
    }
  }
  if (a.pre_ic) {  // q0 carries the transformed momentum; p is the raw sample
    float pf[3];
    sample_momentum(a.seed, (uint64_t)id, a.t_nu, pf);
    for (int d = 0; d < 3; ++d) p[d] = (double)pf[d];
  }
}

// w = 1 - fbar(|q|)/fbar(|p|) = expm1(D/T) / (e^{-|p|/T} + e^{D/T}),
// D = |q| - |p| = (2 p.d + d.d) / (|q| + |p|), d = q - p: no cancellation.
__device__ __forceinline__ double deltaf_weight(const double* q, const double* p, double T) {
  double d[3], pd = 0.0, dd = 0.0, qq = 0.0, pp = 0.0;
  for (int k = 0; k < 3; ++k) {
    d[k] = q[k] - p[k];
    pd += p[k] * d[k];
    dd += d[k] * d[k];
    qq += q[k] * q[k];
    pp += p[k] * p[k];
  }
  const double qn = sqrt(qq), pn = sqrt(pp);
  const double den = qn + pn;
  const double D = den > 0.0 ? (2.0 * pd + dd) / den : 0.0;
  return expm1(D / T) / (exp(-pn / T) + exp(D / T));
}

__global__ void k_weights(OutputArgs a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.seg.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t id = a.seg.id[i];
    double q[3], p[3];
    momenta(a, i, id, q, p);
    a.w_out[id] = deltaf_weight(q, p, a.t_nu);
  }
}

// CIC deposit of w eps (energy density) or w q_axis = w eps v_axis (momentum
// density) times the per-half normalisation G^3 / (N_half <eps>).
template <typename DR>
__global__ void k_deposit(OutputArgs a) {
  const int G = a.G;
  const double ginv = (double)G / a.box;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.seg.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t id = a.seg.id[i];
    double q[3], p[3];
    momenta(a, i, id, q, p);
    const double w = deltaf_weight(q, p, a.t_nu);
    const double eps = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + (a.m * a.a) * (a.m * a.a));
    const int half = a.auto_mode ? 0 : (int)(id & 1u);
    const double val = (a.quantity < 0 ? w * eps : w * q[a.quantity]) * a.norm[half];
    int i0[3], i1[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
      const double x = a.fp64 ? a.seg.xd[d][i] : (double)a.seg.xu[d][i] * (a.box * 0x1p-32);
      const double u = x * ginv;
      const double fl = floor(u);
      t[d] = u - fl;
      i0[d] = ((int)fl) & (G - 1);
      i1[d] = (i0[d] + 1) & (G - 1);
    }
    DR* dst = (DR*)a.dens[half];
    for (int c = 0; c < 8; ++c) {
      const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
      const double wc = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) * (cz ? t[2] : 1 - t[2]);
      const size_t cell = ((size_t)(cx ? i1[0] : i0[0]) * G + (cy ? i1[1] : i0[1])) * G + (cz ? i1[2] : i0[2]);
      atomicAdd(&dst[cell], (DR)(wc * val));
    }
  }
}

// Squared magnitudes of -eps grad psi, -(q^2/eps) grad phi, q (q . grad phi)/eps
// and q phidot at the particle's CIC-interpolated mesh values, summed per
// block in LDS and added to a.out.
__device__ __forceinline__ double term_slot(const TermArgs& a, size_t cell, int slot) {
  if (a.fp64) return ((const double*)a.grid)[cell * a.nslot + slot];
  const uint16_t b = ((const uint16_t*)a.grid)[cell * a.nslot + slot];
  return (double)__uint_as_float((uint32_t)b << 16);
}

__global__ void __launch_bounds__(256) k_force_terms(TermArgs a) {
  __shared__ double red[4][256];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int G = a.G;
  const double ginv = (double)G / a.box;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.seg.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x[3], q[3];
    for (int d = 0; d < 3; ++d) {
      if (a.fp64) { x[d] = a.seg.xd[d][i]; q[d] = a.seg.qd[d][i]; }
      else {
        x[d] = (double)a.seg.xu[d][i] * (a.box * 0x1p-32);
        q[d] = (double)a.seg.q0f[d][i] + (double)a.seg.dqf[d][i];
      }
    }
    int i0[3], i1[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
      const double u = x[d] * ginv;
      const double fl = floor(u);
      t[d] = u - fl;
      i0[d] = ((int)fl) & (G - 1);
      i1[d] = (i0[d] + 1) & (G - 1);
    }
    double gpsi[3] = {0, 0, 0}, gphi[3] = {0, 0, 0}, phidot = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
      const double w = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) * (cz ? t[2] : 1 - t[2]);
      const size_t cell = (size_t)mesh_x(cx ? i1[0] : i0[0], G) + mesh_y(cy ? i1[1] : i0[1], G) +
                          mesh_z(cz ? i1[2] : i0[2]);
      for (int d = 0; d < 3; ++d) {
        gpsi[d] += w * term_slot(a, cell, a.slot_gpsi + d);
        gphi[d] += w * term_slot(a, cell, a.slot_gphi + d);
      }
      if (a.slot_phidot >= 0) phidot += w * term_slot(a, cell, a.slot_phidot);
    }
    const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    const double eps = sqrt(q2 + a.ma * a.ma);
    const double qg = q[0] * gphi[0] + q[1] * gphi[1] + q[2] * gphi[2];
    const double g2psi = gpsi[0] * gpsi[0] + gpsi[1] * gpsi[1] + gpsi[2] * gpsi[2];
    const double g2phi = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
    acc[0] += eps * eps * g2psi;
    acc[1] += (q2 / eps) * (q2 / eps) * g2phi;
    acc[2] += q2 * (qg / eps) * (qg / eps);
    acc[3] += q2 * phidot * phidot;
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) atomicAdd(&a.out[threadIdx.x], red[threadIdx.x][0]);
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  return (int)(g > 65536 * 4 ? 65536 * 4 : (g ? g : 1));
}

}  // namespace

void launch_weights(const OutputArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_weights, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
}

void launch_force_terms(const TermArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_force_terms, dim3(std::min(grid_for((size_t)a.seg.n, 256), 4096)), dim3(256), 0, s, a);
}

void launch_deposit(const OutputArgs& a, hipStream_t s) {
  if (a.fp64) hipLaunchKernelGGL(k_deposit<double>, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_deposit<float>, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
}

// Zero a 16-byte aligned buffer whose size is a multiple of 16 with a plain
// kernel (no memset node, so the work may be captured in a graph).
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (!n16) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n16, 256)), dim3(256), 0, s, (uint4*)ptr, n16);
}

}  // namespace fdf
