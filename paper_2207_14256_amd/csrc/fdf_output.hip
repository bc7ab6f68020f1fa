// Outputs of the push: delta-f weights (sec. 2.2) and the energy-density
// deposit of eq. empirical_rho, gfx950.
#include <algorithm>
#include <type_traits>

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

// Value deposited by particle i: w eps (energy density) or w q_axis = w eps
// v_axis (momentum density), times the per-half normalisation
// G^3 / (N_half <eps>); *half receives the half (even / odd id).
__device__ __forceinline__ double deposit_value(const OutputArgs& a, int64_t i, int* half) {
  const uint32_t id = a.seg.id[i];
  double q[3], p[3];
  momenta(a, i, id, q, p);
  const double w = deltaf_weight(q, p, a.t_nu);
  const double eps = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + (a.m * a.a) * (a.m * a.a));
  *half = a.auto_mode ? 0 : (int)(id & 1u);
  return (a.quantity < 0 ? w * eps : w * q[a.quantity]) * a.norm[*half];
}

// CIC cell and weights of particle i on the G^3 deposit mesh (vertex-centred
// mesh points, periodic): x-major cell index, or (bricked) the 4^3-brick
// index of the gradient meshes, so that a wave of sorted particles adds into
// a few contiguous kilobytes.
template <bool BRICKED>
__device__ __forceinline__ void deposit_cic(const OutputArgs& a, int64_t i, size_t* cell, double* wc) {
  const int G = a.G;
  const double ginv = (double)G / a.box;
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
  for (int c = 0; c < 8; ++c) {
    const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
    wc[c] = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) * (cz ? t[2] : 1 - t[2]);
    const int jx = cx ? i1[0] : i0[0], jy = cy ? i1[1] : i0[1], jz = cz ? i1[2] : i0[2];
    if constexpr (BRICKED)
      cell[c] = (size_t)mesh_x((uint32_t)jx, (uint32_t)G) + mesh_y((uint32_t)jy, (uint32_t)G) + mesh_z((uint32_t)jz);
    else
      cell[c] = ((size_t)jx * G + jy) * G + jz;
  }
}

// Fixed-point deposit (FP32 form).  Every contribution wc * val is rounded
// to an integer multiple of a quantum Q = 2^(e - bits), where 2^e bounds the
// largest |val| of the spectrum's particles and bits leaves headroom for the
// sum over all of them in 63 bits; the integers are summed with 64-bit
// atomics, so the result does not depend on the order of the additions (bit
// for bit the same from run to run, whatever the launch shape or particle
// order).  Pass 1 finds the largest |val| (as binary32 bits, an order-free
// integer maximum); pass 2 deposits; pass 3 converts to binary32.
__device__ __forceinline__ double fixed_inv_quantum(uint32_t max_bits, int bits) {
  int e;
  frexpf(__uint_as_float(max_bits), &e);   // max |val| < 2^e (e = 0 when there is none)
  return ldexp(1.0, bits - e);
}

__global__ void __launch_bounds__(256) k_deposit_max(OutputArgs a) {
  float m = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.seg.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int half;
    const double v = fabs(deposit_value(a, i, &half));
    m = fmaxf(m, __double2float_ru(v));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(a.max_bits, __float_as_uint(m));
}

// Deposit with the additions gathered first in a workgroup hash table in
// LDS (key = 2 cell + half, linear probing), so that the sums of a block's
// 1024 particles reach the mesh with one global atomic per distinct cell and
// half instead of one per corner.  Global atomics are carried out past the
// per-XCD L2 caches, one memory transaction each, and dominate the plain
// kernels' time; sorted particles share most corners (about 8 contributions
// per particle become 2 to 3 global atomics).  A contribution that finds no
// slot within kProbe probes goes to the mesh directly.  V = unsigned long
// long: the fixed-point form, whose integer sums do not depend on how the
// additions are grouped or ordered; V = double: the FP64 form.
template <typename V>
__global__ void __launch_bounds__(256) k_deposit_lds(OutputArgs a) {
  constexpr int R = 4, LOGH = 12;
  constexpr uint32_t H = 1u << LOGH, kEmpty = 0xFFFFFFFFu;
  constexpr int kProbe = 32;
  constexpr bool kFixed = std::is_same<V, unsigned long long>::value;
  __shared__ uint32_t key[H];
  __shared__ V val[H];
  const double scale = kFixed ? fixed_inv_quantum(*a.max_bits, a.fixed_bits) : 1.0;
  constexpr int64_t per = 256 * R;
  const int64_t nchunk = (a.seg.n + per - 1) / per;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    for (uint32_t s = threadIdx.x; s < H; s += 256) { key[s] = kEmpty; val[s] = (V)0; }
    __syncthreads();
    for (int r = 0; r < R; ++r) {
      const int64_t i = ch * per + r * 256 + threadIdx.x;
      if (i >= a.seg.n) break;
      int half;
      const double v0 = deposit_value(a, i, &half) * scale;
      size_t cell[8];
      double wc[8];
      deposit_cic<kFixed>(a, i, cell, wc);
      for (int c = 0; c < 8; ++c) {
        V v;
        if constexpr (kFixed) v = (V)__double2ll_rn(wc[c] * v0);
        else v = wc[c] * v0;
        if (v == (V)0) continue;
        const uint32_t k = (uint32_t)(cell[c] * 2 + half);
        uint32_t h = (k * 0x9E3779B1u) >> (32 - LOGH);
        bool done = false;
        for (int p = 0; p < kProbe; ++p) {
          const uint32_t prev = atomicCAS(&key[h], kEmpty, k);
          if (prev == kEmpty || prev == k) {
            atomicAdd(&val[h], v);
            done = true;
            break;
          }
          h = (h + 1) & (H - 1);
        }
        if (!done) {
          V* const d = (V*)a.dens[half] + cell[c];
          if constexpr (kFixed) atomicAdd(d, v);
          else unsafeAtomicAdd(d, v);
        }
      }
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < H; s += 256) {
      const uint32_t k = key[s];
      const V v = val[s];
      if (k == kEmpty || v == (V)0) continue;
      V* const d = (V*)a.dens[k & 1u] + (k >> 1);
      if constexpr (kFixed) atomicAdd(d, v);
      else unsafeAtomicAdd(d, v);
    }
    __syncthreads();
  }
}

// Bricked fixed-point halves -> x-major binary32 meshes, four cells along z
// per thread: they are contiguous in both layouts (one 32-byte read of the
// brick's z-run, one 16-byte write).
__global__ void k_fixed_to_real(FixedToRealArgs a) {
  const double q = 1.0 / fixed_inv_quantum(*a.max_bits, a.fixed_bits);
  const uint32_t G = (uint32_t)a.G, lg = 31 - __clz(G);
  const size_t n4 = a.n / 4, h4 = a.n_half / 4;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const int h = i >= h4;
    const size_t j = 4 * (i - (h ? h4 : 0));     // x-major cell (ix, iy, iz), iz = 0 mod 4
    const uint32_t iz = (uint32_t)(j & (G - 1)), iy = (uint32_t)((j >> lg) & (G - 1)), ix = (uint32_t)(j >> (2 * lg));
    const size_t b = (size_t)mesh_x(ix, G) + mesh_y(iy, G) + mesh_z(iz);
    const longlong2* src = (const longlong2*)(a.src[h] + b);
    const longlong2 v0 = src[0], v1 = src[1];
    *(float4*)(a.dst[h] + j) = make_float4((float)((double)v0.x * q), (float)((double)v0.y * q),
                                           (float)((double)v1.x * q), (float)((double)v1.y * q));
  }
}

// Bin sums [count][sum |k|][sum P] -> [mean |k|][mean P][count]; an empty
// bin's means are NaN.
__global__ void k_bins_finalize(const double* bins, int nbins, double* out) {
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const double cnt = bins[b];
    out[b] = cnt > 0 ? bins[nbins + b] / cnt : nan;
    out[nbins + b] = cnt > 0 ? bins[2 * nbins + b] / cnt : nan;
    out[2 * nbins + b] = cnt;
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
  // grid_n <= 1024 (checked at creation): the keys 2 cell + half stay below
  // the empty key in 32 bits
  const int grid = grid_for((size_t)a.seg.n, 1024);
  if (a.fp64) hipLaunchKernelGGL(k_deposit_lds<double>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_deposit_lds<unsigned long long>, dim3(grid), dim3(256), 0, s, a);
}

void launch_bins_finalize(const double* bins, int nbins, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bins_finalize, dim3(1), dim3(256), 0, s, bins, nbins, out);
}

void launch_deposit_max(const OutputArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_deposit_max, dim3(std::min(grid_for((size_t)a.seg.n, 256), 8192)), dim3(256), 0, s, a);
}

void launch_fixed_to_real(const FixedToRealArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fixed_to_real, dim3(grid_for(a.n / 4, 256)), dim3(256), 0, s, a);
}

// Zero a 16-byte aligned buffer whose size is a multiple of 16 with a plain
// kernel (no memset node, so the work may be captured in a graph).
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (!n16) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n16, 256)), dim3(256), 0, s, (uint4*)ptr, n16);
}

}  // namespace fdf
