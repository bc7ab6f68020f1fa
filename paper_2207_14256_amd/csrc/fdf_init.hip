// Initial data on the device: seeded Gaussian field, particle sample, and the
// pre-initial-condition transform (sec. 2.1).
#include "fdf_device.h"
#include "fdf_internal.h"

namespace fdf {
namespace {

// BBKS transfer function, q = k / (Gamma h) with k in 1/Mpc.
__device__ __forceinline__ double bbks(double k, double gamma, double h) {
  const double q = k / (gamma * h);
  const double a = 3.89 * q, b = 16.1 * q, c = 5.46 * q, d = 6.71 * q;
  const double poly = 1.0 + a + b * b + c * c * c + (d * d) * (d * d);
  return log1p(2.34 * q) / (2.34 * q) * pow(poly, -0.25);
}

// One thread per stored mode (ix, iy, iz), iz in [0, G/2).  The Philox counter
// is the mode's index in the (G, G, G/2+1) half-complex array, so the draws
// do not depend on storage.  On the iz = 0 plane the mode with the larger
// index takes the conjugate of its partner (-nx, -ny, 0).
template <typename R>
__global__ void k_field_gen(FieldGenArgs a) {
  const int G = a.G, M = G / 2, H = G / 2 + 1;
  const size_t total = (size_t)G * G * M;
  const double V = a.box * a.box * a.box;
  const double kf = 2.0 * 3.14159265358979323846 / a.box;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int iz = (int)(e % M), iy = (int)((e / M) % G), ix = (int)(e / ((size_t)M * G));
    cplx<R> val = {(R)0, (R)0};
    const bool zero = ix == G / 2 || iy == G / 2 || (ix == 0 && iy == 0 && iz == 0);
    if (!zero) {
      int sx = ix, sy = iy;
      bool conj = false;
      if (iz == 0) {
        const int px = (G - ix) % G, py = (G - iy) % G;
        if ((long)ix * G + iy > (long)px * G + py) { sx = px; sy = py; conj = true; }
      }
      const uint64_t m = ((uint64_t)sx * G + sy) * H + iz;
      const u64x4 w = philox4x64(m, 0, 0, 0, a.seed, kStreamField);
      const double u1 = unit_open(w.v[0]), u2 = unit_open(w.v[1]);
      const double r = a.fixed_amp ? 1.0 : sqrt(-log(u1));
      const double ph = 2.0 * 3.14159265358979323846 * u2;
      const int nx = ix < G / 2 ? ix : ix - G, ny = iy < G / 2 ? iy : iy - G;
      const double k = sqrt((kf * nx) * (kf * nx) + (kf * ny) * (kf * ny) + (kf * iz) * (kf * iz));
      const double t = bbks(k, a.gamma, a.h);
      const double pk = a.amp * pow(k, a.ns) * (t * t);
      const double s = sqrt(pk / V) * r;
      double re = s * cos(ph), im = s * sin(ph);
      if (conj) im = -im;
      val = {(R)re, (R)im};
    }
    ((cplx<R>*)a.out)[e] = val;
  }
}

// Particle sample: uniform positions on the 2^-32 L lattice, |q| from
// q^2 fbar(q) by Gamma(3)-proposal rejection, isotropic directions; momentum
// components rounded once to binary32 (the canonical state of both forms).
__global__ void k_sample(SampleArgs a) {
  const int64_t n = a.seg.n;
  const double T = a.t_nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t id = a.by_id ? (uint64_t)a.seg.id[i] : (uint64_t)i;
    const u64x4 wp = philox4x64(id, 0, 0, 0, a.seed, kStreamPosition);
    uint32_t xu[3];
    for (int d = 0; d < 3; ++d) xu[d] = (uint32_t)(wp.v[d] >> 32);
    float qf[3];
    sample_momentum(a.seed, id, T, qf);
    if (a.fp64) {
      const double scale = a.box * 0x1p-32;
      for (int d = 0; d < 3; ++d) {
        a.seg.xd[d][i] = (double)xu[d] * scale;
        a.seg.qd[d][i] = (double)qf[d];
        a.seg.q0d[d][i] = (double)qf[d];
      }
    } else {
      for (int d = 0; d < 3; ++d) {
        a.seg.xu[d][i] = xu[d];
        a.seg.q0f[d][i] = qf[d];
        a.seg.dqf[d][i] = 0.0f;
      }
    }
    if (!a.by_id) a.seg.id[i] = (uint32_t)i;
  }
}

// Pre-initial conditions (sec. 2.1, eq. transform) with the super-horizon
// moments delta = -2 psi and theta_k = k^2 tau psi_k / 2, for which
// grad(nabla^-2 theta) = -(tau/2) grad psi; with nu = 4 and omega = 4/3:
//   q_i -> q_i (1 - psi/2) - (eps tau / 6) d_i psi,  eps = sqrt(q^2 + m^2 a^2).
// grid: [G^3][4] = (d psi/dx, d psi/dy, d psi/dz, psi), CIC-interpolated.
template <typename GR>
__global__ void k_pre_ic(PreIcArgs a) {
  const int64_t n = a.seg.n;
  const int G = a.G;
  const GR* grid = (const GR*)a.grid;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
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
      const double u = x[d] * ((double)G / a.box);
      const double fl = floor(u);
      t[d] = u - fl;
      const int ii = ((int)fl % G + G) % G;
      i0[d] = ii; i1[d] = (ii + 1) % G;
    }
    double acc[4] = {0, 0, 0, 0};
    for (int c = 0; c < 8; ++c) {
      const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
      const double w = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) * (cz ? t[2] : 1 - t[2]);
      const size_t cell = (size_t)mesh_x(cx ? i1[0] : i0[0], G) + mesh_y(cy ? i1[1] : i0[1], G) +
                          mesh_z(cz ? i1[2] : i0[2]);
      for (int s = 0; s < 4; ++s) acc[s] += w * (double)grid[cell * 4 + s];
    }
    const double eps = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + (a.m * a.a) * (a.m * a.a));
    for (int d = 0; d < 3; ++d) {
      const float qn = (float)(q[d] * (1.0 - 0.5 * acc[3]) - (eps * a.tau / 6.0) * acc[d]);
      if (a.fp64) { a.seg.qd[d][i] = qn; a.seg.q0d[d][i] = qn; }
      else { a.seg.q0f[d][i] = qn; a.seg.dqf[d][i] = 0.0f; }
    }
  }
}

int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  return (int)(g > 65536 * 4 ? 65536 * 4 : (g ? g : 1));
}

}  // namespace

void launch_field_gen(const FieldGenArgs& a, hipStream_t s) {
  const size_t total = (size_t)a.G * a.G * (a.G / 2);
  if (a.fp64) hipLaunchKernelGGL(k_field_gen<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_field_gen<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, a);
}

void launch_sample_species(const SampleArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sample, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
}

void launch_pre_ic(const PreIcArgs& a, hipStream_t s) {
  if (a.fp64) hipLaunchKernelGGL(k_pre_ic<double>, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_pre_ic<float>, dim3(grid_for((size_t)a.seg.n, 256)), dim3(256), 0, s, a);
}

}  // namespace fdf
