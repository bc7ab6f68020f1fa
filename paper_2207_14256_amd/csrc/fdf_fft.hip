// Potential grids and power spectra: Fourier stage + 3-D Stockham FFTs (gfx950).
//
// Inverse direction (grid build, sec. 2.1 "potential grids"): delta_0(k) is
// multiplied by the transfer functions and i k_a, then transformed by three
// LDS-resident passes:
//   X pass  : strided C2C along x, fused with the Fourier-stage multipliers;
//             one block = NB consecutive z-columns of one y row, all x;
//   Y pass  : strided C2C along y, in place;
//   Z pass  : contiguous C2R along z through a half-length complex FFT,
//             writing all slots of a cell together (packed [G^3][nslot]).
// Forward direction (P(k), sec. 4): Z pass R2C, Y pass, X pass in place (or,
// for the momentum spectrum, multiplied by i k_a and summed over the axes),
// then exact log-|k| binning of Re(A conj B) in fixed point.
//
// Half-complex intermediates keep only n_z in [0, G/2): every Nyquist mode
// of delta_0 is zero, and the spectrum bins stop below k_N, so the n_z = G/2
// plane is never needed.
//
// Stockham stage (radix R, Ns = product of earlier radices), for butterfly j:
//   v_r = in[j + r N/R] * W_{Ns R}^{r (j mod Ns)},  v = DFT_R(v),
//   out[(j/Ns) Ns R + (j mod Ns) + r Ns] = v_r.
#include <type_traits>

#include "fdf_device.h"
#include "fdf_internal.h"

namespace fdf {
namespace {

// ------------------------------------------------------------ butterflies --
template <bool INV, typename R>
__device__ __forceinline__ void bfly2(cplx<R>* v) {
  cplx<R> a = cadd(v[0], v[1]), b = csub(v[0], v[1]);
  v[0] = a; v[1] = b;
}

template <bool INV, typename R>
__device__ __forceinline__ void bfly4(cplx<R>& v0, cplx<R>& v1, cplx<R>& v2, cplx<R>& v3) {
  cplx<R> a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = csub(v1, v3);
  v0 = cadd(a0, a2);
  v2 = csub(a0, a2);
  if (INV) {  // X1 = a1 + i a3, X3 = a1 - i a3
    v1 = {a1.x - a3.y, a1.y + a3.x};
    v3 = {a1.x + a3.y, a1.y - a3.x};
  } else {    // X1 = a1 - i a3, X3 = a1 + i a3
    v1 = {a1.x + a3.y, a1.y - a3.x};
    v3 = {a1.x - a3.y, a1.y + a3.x};
  }
}

template <bool INV, typename R>
__device__ __forceinline__ void bfly8(cplx<R>* v) {
  const R c = (R)0.70710678118654752440084436210484903928;
  cplx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  bfly4<INV>(e0, e1, e2, e3);
  bfly4<INV>(o0, o1, o2, o3);
  cplx<R> t1, t2, t3;
  if (INV) {  // W8^s = e^{+i pi s/4}
    t1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};
    t2 = {-o2.y, o2.x};
    t3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};
  } else {    // W8^s = e^{-i pi s/4}
    t1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};
    t2 = {o2.y, -o2.x};
    t3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};
  }
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1); v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2); v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3); v[7] = csub(e3, t3);
}

template <int RAD, bool INV, typename R>
__device__ __forceinline__ void bfly(cplx<R>* v) {
  if constexpr (RAD == 8) bfly8<INV>(v);
  else if constexpr (RAD == 4) bfly4<INV>(v[0], v[1], v[2], v[3]);
  else bfly2<INV>(v);
}

// ------------------------------------------------------------ LDS stages --
// buf holds NB lines of length N with element n of line b at buf[n*NB + b].
// tw is the global table e^{-2 pi i m / G}; the length-N root of unity
// W_N^m is tw[m * TWS] with TWS = G / N.
template <typename R, int N, int NB, int NT, bool INV, int NS, int RAD, int TWS>
__device__ __forceinline__ void fft_stage(cplx<R>* buf, const cplx<R>* __restrict__ tw) {
  constexpr int NBF = NB * (N / RAD);
  constexpr int PER = (NBF + NT - 1) / NT;
  cplx<R> v[PER][RAD];
  const int tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int t = tid + p * NT;
    if (NBF % NT == 0 || t < NBF) {
      const int b = t % NB, j = t / NB;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[p][r] = buf[(j + r * (N / RAD)) * NB + b];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int t = tid + p * NT;
    if (NBF % NT == 0 || t < NBF) {
      const int b = t % NB, j = t / NB;
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          cplx<R> w = tw[(r * k * (N / (NS * RAD))) * TWS];
          v[p][r] = INV ? cmulc(v[p][r], w) : cmul(v[p][r], w);
        }
      }
      bfly<RAD, INV>(v[p]);
      const int base = (j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[(base + r * NS) * NB + b] = v[p][r];
    }
  }
  __syncthreads();
}

template <typename R, int N, int NB, int NT, bool INV, int TWS, int NS = 1>
__device__ __forceinline__ void fft_lines(cplx<R>* buf, const cplx<R>* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int REM = N / NS;
    constexpr int RAD = REM >= 8 ? 8 : REM;
    fft_stage<R, N, NB, NT, INV, NS, RAD, TWS>(buf, tw);
    fft_lines<R, N, NB, NT, INV, TWS, NS * RAD>(buf, tw);
  }
}

// ---------------------------------------------------------- block shapes --
template <typename R, int G> struct Shape {
  static constexpr int CS = (int)sizeof(cplx<R>);
  static constexpr int NB0 = 65536 / (G * CS);
  static constexpr int NB = NB0 > 16 ? 16 : (NB0 < 1 ? 1 : NB0);     // columns per strided block
  static constexpr int NBC = NB > G / 2 ? G / 2 : NB;
  static constexpr int NBX = NBC;                                    // columns per X-pass block
  static constexpr int NT = 256;
  static constexpr int M = G / 2;
  static constexpr int NL0 = 1024 / G;
  static constexpr int NL1 = NL0 > 16 ? 16 : (NL0 < 1 ? 1 : NL0);
  static constexpr int NL = NL1 > G ? G : NL1;                        // lines per contiguous block
};

__device__ __forceinline__ int signed_index(int i, int G) { return i < G / 2 ? i : i - G; }

// Fourier-stage multiplier of one slot at wave numbers (nx, ny, nz).
__device__ __forceinline__ void slot_multiplier(int kind, int nx, int ny, int nz, double kf,
                                                const Transfer& tr, double& re, double& im) {
  re = 0.0; im = 0.0;
  const double k2 = kf * kf * (double)(nx * nx + ny * ny + nz * nz);
  if (k2 == 0.0 || kind == SK_ZERO) return;
  const double tphi = tr.c_phi / k2;
  if (kind == SK_PHIDOT) { re = tr.c_phidot / k2; return; }
  if (kind == SK_PHI) { re = tphi; return; }
  double t = tphi;
  if (kind == SK_DX_PSI || kind == SK_DY_PSI || kind == SK_DZ_PSI || kind == SK_PSI || kind == SK_PHI_PSI)
    t = tphi * (1.0 - tr.slip_amp * exp(-sqrt(k2) / tr.slip_k));
  if (kind == SK_PSI) { re = t; return; }
  if (kind == SK_PHI_PSI) { re = tphi + t; return; }
  int n = (kind == SK_DX_PSI || kind == SK_DX_PHI) ? nx
        : (kind == SK_DY_PSI || kind == SK_DY_PHI) ? ny : nz;
  im = kf * (double)n * t;   // i k_a T
}

// ------------------------------------------------------------------ X pass --
// delta_0 is read again for every field (from L2 after the first) rather
// than held in registers across the fields: the multipliers' binary64
// arithmetic then leaves room for several waves per SIMD.
template <typename R, int G>
__global__ void __launch_bounds__(256) k_xpass_inverse(GridBuildArgs a) {
  using S = Shape<R, G>;
  constexpr int NB = S::NBX, NT = S::NT, M = S::M;
  constexpr int PER = (G * NB + NT - 1) / NT;
  __shared__ cplx<R> buf[G * NB];
  const int nzb = M / NB;
  const int iy = blockIdx.x / nzb, iz0 = (blockIdx.x % nzb) * NB;
  const cplx<R>* __restrict__ din = (const cplx<R>*)a.delta_k;
  const cplx<R>* __restrict__ tw = (const cplx<R>*)a.twiddle;
  cplx<R>* scr = (cplx<R>*)a.scratch;
  const size_t plane = (size_t)G * G * M;
  const int ny = signed_index(iy, G);
  for (int f = 0; f < a.nfft; ++f) {
    const int kind = a.kind[f];
#pragma unroll 2
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((G * NB) % NT == 0 || e < G * NB) {
        const int ix = e / NB, b = e % NB;
        const cplx<R> d = din[((size_t)ix * G + iy) * M + iz0 + b];
        double re, im;
        slot_multiplier(kind, signed_index(ix, G), ny, iz0 + b, a.kf, a.tr, re, im);
        const double dx = (double)d.x, dy = (double)d.y;
        buf[ix * NB + b] = {(R)(re * dx - im * dy), (R)(re * dy + im * dx)};
      }
    }
    __syncthreads();
    fft_lines<R, G, NB, NT, true, 1>(buf, tw);
#pragma unroll 4
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((G * NB) % NT == 0 || e < G * NB) {
        const int ix = e / NB, b = e % NB;
        scr[f * plane + ((size_t)ix * G + iy) * M + iz0 + b] = buf[ix * NB + b];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------- Y pass (either direction) --
// blocks over (field h, ix, z-column block); lines along y; in place.
template <typename R, int G, bool INV>
__global__ void __launch_bounds__(256) k_ypass(cplx<R>* scr, const cplx<R>* __restrict__ tw) {
  using S = Shape<R, G>;
  constexpr int NB = S::NBC, NT = S::NT, M = S::M;
  constexpr int PER = (G * NB + NT - 1) / NT;
  __shared__ cplx<R> buf[G * NB];
  const int nzb = M / NB;
  const int blk = blockIdx.x;
  const int izb = blk % nzb, ix = (blk / nzb) % G, f = blk / (nzb * G);
  const int iz0 = izb * NB;
  cplx<R>* base = scr + (size_t)f * G * G * M + (size_t)ix * G * M + iz0;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * NT;
    if ((G * NB) % NT == 0 || e < G * NB) {
      const int iy = e / NB, b = e % NB;
      buf[iy * NB + b] = base[(size_t)iy * M + b];
    }
  }
  __syncthreads();
  fft_lines<R, G, NB, NT, INV, 1>(buf, tw);
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * NT;
    if ((G * NB) % NT == 0 || e < G * NB) {
      const int iy = e / NB, b = e % NB;
      base[(size_t)iy * M + b] = buf[iy * NB + b];
    }
  }
}

// ------------------------------------------------ Z pass: C2R + slot packing --
template <int NSLOT, int OT, typename R>
__device__ __forceinline__ void store_cell(void* out, size_t cell, const R* vals);

template <> __device__ __forceinline__ void store_cell<8, GT_BF16, float>(void* out, size_t cell, const float* v) {
  uint4 w;
  w.x = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
  w.y = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
  w.z = f32_to_bf16_bits(v[4]) | (f32_to_bf16_bits(v[5]) << 16);
  w.w = f32_to_bf16_bits(v[6]) | (f32_to_bf16_bits(v[7]) << 16);
  ((uint4*)out)[cell] = w;
}
template <> __device__ __forceinline__ void store_cell<6, GT_BF16, float>(void* out, size_t cell, const float* v) {
  uint32_t* o = (uint32_t*)out + 3 * cell;   // 12-byte cell
  o[0] = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
  o[1] = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
  o[2] = f32_to_bf16_bits(v[4]) | (f32_to_bf16_bits(v[5]) << 16);
}
template <> __device__ __forceinline__ void store_cell<4, GT_BF16, float>(void* out, size_t cell, const float* v) {
  uint2 w;
  w.x = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
  w.y = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
  ((uint2*)out)[cell] = w;
}
template <> __device__ __forceinline__ void store_cell<4, GT_F32, float>(void* out, size_t cell, const float* v) {
  ((float4*)out)[cell] = make_float4(v[0], v[1], v[2], v[3]);
}
template <> __device__ __forceinline__ void store_cell<8, GT_F32, float>(void* out, size_t cell, const float* v) {
  ((float4*)out)[2 * cell] = make_float4(v[0], v[1], v[2], v[3]);
  ((float4*)out)[2 * cell + 1] = make_float4(v[4], v[5], v[6], v[7]);
}
template <> __device__ __forceinline__ void store_cell<4, GT_F64, double>(void* out, size_t cell, const double* v) {
  double2* o = (double2*)out + 2 * cell;
  o[0] = make_double2(v[0], v[1]);
  o[1] = make_double2(v[2], v[3]);
}
template <> __device__ __forceinline__ void store_cell<6, GT_F64, double>(void* out, size_t cell, const double* v) {
  double2* o = (double2*)out + 3 * cell;
  o[0] = make_double2(v[0], v[1]);
  o[1] = make_double2(v[2], v[3]);
  o[2] = make_double2(v[4], v[5]);
}
template <> __device__ __forceinline__ void store_cell<8, GT_F64, double>(void* out, size_t cell, const double* v) {
  double2* o = (double2*)out + 4 * cell;
  o[0] = make_double2(v[0], v[1]);
  o[1] = make_double2(v[2], v[3]);
  o[2] = make_double2(v[4], v[5]);
  o[3] = make_double2(v[6], v[7]);
}

// blocks over (ix, y-line block of NL lines)
template <typename R, int G, int NSLOT, int OT>
__global__ void __launch_bounds__(256) k_zpass_c2r(GridBuildArgs a) {
  using S = Shape<R, G>;
  constexpr int NL = S::NL, NT = S::NT, M = S::M;
  constexpr int PER = (M * NL + NT - 1) / NT;
  __shared__ cplx<R> buf[M * NL];
  __shared__ R stage[NL * G * NSLOT];
  const int nyb = G / NL;
  const int ix = blockIdx.x / nyb, iy0 = (blockIdx.x % nyb) * NL;
  const cplx<R>* __restrict__ tw = (const cplx<R>*)a.twiddle;
  const cplx<R>* scr = (const cplx<R>*)a.scratch;
  const size_t plane = (size_t)G * G * M;
  for (int e = threadIdx.x; e < NL * G * NSLOT; e += NT) stage[e] = (R)0;
  for (int f = 0; f < a.nfft; ++f) {
    const int slot = a.slot[f];
    cplx<R> x[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {   // coalesced: consecutive threads, consecutive k
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e / M, k = e % M;
        x[p] = scr[f * plane + ((size_t)ix * G + iy0 + line) * M + k];
      }
    }
    __syncthreads();   // previous field's results have left buf
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e / M, k = e % M;
        buf[k * NL + line] = x[p];
      }
    }
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i e^{2 pi i k/G} (X[k] - conj X[M-k]), X[M] = 0
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e / M, k = e % M;
        cplx<R> xk = x[p];
        cplx<R> xm = k ? buf[(M - k) * NL + line] : cplx<R>{(R)0, (R)0};
        cplx<R> s = {xk.x + xm.x, xk.y - xm.y};          // X[k] + conj X[M-k]
        cplx<R> d = {xk.x - xm.x, xk.y + xm.y};          // X[k] - conj X[M-k]
        cplx<R> w = tw[k];                               // e^{-2 pi i k/G}
        cplx<R> wd = cmulc(d, w);                        // d e^{+2 pi i k/G}
        x[p] = {s.x - wd.y, s.y + wd.x};                 // s + i wd
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e / M, k = e % M;
        buf[k * NL + line] = x[p];
      }
    }
    __syncthreads();
    fft_lines<R, M, NL, NT, true, 2>(buf, tw);
    for (int e = threadIdx.x; e < M * NL; e += NT) {
      const int line = e / M, m = e % M;
      cplx<R> z = buf[m * NL + line];
      stage[(line * G + 2 * m) * NSLOT + slot] = z.x;
      stage[(line * G + 2 * m + 1) * NSLOT + slot] = z.y;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NL * G; e += NT) {
    const int line = e / G, iz = e % G;
    const size_t cell = (size_t)mesh_x(ix, G) + mesh_y(iy0 + line, G) + mesh_z(iz);   // bricked layout
    store_cell<NSLOT, OT, R>(a.out, cell, &stage[e * NSLOT]);
  }
}

// ---------------------------------------------------- forward Z pass: R2C --
// blocks over (half h, ix, y-line block)
template <typename R, int G>
__global__ void __launch_bounds__(256) k_zpass_r2c(PkArgs a) {
  using S = Shape<R, G>;
  constexpr int NL = S::NL, NT = S::NT, M = S::M;
  constexpr int PER = (M * NL + NT - 1) / NT;
  __shared__ cplx<R> buf[M * NL];
  const int nyb = G / NL;
  const int blk = blockIdx.x;
  const int h = blk / (G * nyb);
  const int ix = (blk / nyb) % G, iy0 = (blk % nyb) * NL;
  const cplx<R>* __restrict__ tw = (const cplx<R>*)a.twiddle;
  const cplx<R>* src = (const cplx<R>*)(h ? a.grid_b : a.grid_a);   // reals read in pairs
  cplx<R>* dst = (cplx<R>*)a.scratch + (size_t)h * G * G * M;
  for (int e = threadIdx.x; e < M * NL; e += NT) {
    const int line = e / M, m = e % M;
    buf[m * NL + line] = src[((size_t)ix * G + iy0 + line) * M + m];   // z[m] = x[2m] + i x[2m+1]
  }
  __syncthreads();
  fft_lines<R, M, NL, NT, false, 2>(buf, tw);
  // X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) e^{-2 pi i k/G} (Z[k] - conj Z[M-k]),  Z[M] = Z[0]
  cplx<R> x[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * NT;
    if ((M * NL) % NT == 0 || e < M * NL) {
      const int line = e / M, k = e % M;
      cplx<R> zk = buf[k * NL + line];
      cplx<R> zm = buf[((M - k) % M) * NL + line];
      cplx<R> s = {zk.x + zm.x, zk.y - zm.y};
      cplx<R> d = {zk.x - zm.x, zk.y + zm.y};
      cplx<R> wd = cmul(d, tw[k]);                     // d e^{-2 pi i k/G}
      x[p] = {(R)0.5 * (s.x + wd.y), (R)0.5 * (s.y - wd.x)};   // s/2 - (i/2) wd
    }
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * NT;
    if ((M * NL) % NT == 0 || e < M * NL) {
      const int line = e / M, k = e % M;
      dst[((size_t)ix * G + iy0 + line) * M + k] = x[p];
    }
  }
}

// ------------------------- forward X pass + i k_axis, summed over the axes --
// Density spectrum (deriv_axis < 0): the x transform of each half, in place.
// Momentum spectrum: Theta = sum_a i k_a J_a(k), one axis per call, summed
// into planes 2 (and 3).
template <typename R, int G>
__global__ void __launch_bounds__(256) k_xpass_accum(PkArgs a) {
  using S = Shape<R, G>;
  constexpr int NB0 = S::NBC / 2 > 0 ? S::NBC / 2 : 1;
  constexpr int NB = NB0, NT = S::NT, M = S::M;
  __shared__ cplx<R> buf[G * NB];
  const int nzb = M / NB;
  const int halves = a.auto_mode ? 1 : 2;
  const int h = blockIdx.x / (G * nzb);
  const int blk = blockIdx.x % (G * nzb);
  const int iy = blk / nzb, iz0 = (blk % nzb) * NB;
  const cplx<R>* __restrict__ tw = (const cplx<R>*)a.twiddle;
  cplx<R>* scr = (cplx<R>*)a.scratch;
  const size_t plane = (size_t)G * G * M;
  if (h >= halves) return;
  for (int e = threadIdx.x; e < G * NB; e += NT) {
    const int ix = e / NB, b = e % NB;
    buf[ix * NB + b] = scr[h * plane + ((size_t)ix * G + iy) * M + iz0 + b];
  }
  __syncthreads();
  fft_lines<R, G, NB, NT, false, 1>(buf, tw);
  const int ny = signed_index(iy, G);
  if (a.deriv_axis < 0) {   // each block owns its columns: in place is safe
    for (int e = threadIdx.x; e < G * NB; e += NT) {
      const int ix = e / NB, b = e % NB;
      scr[h * plane + ((size_t)ix * G + iy) * M + iz0 + b] = buf[ix * NB + b];
    }
    return;
  }
  cplx<R>* acc = scr + (2 + h) * plane;
  for (int e = threadIdx.x; e < G * NB; e += NT) {
    const int ix = e / NB, b = e % NB;
    const int n = a.deriv_axis == 0 ? signed_index(ix, G) : a.deriv_axis == 1 ? ny : iz0 + b;
    const R kn = (R)(a.kf * (double)n);
    const cplx<R> v = buf[ix * NB + b];
    const cplx<R> t = {-kn * v.y, kn * v.x};          // i k_axis v
    const size_t gi = ((size_t)ix * G + iy) * M + iz0 + b;
    if (a.accum_first) acc[gi] = t;
    else acc[gi] = {acc[gi].x + t.x, acc[gi].y + t.y};
  }
}

// Log binning of planes bin_plane (and bin_plane + 1), laid out [kx][ky][kz]:
// per bin the mode count, the sum of |n| and the sum of P = V Re(A conj B)
// (modes with n_z > 0 count twice).  The sums are exact integer sums, so the
// result does not depend on the order of the additions (bit for bit the same
// from run to run): |n| in units of 2^-50 and P in units of 2^(e - 61), with
// 2^e above every |P| (from a first pass), accumulated in 128 bits (a low
// word whose carry goes to a high word) with 64-bit atomics.
__device__ __forceinline__ int mode_bin(size_t gi, int G, int nbins, long* n2_out, int* nz_out) {
  const int M = G / 2;
  const int nz = (int)(gi % M), iy = (int)((gi / M) % G), ix = (int)(gi / ((size_t)M * G));
  const int nx = signed_index(ix, G), ny = signed_index(iy, G);
  const long n2 = (long)nx * nx + (long)ny * ny + (long)nz * nz;
  *n2_out = n2;
  *nz_out = nz;
  if (n2 == 0) return -1;
  const double log2h = (double)(31 - __clz(G / 2));
  const int bin = (int)floor((double)nbins * log2((double)n2) / (2.0 * log2h));
  return bin < nbins ? bin : -1;
}

template <typename R, int G>
__device__ __forceinline__ double mode_power(const PkArgs& a, size_t gi) {
  const size_t plane = (size_t)G * G * (G / 2);
  const cplx<R>* scr = (const cplx<R>*)a.scratch;
  const cplx<R> u = scr[a.bin_plane * plane + gi];
  const cplx<R> v = a.auto_mode ? u : scr[(a.bin_plane + 1) * plane + gi];
  const double norm = a.volume / ((double)G * G * G * (double)G * G * G);
  return norm * ((double)u.x * (double)v.x + (double)u.y * (double)v.y);
}

template <typename R, int G>
__global__ void __launch_bounds__(256) k_bin_max(PkArgs a) {
  const size_t plane = (size_t)G * G * (G / 2);
  float m = 0.0f;
  for (size_t gi = blockIdx.x * (size_t)blockDim.x + threadIdx.x; gi < plane;
       gi += (size_t)gridDim.x * blockDim.x) {
    long n2;
    int nz;
    if (mode_bin(gi, G, a.nbins, &n2, &nz) < 0) continue;
    m = fmaxf(m, __double2float_ru(fabs(mode_power<R, G>(a, gi))));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(a.max_bits, __float_as_uint(m));
}

// 128-bit add of a signed 64-bit value into (lo, hi) words.
__device__ __forceinline__ void add128(unsigned long long* lo, unsigned long long* hi, long long v) {
  const unsigned long long u = (unsigned long long)v;
  const unsigned long long old = atomicAdd(lo, u);
  const unsigned long long carry = (old + u < old) ? 1ull : 0ull;
  const unsigned long long h = (v < 0 ? ~0ull : 0ull) + carry;
  if (h) atomicAdd(hi, h);
}

constexpr double kNScale = 1125899906842624.0;   // 2^50: units of the |n| sums

template <typename R, int G>
__global__ void __launch_bounds__(256) k_bin_fixed(PkArgs a) {
  __shared__ unsigned long long acc[5 * 256];
  const int nb = a.nbins;
  const size_t plane = (size_t)G * G * (G / 2);
  for (int e = threadIdx.x; e < 5 * nb; e += blockDim.x) acc[e] = 0;
  __syncthreads();
  int e2;
  frexpf(__uint_as_float(*a.max_bits), &e2);       // every |P| < 2^e2
  const double inv_q = ldexp(1.0, 61 - e2);
  for (size_t gi = blockIdx.x * (size_t)blockDim.x + threadIdx.x; gi < plane;
       gi += (size_t)gridDim.x * blockDim.x) {
    long n2;
    int nz;
    const int bin = mode_bin(gi, G, nb, &n2, &nz);
    if (bin < 0) continue;
    const long long w = nz == 0 ? 1 : 2;
    const long long pq = __double2ll_rn(mode_power<R, G>(a, gi) * inv_q) * w;
    const long long nq = __double2ll_rn(sqrt((double)n2) * kNScale) * w;
    atomicAdd(&acc[bin], (unsigned long long)w);
    add128(&acc[nb + bin], &acc[2 * nb + bin], nq);
    add128(&acc[3 * nb + bin], &acc[4 * nb + bin], pq);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (!acc[b]) continue;
    atomicAdd(&a.acc[b], acc[b]);
    for (int k = 0; k < 2; ++k) {   // 128-bit block sums into the global ones
      const unsigned long long lo = acc[(1 + 2 * k) * nb + b], hi = acc[(2 + 2 * k) * nb + b];
      const unsigned long long old = atomicAdd(&a.acc[(1 + 2 * k) * nb + b], lo);
      const unsigned long long h = hi + ((old + lo < old) ? 1ull : 0ull);
      if (h) atomicAdd(&a.acc[(2 + 2 * k) * nb + b], h);
    }
  }
}

// Exact sums -> [count][sum |k|][sum P] in binary64.
__global__ void k_bin_sums(PkArgs a) {
  const int nb = a.nbins;
  int e2;
  frexpf(__uint_as_float(*a.max_bits), &e2);
  const double q = ldexp(1.0, e2 - 61);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double nsum = ((double)a.acc[2 * nb + b] * 18446744073709551616.0 + (double)a.acc[nb + b]) / kNScale;
    const double psum = ((double)(long long)a.acc[4 * nb + b] * 18446744073709551616.0 +
                         (double)a.acc[3 * nb + b]) * q;
    a.bins[b] = (double)a.acc[b];
    a.bins[nb + b] = a.kf * nsum;
    a.bins[2 * nb + b] = psum;
  }
}

// bfloat16 meshes: one block = 2 x-values by 4 y-lines (8 z-lines), so that
// it writes whole halves of 4^3-cell bricks (32 cells of 2 NSLOT bytes: whole
// 128-byte lines, one vector store per cell) instead of fragments of lines
// shared with blocks on other XCDs.  Element e of a field's 8 lines is
// (line e % 8, frequency e / 8) throughout, so that every LDS access of the
// half-length transform's pre-processing is conflict-free; the results are
// staged as bfloat16 pairs (the same rounding as the per-cell stores above)
// in per-slot rows padded to spread the 8 lines over the banks.
template <int NSLOT> struct CellWords;
template <> struct CellWords<8> { using T = uint4; };
template <> struct CellWords<6> { using T = uint3; };
template <> struct CellWords<4> { using T = uint2; };

template <int G, int NSLOT>
__global__ void __launch_bounds__(256) k_zpass_c2r_bf16(GridBuildArgs a) {
  using R = float;
  constexpr int M = G / 2, NT = 256, NL = 8;
  constexpr int PER = (M * NL + NT - 1) / NT;
  constexpr int SW = (G + 16) / 2;                  // 32-bit words per staged row (line, slot)
  __shared__ cplx<R> buf[M * NL];
  __shared__ uint32_t stage[NSLOT * NL * SW];
  const int nyb = G / 4;
  const int ix0 = (blockIdx.x / nyb) * 2, iy0 = (blockIdx.x % nyb) * 4;
  const cplx<R>* __restrict__ tw = (const cplx<R>*)a.twiddle;
  const cplx<R>* scr = (const cplx<R>*)a.scratch;
  const size_t plane = (size_t)G * G * M;
  for (int e = threadIdx.x; e < NSLOT * NL * SW; e += NT) stage[e] = 0u;
  // line l = 4 (x offset) + (y offset); the next field's lines are loaded
  // while this field is transformed
  auto load = [&](int f, cplx<R>* v) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e % NL, k = e / NL;
        v[p] = scr[f * plane + ((size_t)(ix0 + (line >> 2)) * G + iy0 + (line & 3)) * M + k];
      }
    }
  };
  cplx<R> xn[PER];
  if (a.nfft > 0) load(0, xn);
  for (int f = 0; f < a.nfft; ++f) {
    const int slot = a.slot[f];
    cplx<R> x[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) x[p] = xn[p];
    if (f + 1 < a.nfft) load(f + 1, xn);
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) buf[e] = x[p];
    }
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i e^{2 pi i k/G} (X[k] - conj X[M-k]), X[M] = 0
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) {
        const int line = e % NL, k = e / NL;
        cplx<R> xk = x[p];
        cplx<R> xm = k ? buf[(M - k) * NL + line] : cplx<R>{(R)0, (R)0};
        cplx<R> s = {xk.x + xm.x, xk.y - xm.y};
        cplx<R> d = {xk.x - xm.x, xk.y + xm.y};
        cplx<R> w = tw[k];
        cplx<R> wd = cmulc(d, w);
        x[p] = {s.x - wd.y, s.y + wd.x};
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if ((M * NL) % NT == 0 || e < M * NL) buf[e] = x[p];
    }
    __syncthreads();
    fft_lines<R, M, NL, NT, true, 2>(buf, tw);
#pragma unroll 4
    for (int e = threadIdx.x; e < M * NL; e += NT) {
      const int line = e % NL, m = e / NL;
      const cplx<R> z = buf[e];
      stage[(slot * NL + line) * SW + m] = f32_to_bf16_bits(z.x) | (f32_to_bf16_bits(z.y) << 16);
    }
    __syncthreads();   // buf is rewritten by the next field
  }
  // brick j along z: cells base(j) + c, c = 16 dx + 4 dy + dz in [0, 32)
  using W = typename CellWords<NSLOT>::T;
  const uint16_t* st = (const uint16_t*)stage;
  W* out = (W*)a.out;
  const size_t base0 = (size_t)mesh_x(ix0, G) + mesh_y(iy0, G);
#pragma unroll 2
  for (int t = threadIdx.x; t < (G / 4) * 32; t += NT) {
    const int j = t >> 5, c = t & 31;
    const int line = (c >> 4) * 4 + ((c >> 2) & 3), iz = 4 * j + (c & 3);
    uint32_t wv[NSLOT / 2];
#pragma unroll
    for (int q = 0; q < NSLOT / 2; ++q)
      wv[q] = (uint32_t)st[2 * ((2 * q) * NL * SW + line * SW) + iz] |
              ((uint32_t)st[2 * ((2 * q + 1) * NL * SW + line * SW) + iz] << 16);
    W v;
    if constexpr (NSLOT == 8) v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    else if constexpr (NSLOT == 6) v = make_uint3(wv[0], wv[1], wv[2]);
    else v = make_uint2(wv[0], wv[1]);
    out[base0 + mesh_z(4 * j) + c] = v;
  }
}

// --------------------------------------------------------------- dispatch --
template <typename R, int G>
void build_grids_g(const GridBuildArgs& a, hipStream_t s) {
  using S = Shape<R, G>;
  const int nzb = S::M / S::NBC;
  hipLaunchKernelGGL((k_xpass_inverse<R, G>), dim3(G * (S::M / S::NBX)), dim3(S::NT), 0, s, a);
  hipLaunchKernelGGL((k_ypass<R, G, true>), dim3(a.nfft * G * nzb), dim3(S::NT), 0, s,
                     (cplx<R>*)a.scratch, (const cplx<R>*)a.twiddle);
  const int nyb = G / S::NL;
  const dim3 zg(G * nyb);
  if constexpr (std::is_same<R, float>::value) {
    if constexpr (G <= 512) {   // the staged outputs of 8 lines fit in LDS
      if (a.out_type == GT_BF16) {
        const dim3 zb((G / 2) * (G / 4));
        if (a.nslot == 8) hipLaunchKernelGGL((k_zpass_c2r_bf16<G, 8>), zb, dim3(S::NT), 0, s, a);
        else if (a.nslot == 6) hipLaunchKernelGGL((k_zpass_c2r_bf16<G, 6>), zb, dim3(S::NT), 0, s, a);
        else hipLaunchKernelGGL((k_zpass_c2r_bf16<G, 4>), zb, dim3(S::NT), 0, s, a);
        return;
      }
    }
    if (a.out_type == GT_BF16) {
      if (a.nslot == 8) hipLaunchKernelGGL((k_zpass_c2r<R, G, 8, GT_BF16>), zg, dim3(S::NT), 0, s, a);
      else if (a.nslot == 6) hipLaunchKernelGGL((k_zpass_c2r<R, G, 6, GT_BF16>), zg, dim3(S::NT), 0, s, a);
      else hipLaunchKernelGGL((k_zpass_c2r<R, G, 4, GT_BF16>), zg, dim3(S::NT), 0, s, a);
    } else {
      if (a.nslot == 8) hipLaunchKernelGGL((k_zpass_c2r<R, G, 8, GT_F32>), zg, dim3(S::NT), 0, s, a);
      else hipLaunchKernelGGL((k_zpass_c2r<R, G, 4, GT_F32>), zg, dim3(S::NT), 0, s, a);
    }
  } else {
    if (a.nslot == 8) hipLaunchKernelGGL((k_zpass_c2r<R, G, 8, GT_F64>), zg, dim3(S::NT), 0, s, a);
    else if (a.nslot == 6) hipLaunchKernelGGL((k_zpass_c2r<R, G, 6, GT_F64>), zg, dim3(S::NT), 0, s, a);
    else hipLaunchKernelGGL((k_zpass_c2r<R, G, 4, GT_F64>), zg, dim3(S::NT), 0, s, a);
  }
}

template <typename R, int G>
void power_spectrum_g(const PkArgs& a, hipStream_t s) {
  using S = Shape<R, G>;
  const int halves = a.auto_mode ? 1 : 2;
  const int nyb = G / S::NL;
  hipLaunchKernelGGL((k_zpass_r2c<R, G>), dim3(halves * G * nyb), dim3(S::NT), 0, s, a);
  const int nzb = S::M / S::NBC;
  hipLaunchKernelGGL((k_ypass<R, G, false>), dim3(halves * G * nzb), dim3(S::NT), 0, s,
                     (cplx<R>*)a.scratch, (const cplx<R>*)a.twiddle);
  constexpr int NBb = S::NBC / 2 > 0 ? S::NBC / 2 : 1;
  hipLaunchKernelGGL((k_xpass_accum<R, G>), dim3(halves * G * (S::M / NBb)), dim3(S::NT), 0, s, a);
}

template <typename R, int G>
void bin_g(const PkArgs& a, hipStream_t s) {
  const size_t plane = (size_t)G * G * (G / 2);
  const size_t blocks = std::min<size_t>((plane + 255) / 256, 2048);
  hipLaunchKernelGGL((k_bin_max<R, G>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_bin_fixed<R, G>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_bin_sums, dim3(1), dim3(256), 0, s, a);
}

template <typename R>
void build_grids_r(const GridBuildArgs& a, hipStream_t s) {
  switch (a.G) {
    case 8: build_grids_g<R, 8>(a, s); break;
    case 16: build_grids_g<R, 16>(a, s); break;
    case 32: build_grids_g<R, 32>(a, s); break;
    case 64: build_grids_g<R, 64>(a, s); break;
    case 128: build_grids_g<R, 128>(a, s); break;
    case 256: build_grids_g<R, 256>(a, s); break;
    case 512: build_grids_g<R, 512>(a, s); break;
    case 1024: build_grids_g<R, 1024>(a, s); break;
    default: break;
  }
}

template <typename R>
void bin_r(const PkArgs& a, hipStream_t s) {
  switch (a.G) {
    case 8: bin_g<R, 8>(a, s); break;
    case 16: bin_g<R, 16>(a, s); break;
    case 32: bin_g<R, 32>(a, s); break;
    case 64: bin_g<R, 64>(a, s); break;
    case 128: bin_g<R, 128>(a, s); break;
    case 256: bin_g<R, 256>(a, s); break;
    case 512: bin_g<R, 512>(a, s); break;
    case 1024: bin_g<R, 1024>(a, s); break;
    default: break;
  }
}

template <typename R>
void power_spectrum_r(const PkArgs& a, hipStream_t s) {
  switch (a.G) {
    case 8: power_spectrum_g<R, 8>(a, s); break;
    case 16: power_spectrum_g<R, 16>(a, s); break;
    case 32: power_spectrum_g<R, 32>(a, s); break;
    case 64: power_spectrum_g<R, 64>(a, s); break;
    case 128: power_spectrum_g<R, 128>(a, s); break;
    case 256: power_spectrum_g<R, 256>(a, s); break;
    case 512: power_spectrum_g<R, 512>(a, s); break;
    case 1024: power_spectrum_g<R, 1024>(a, s); break;
    default: break;
  }
}

}  // namespace

void launch_build_grids(const GridBuildArgs& a, hipStream_t s) {
  if (a.fp64) build_grids_r<double>(a, s);
  else build_grids_r<float>(a, s);
}

void launch_power_spectrum(const PkArgs& a, hipStream_t s) {
  if (a.fp64) power_spectrum_r<double>(a, s);
  else power_spectrum_r<float>(a, s);
}

void launch_bin(const PkArgs& a, hipStream_t s) {
  if (a.fp64) bin_r<double>(a, s);
  else bin_r<float>(a, s);
}

}  // namespace fdf
