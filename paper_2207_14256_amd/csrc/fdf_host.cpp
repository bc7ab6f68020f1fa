// Host runtime and C ABI of the FastDF push (see include/fastdf.h).
//
// Host work is FP64 bookkeeping: configuration checks, the constant-Delta-log-a
// schedule with its conformal-time integrals (sec. 3.3), the sigma_8
// normalisation of the seeded field, <eps>(a) for the density estimator
// (sec. 2.2), carving the caller's workspace, and enqueuing kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fastdf.h"
#include "fdf_internal.h"

using namespace fdf;

namespace {

constexpr double kCkms = 299792.458;          // speed of light [km/s]
constexpr double kBoltzmannEvK = 8.617333262e-5;
constexpr double kTnuKelvin = 1.95;           // present neutrino temperature (sec. 2)
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxBins = 256;
// Spectrum bins region: [3][kMaxBins] binary64 results, then the exact sums
// [5][kMaxBins] (64-bit words), then the largest |P| word.
constexpr size_t kBinsBytes = (8 * kMaxBins + 2) * 8;
constexpr size_t kAlign = 256;

double t_nu_ev() { return kTnuKelvin * kBoltzmannEvK; }
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------- quadrature --
struct GaussLegendre {
  double x[16], w[16];
  GaussLegendre() {
    // nodes of P_16 by Newton's method on the Legendre recurrence
    const int n = 16;
    for (int i = 0; i < n; ++i) {
      long double z = cosl(kPi * (i + 0.75L) / (n + 0.5L)), pp = 0;
      for (int it = 0; it < 100; ++it) {
        long double p1 = 1, p2 = 0;
        for (int j = 1; j <= n; ++j) {
          long double p3 = p2;
          p2 = p1;
          p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1);
        long double dz = p1 / pp;
        z -= dz;
        if (fabsl(dz) < 1e-19L) break;
      }
      x[i] = (double)z;
      w[i] = (double)(2 / ((1 - z * z) * pp * pp));
    }
  }
  template <class F> double integrate(F f, double lo, double hi, int panels) const {
    long double sum = 0;
    const double h = (hi - lo) / panels;
    for (int p = 0; p < panels; ++p) {
      const double c = lo + (p + 0.5) * h, r = 0.5 * h;
      for (int i = 0; i < 16; ++i) sum += (long double)w[i] * r * f(c + r * x[i]);
    }
    return (double)sum;
  }
};
const GaussLegendre& gl16() { static GaussLegendre g; return g; }

struct Cosmo {
  double h, om, orad, ol;
  double H0() const { return 100.0 * h / kCkms; }
  double H(double a) const { return H0() * std::sqrt(orad / (a * a * a * a) + om / (a * a * a) + ol); }
};

// Delta tau = int_{ln a0}^{ln a1} dln a / (a H)  (sec. 3.3, step sizes)
double dtau(const Cosmo& c, double lna0, double lna1) {
  const int panels = std::max(1, (int)std::ceil(std::fabs(lna1 - lna0) / 0.02));
  return gl16().integrate([&](double l) { const double a = std::exp(l); return 1.0 / (a * c.H(a)); },
                          lna0, lna1, panels);
}

// tau(a) from a = 0 (the integrand vanishes like a^(1/2) or a as a -> 0)
double conformal_time(const Cosmo& c, double a) {
  const double l1 = std::log(a), l0 = l1 - 80.0;
  return dtau(c, l0, l1);
}

double bbks(double k, double gamma, double h) {
  const double q = k / (gamma * h);
  if (q <= 0) return 1.0;
  const double b = 16.1 * q, cc = 5.46 * q, d = 6.71 * q;
  const double poly = 1.0 + 3.89 * q + b * b + cc * cc * cc + (d * d) * (d * d);
  return std::log1p(2.34 * q) / (2.34 * q) * std::pow(poly, -0.25);
}

double tophat(double x) {
  if (std::fabs(x) < 0.1) {
    const double x2 = x * x;
    return 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0 + x2 * x2 * x2 * x2 / 1330560.0;
  }
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

// A with sigma(8 Mpc/h) = sigma8 for P = A k^ns T_BBKS^2
double power_amplitude(double sigma8, double ns, double gamma, double h) {
  const double R = 8.0 / h;
  auto f_lnk = [&](double l) {
    const double k = std::exp(l), t = bbks(k, gamma, h), w = tophat(k * R);
    return k * k * k * std::pow(k, ns) * t * t * w * w;
  };
  auto f_k = [&](double k) {
    const double t = bbks(k, gamma, h), w = tophat(k * R);
    return k * k * std::pow(k, ns) * t * t * w * w;
  };
  double s2 = gl16().integrate(f_lnk, std::log(1e-7), 0.0, 400);
  s2 += gl16().integrate(f_k, 1.0, 1000.0, 20000);
  s2 /= 2.0 * kPi * kPi;
  return sigma8 * sigma8 / s2;
}

// <eps>(a) = int q^2 sqrt(q^2 + m^2 a^2) fbar / int q^2 fbar  (eq. rho_def normalisation)
double mean_energy(double m, double a) {
  const double T = t_nu_ev(), ma = m * a;
  auto num = [&](double x) { return x * x * std::sqrt(x * x * T * T + ma * ma) / (1.0 + std::exp(x)); };
  auto den = [&](double x) { return x * x / (1.0 + std::exp(x)); };
  return gl16().integrate(num, 0.0, 200.0, 800) / gl16().integrate(den, 0.0, 200.0, 800);
}

// Radiation-to-matter potential factor g(a) = (10/9) Phi(y)/Phi(0), y = a/a_eq,
// Phi(y)/Phi(0) = 1 - y (s^2 + 4 s + 5) / (10 (s+1)^4), s = sqrt(1+y)
// (Kodama-Sasaki super-horizon solution without cancellation), and dg/da.
void radmat_factor(double a, double om, double orad, double* g, double* dg) {
  const double aeq = orad / om, y = a / aeq, s = std::sqrt(1.0 + y);
  const double num = y + 6.0 + 4.0 * s, den = std::pow(s + 1.0, 4);
  const double hfun = y * num / den;
  const double dnum = 1.0 + 2.0 / s, dden = 4.0 * std::pow(s + 1.0, 3) / (2.0 * s);
  const double dh = (num + y * dnum) / den - y * num * dden / (den * den);
  *g = (10.0 / 9.0) * (1.0 - hfun / 10.0);
  *dg = -(1.0 / 9.0) * dh / aeq;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) { int r = 0; while ((1 << r) < v) ++r; return r; }

// ----------------------------------------------------------------- layout --
struct Layout {
  size_t twiddle_d, twiddle_f, seg, bins, dep, scratch, dens, fields, parts, sort_count, sort_scan, sort_rank,
      sort_bucket, sort_src, total;
  int64_t sort_keys_max;
  int grid_sets;
  size_t field_dk_bytes, field_grid_bytes, scratch_bytes, dens_bytes, parts_bytes;
  int nslot;
};

bool eom_potentials(const fdf_config& c) { return c.eom == FDF_EOM_EXACT || c.eom == FDF_EOM_CANONICAL; }
// Slots per mesh cell.  Separable form: grad psi and phi-dot (4) when
// psi = phi; else grad psi, grad phi and phi-dot (8).  When phi-dot is zero
// the cell drops it and the pad: 6 slots (binary64: three 16-byte loads per
// corner; bfloat16: one 12-byte load), unless pad_mesh asks for the aligned
// 16-byte bfloat16 cell.
int slots_for(const fdf_config& c) {
  if (c.eom == FDF_EOM_SEPARABLE) {
    if (c.slip_amp == 0.0) return 4;
    const bool f64 = c.precision == FDF_PREC_FP64;
    if (c.potential_model == FDF_MODEL_RADMAT) return 8;
    return (f64 || !c.pad_mesh) ? 6 : 8;
  }
  return eom_potentials(c) ? 8 : 4;
}
int fft_planes(const fdf_config& c) { return eom_potentials(c) ? 8 : 7; }

// Stored slot of a grid quantity (0-2 grad psi, 3-5 grad phi, 6 phi-dot,
// 7 psi, 8 phi, 9 phi + psi): >= 0 the slot, -1 identically zero in this
// configuration, -2 not stored for this equation of motion.
int grid_slot(const fdf_config& c, int quantity) {
  const bool tdep = c.potential_model == FDF_MODEL_RADMAT;
  const bool same = c.slip_amp == 0.0;   // phi = psi
  switch (c.eom) {
    case FDF_EOM_SEPARABLE:
      if (slots_for(c) == 8) return quantity <= 5 ? quantity : quantity == 6 ? (tdep ? 6 : -1) : -2;
      if (slots_for(c) == 6) return quantity <= 5 ? quantity : quantity == 6 ? -1 : -2;
      if (quantity <= 5) return quantity % 3;
      return quantity == 6 ? (tdep ? 3 : -1) : -2;
    case FDF_EOM_EXACT:
      if (quantity <= 5) return quantity;
      return quantity == 6 ? (tdep ? 6 : -1) : quantity == 9 ? 7 : -2;
    case FDF_EOM_CANONICAL:
      if (quantity <= 5) return quantity;
      return quantity == 7 ? 6 : quantity == 8 ? 7 : -2;
    default:
      if (quantity <= 2) return quantity;
      return (quantity <= 5 && same) ? quantity - 3 : -2;
  }
}
size_t real_bytes(const fdf_config& c) { return c.precision == FDF_PREC_FP64 ? 8 : 4; }
size_t slot_bytes(const fdf_config& c) { return c.precision == FDF_PREC_FP64 ? 8 : 2; }
size_t particle_bytes(const fdf_config& c) { return c.precision == FDF_PREC_FP64 ? 76 : 40; }
int arrays_per_species(const fdf_config& c) { return c.precision == FDF_PREC_FP64 ? 10 : 10; }

Layout plan(const fdf_config& c) {
  Layout L{};
  const size_t G = (size_t)c.grid_n, rb = real_bytes(c), cb = 2 * rb;
  L.nslot = slots_for(c);
  L.field_dk_bytes = align_up(G * G * (G / 2) * cb);
  L.field_grid_bytes = align_up(G * G * G * (size_t)L.nslot * slot_bytes(c));
  L.scratch_bytes = align_up((size_t)fft_planes(c) * G * G * (G / 2) * cb);
  L.dens_bytes = align_up(4 * G * G * G * rb);   // two halves, or a 4-slot pre-IC grid
  const int copies = c.sort_every > 0 ? 2 : 1;
  L.parts_bytes = align_up((size_t)c.max_particles * particle_bytes(c) * copies +
                           (size_t)c.max_species * arrays_per_species(c) * copies * kAlign);
  size_t off = 0;
  // twiddles of the G-point transform, then those of G/2, G/4, ... 8 (the
  // analysis meshes of the spectra): the table of n points starts at entry 2 (G - n)
  L.twiddle_d = off; off += align_up(2 * G * 16);
  L.twiddle_f = off; off += align_up(2 * G * 8);
  L.seg = off; off += 2 * align_up((size_t)c.max_species * sizeof(Segment));
  L.bins = off; off += align_up(kBinsBytes);
  L.dep = off; off += kAlign;   // the fixed-point deposit's largest |value|
  L.scratch = off; off += L.scratch_bytes;
  L.dens = off; off += L.dens_bytes;
  L.grid_sets = (c.potential_model == FDF_MODEL_RADMAT && c.superstep_tol > 0) ? 2 : 1;
  L.fields = off; off += (size_t)c.max_fields * (L.field_dk_bytes + L.grid_sets * L.field_grid_bytes);
  L.parts = off; off += L.parts_bytes;
  const int64_t tmax = std::min<int64_t>(c.grid_n, 256);
  const bool sorting = c.sort_every > 0;
  L.sort_keys_max = sorting ? tmax * tmax * tmax : 0;
  L.sort_count = off; off += align_up((size_t)L.sort_keys_max * 4);
  L.sort_scan = off; off += sorting ? align_up(sort_scan_scratch_words(L.sort_keys_max) * 4) : 0;
  L.sort_rank = off; off += sorting ? align_up((size_t)c.max_particles * 4) : 0;
  L.sort_bucket = off; off += sorting ? align_up((size_t)c.max_particles * 4) : 0;
  L.sort_src = off; off += sorting ? align_up((size_t)c.max_particles * 4) : 0;
  L.total = off;
  return L;
}

const char* validate(const fdf_config* c) {
  if (!c) return "config is NULL";
  if (c->abi_version != FDF_ABI_VERSION) return "abi_version mismatch";
  if (!is_pow2(c->grid_n) || c->grid_n < 8 || c->grid_n > 1024) return "grid_n must be a power of two in [8, 1024]";
  if (!(c->box_mpc > 0) || !std::isfinite(c->box_mpc)) return "box_mpc must be positive";
  if (!(c->h > 0)) return "h must be positive";
  if (c->omega_m < 0 || c->omega_r < 0 || c->omega_l < 0 || c->omega_m + c->omega_r <= 0)
    return "need omega_m + omega_r > 0 and non-negative densities";
  if (!(c->z_begin > -1) || !(c->z_end > -1)) return "redshifts must exceed -1";
  if (c->z_begin == c->z_end) return "z_begin must differ from z_end";
  if (c->n_steps < 1) return "n_steps must be >= 1";
  if (c->precision != FDF_PREC_FP64 && c->precision != FDF_PREC_FP32) return "unknown precision";
  if (c->potential_model != FDF_MODEL_POISSON && c->potential_model != FDF_MODEL_RADMAT) return "unknown potential model";
  if (c->potential_model == FDF_MODEL_RADMAT && !(c->omega_r > 0)) return "RADMAT needs omega_r > 0";
  if (c->slip_amp < 0 || c->slip_amp >= 1 || !(c->slip_k > 0)) return "slip_amp in [0,1) and slip_k > 0 required";
  if (!(c->sigma8 > 0) || !(c->gamma > 0)) return "sigma8 and gamma must be positive";
  if (c->sort_every < 0) return "sort_every must be >= 0";
  if (c->max_fields < 1 || c->max_species < 1 || c->max_particles < 1) return "capacities must be >= 1";
  if (c->max_particles > ((int64_t)1 << 32)) return "at most 2^32 particles";
  if (!(c->superstep_tol >= 0) || !std::isfinite(c->superstep_tol)) return "superstep_tol must be >= 0";
  if (c->eom < FDF_EOM_SEPARABLE || c->eom > FDF_EOM_NEWTONIAN) return "unknown equation of motion";
  if (c->interp_order < 0 || c->interp_order > 2) return "interp_order must be 0, 1 (CIC) or 2 (TSC)";
  if (c->pad_mesh != 0 && c->pad_mesh != 1) return "pad_mesh must be 0 or 1";
  return nullptr;
}

struct FieldRec {
  uint64_t seed = 0;
  void* dk = nullptr;
  void* grid = nullptr;
  void* grid2 = nullptr;      // second grid set (super-steps)
  bool has_grid = false;
  double grid_a = 0;
  int tag[2] = {-1, -1};      // super-steps: anchor (schedule index) held by each set
};

struct SpeciesRec {
  int field = 0;
  double m = 0;
  int64_t n = 0;
  uint64_t seed = 0;
  int flags = 0;
  Segment seg[2];   // state buffers (second copy only with sorting)
  int cur = 0;
  bool pristine = false;   // state is exactly the sampled one (no pre-IC, not stepped)
  double drift_cells = 0;  // typical drift since its last re-sort, in mesh cells
};

// A captured step sequence: the host state it was captured from and the host
// state it leaves behind, so a replay can stand in for the enqueue.
struct HostStepState {
  int step_index = 0;
  bool sorted_once = false;
  std::vector<int> cur;            // per species: the copy holding its state
  std::vector<double> drift_cells; // per species
  std::vector<double> grid_a;      // per field; NaN = no grid
  std::vector<int> tags;           // per field, two super-step set tags
  std::vector<char> pristine;      // per species
  bool operator==(const HostStepState& o) const {
    if (step_index != o.step_index || cur != o.cur || sorted_once != o.sorted_once || tags != o.tags ||
        pristine != o.pristine || grid_a.size() != o.grid_a.size() ||
        drift_cells.size() != o.drift_cells.size())
      return false;
    for (size_t i = 0; i < grid_a.size(); ++i)
      if (std::memcmp(&grid_a[i], &o.grid_a[i], sizeof(double)) != 0) return false;
    for (size_t i = 0; i < drift_cells.size(); ++i)
      if (std::memcmp(&drift_cells[i], &o.drift_cells[i], sizeof(double)) != 0) return false;
    return true;
  }
};

struct GraphRec {
  int n = 0;
  std::vector<double> layout;      // fields and species that fix every device pointer
  HostStepState before, after;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct TimingRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double total_ms = 0;
  int64_t launches = 0;
  int64_t work[3] = {0, 0, 0};   // particle-updates with a drift, kick-only updates, mesh cells read
};

}  // namespace

struct fdf_ctx {
  fdf_config cfg{};
  Cosmo cos{};
  hipStream_t stream = nullptr;
  std::vector<double> a, a_half, kick1, kick2, drift;
  std::vector<int> anchors;   // super-step anchors (schedule indices), empty when unused
  double amp = 0, tau_begin = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay{};
  size_t field_next = 0, part_next = 0;
  std::vector<FieldRec> fields;
  std::vector<SpeciesRec> species;
  int step_index = 0;
  bool stepped = false;
  bool seg_dirty = true;
  int ppt = 4;
  int sort_tiles = 0;       // tiles per axis of the sort key (0: default)
  int sort_every = 0;       // current re-sort cadence
  float sort_cells = 0;     // adaptive cadence threshold in cells (0: fixed cadence)
  int persistent = 0;       // push grid size when > 0 (a multiple of 8)
  bool use_graph = false;   // capture step sequences into hipGraphs
  bool sort_predict = true; // sort keys from positions extrapolated to mid-interval
  bool sort_fused = true;   // FP32 separable: re-sorts after the first ride on the push
  int push_waves = 0;       // cap on resident push waves per SIMD (0: none)
  int sort_push_ppt = 4;    // particles per thread of the fused re-sort push
  bool sort_keys_push = true;   // the push before a re-sort writes the sort keys
  hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
  hipStream_t launch_stream = nullptr;  // stream kernels are enqueued on right now
  std::vector<GraphRec> graphs;       // captured step sequences
  bool sorted_once = false;
  std::string err;
  bool timing = false;
  TimingRec tim[FDF_KERNEL_COUNT];
  bool have_density = false;
  int density_auto = 0;
};

namespace {

int fail(fdf_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_check(fdf_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return FDF_OK;
  return fail(c, FDF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int launched(fdf_ctx* c, const char* what) { return hip_check(c, hipGetLastError(), what); }

hipStream_t stream_of(fdf_ctx* c) { return c->launch_stream ? c->launch_stream : c->stream; }

void clear_graphs(fdf_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

void timing_begin(fdf_ctx* c, int cls, std::pair<hipEvent_t, hipEvent_t>* ev) {
  if (!c->timing || c->launch_stream) return;
  TimingRec& t = c->tim[cls];
  if (t.pool.empty()) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    t.pool.push_back({e0, e1});
  }
  *ev = t.pool.back();
  t.pool.pop_back();
  (void)hipEventRecord(ev->first, c->stream);
}

void timing_end(fdf_ctx* c, int cls, std::pair<hipEvent_t, hipEvent_t>& ev) {
  if (!c->timing || c->launch_stream) return;
  (void)hipEventRecord(ev.second, c->stream);
  c->tim[cls].pending.push_back(ev);
  c->tim[cls].launches++;
}

// Work done by the launches of a timed class (counted while timing is on).
void timing_work(fdf_ctx* c, int cls, int64_t updates_drift, int64_t updates_kick, int64_t mesh_cells) {
  if (!c->timing || c->launch_stream) return;
  c->tim[cls].work[0] += updates_drift;
  c->tim[cls].work[1] += updates_kick;
  c->tim[cls].work[2] += mesh_cells;
}

void timing_collect(fdf_ctx* c) {
  for (auto& t : c->tim) {
    for (auto& ev : t.pending) {
      float ms = 0;
      (void)hipEventSynchronize(ev.second);
      (void)hipEventElapsedTime(&ms, ev.first, ev.second);
      t.total_ms += ms;
      t.pool.push_back(ev);
    }
    t.pending.clear();
  }
}

bool needs_ws(fdf_ctx* c) { return c->ws != nullptr; }

// Carve the state arrays of one copy of a species.
bool carve_species(fdf_ctx* c, Segment& s, int64_t n) {
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  auto take = [&](size_t bytes) -> void* {
    const size_t sz = align_up(bytes);
    if (c->part_next + sz > c->lay.parts_bytes) return nullptr;
    void* p = c->ws + c->lay.parts + c->part_next;
    c->part_next += sz;
    return p;
  };
  std::memset(&s, 0, sizeof(s));
  for (int d = 0; d < 3; ++d) {
    if (f64) {
      s.xd[d] = (double*)take(n * 8);
      s.qd[d] = (double*)take(n * 8);
      s.q0d[d] = (double*)take(n * 8);
      if (!s.xd[d] || !s.qd[d] || !s.q0d[d]) return false;
    } else {
      s.xu[d] = (uint32_t*)take(n * 4);
      s.q0f[d] = (float*)take(n * 4);
      s.dqf[d] = (float*)take(n * 4);
      if (!s.xu[d] || !s.q0f[d] || !s.dqf[d]) return false;
    }
  }
  s.id = (uint32_t*)take(n * 4);
  s.n = n;
  return s.id != nullptr;
}

GridBuildArgs grid_recipe(fdf_ctx* c, const FieldRec& f, double a, bool pre_ic_grid) {
  GridBuildArgs g{};
  const fdf_config& cf = c->cfg;
  g.G = cf.grid_n;
  g.fp64 = cf.precision == FDF_PREC_FP64;
  g.kf = 2.0 * kPi / cf.box_mpc;
  const double base = -1.5 * c->cos.H0() * c->cos.H0() * cf.omega_m;   // Poisson: D(a)/a = 1
  double gf = 1.0, dgf = 0.0;
  if (cf.potential_model == FDF_MODEL_RADMAT) radmat_factor(a, cf.omega_m, cf.omega_r, &gf, &dgf);
  g.tr.c_phi = base * gf;
  g.tr.c_phidot = base * (a * a * c->cos.H(a) * dgf);
  g.tr.slip_amp = cf.slip_amp;
  g.tr.slip_k = cf.slip_k;
  g.delta_k = f.dk;
  g.scratch = c->ws + c->lay.scratch;
  g.twiddle = c->ws + (g.fp64 ? c->lay.twiddle_d : c->lay.twiddle_f);
  const bool phidot = cf.potential_model == FDF_MODEL_RADMAT;
  int n = 0;
  if (pre_ic_grid) {
    g.nslot = 4;
    g.out_type = g.fp64 ? GT_F64 : GT_F32;
    const int kinds[4] = {SK_DX_PSI, SK_DY_PSI, SK_DZ_PSI, SK_PSI};
    for (int i = 0; i < 4; ++i) { g.kind[n] = kinds[i]; g.slot[n] = i; ++n; }
    g.out = c->ws + c->lay.dens;
  } else {
    g.nslot = c->lay.nslot;
    g.out_type = g.fp64 ? GT_F64 : GT_BF16;
    g.out = f.grid;
    g.kind[n] = SK_DX_PSI; g.slot[n++] = 0;
    g.kind[n] = SK_DY_PSI; g.slot[n++] = 1;
    g.kind[n] = SK_DZ_PSI; g.slot[n++] = 2;
    if (cf.eom != FDF_EOM_SEPARABLE) {
      if (eom_potentials(cf)) {
        g.kind[n] = SK_DX_PHI; g.slot[n++] = 3;
        g.kind[n] = SK_DY_PHI; g.slot[n++] = 4;
        g.kind[n] = SK_DZ_PHI; g.slot[n++] = 5;
      }
      if (cf.eom == FDF_EOM_EXACT) {
        if (phidot) { g.kind[n] = SK_PHIDOT; g.slot[n++] = 6; }
        g.kind[n] = SK_PHI_PSI; g.slot[n++] = 7;
      } else if (cf.eom == FDF_EOM_CANONICAL) {
        g.kind[n] = SK_PSI; g.slot[n++] = 6;
        g.kind[n] = SK_PHI; g.slot[n++] = 7;
      }
    } else if (g.nslot >= 6) {
      g.kind[n] = SK_DX_PHI; g.slot[n++] = 3;
      g.kind[n] = SK_DY_PHI; g.slot[n++] = 4;
      g.kind[n] = SK_DZ_PHI; g.slot[n++] = 5;
      if (phidot) { g.kind[n] = SK_PHIDOT; g.slot[n++] = 6; }
    } else if (phidot) {
      g.kind[n] = SK_PHIDOT; g.slot[n++] = 3;
    }
  }
  g.nfft = n;
  return g;
}

int build_grid(fdf_ctx* c, int field, double a, int buf = 0) {
  FieldRec& f = c->fields[field];
  c->have_density = false;   // the FFT scratch holds the FP32 form's density copy
  GridBuildArgs g = grid_recipe(c, f, a, false);
  if (buf == 1) g.out = f.grid2;
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_GRID, &ev);
  launch_build_grids(g, stream_of(c));
  timing_end(c, FDF_KERNEL_GRID, ev);
  if (buf == 0) {
    f.has_grid = true;
    f.grid_a = a;
  }
  return launched(c, "grid build");
}

// Two device tables of segments: one per buffer copy (all species sort together,
// so they always sit in the same copy).
int upload_segments(fdf_ctx* c) {
  if (!c->seg_dirty) return FDF_OK;
  const int64_t per = push_chunk_particles(c->ppt);
  const size_t table = align_up((size_t)c->cfg.max_species * sizeof(Segment));
  for (int copy = 0; copy < 2; ++copy) {
    std::vector<Segment> segs;
    int64_t chunk = 0;
    for (auto& s : c->species) {
      Segment g = s.seg[copy];
      g.grid = c->fields[s.field].grid;
      g.grid2 = c->fields[s.field].grid2;
      g.m = s.m;
      g.chunk_begin = chunk;
      chunk += (s.n + per - 1) / per;
      segs.push_back(g);
    }
    int rc = hip_check(c, hipMemcpyAsync(c->ws + c->lay.seg + copy * table, segs.data(),
                                         segs.size() * sizeof(Segment), hipMemcpyHostToDevice, c->stream),
                       "segment upload");
    if (rc) return rc;
  }
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "segment upload");
  c->seg_dirty = false;
  return rc;
}

// LDS bytes per 4-wave push block that leave room for exactly `waves` blocks
// (one wave per SIMD each) in the 160 KB of a CU; 0 for no cap.
int push_lds_reserve(int waves) {
  if (waves <= 0) return 0;
  const int lds_per_cu = 160 * 1024;
  return (lds_per_cu / (waves + 1) + 256 + 255) / 256 * 256;
}

// Buckets per axis of the sort: default one per 4^3 cells, at most 256.
int sort_tiles_of(fdf_ctx* c) {
  const int tmax = std::min(c->cfg.grid_n, 256);
  int t = c->sort_tiles > 0 ? c->sort_tiles : std::max(1, c->cfg.grid_n / 4);
  return std::min(t, tmax);
}

// Drift of a mean-momentum particle (|q| = 3.151 T) of mass m over one drift
// of length dt at a, in mesh cells: the adaptive sort cadence of a species.
double typical_drift_cells(fdf_ctx* c, double dt, double a, double m) {
  const double q = 3.151374 * t_nu_ev();
  const double v = q / std::sqrt(q * q + m * m * a * a);
  return std::fabs(dt) * v * c->cfg.grid_n / c->cfg.box_mpc;
}

// Species sort on their own cadence (a mask of up to 64 species); more
// species than that all sort together, at the cadence of the fastest.
bool per_species_sorting(const fdf_ctx* c) { return c->species.size() <= 64; }

// Prediction of a re-sort: order by x + v tau at scale factor a_mid.
struct SortPrediction { double tau = 0, a_mid = 0; };

// Spatial re-sort of every species into its other buffer copy, ordered by
// the positions extrapolated by predict_tau at scale factor a_pred.
SortArgs sort_args(fdf_ctx* c, const SpeciesRec& s, double predict_tau, double a_pred) {
  const int tiles = sort_tiles_of(c);
  SortArgs a{};
  a.seg = s.seg[s.cur];
  a.dst = s.seg[s.cur ^ 1];
  a.predict_tau = predict_tau;
  a.ma = s.m * a_pred;
  a.fp64 = c->cfg.precision == FDF_PREC_FP64;
  a.grid_n = c->cfg.grid_n;
  a.cell_shift = 32 - ilog2(c->cfg.grid_n);
  a.fine_bits = ilog2(c->cfg.grid_n / tiles);
  a.box = c->cfg.box_mpc;
  a.nkeys = (int64_t)tiles * tiles * tiles;
  a.count = (uint32_t*)(c->ws + c->lay.sort_count);
  a.scan_scratch = (uint32_t*)(c->ws + c->lay.sort_scan);
  a.rank = (uint32_t*)(c->ws + c->lay.sort_rank);
  a.bucket = (uint32_t*)(c->ws + c->lay.sort_bucket);
  a.src = (uint32_t*)(c->ws + c->lay.sort_src);
  return a;
}

// resample: a species whose state is still the sampled one moves its ids
// alone and is sampled again, by id, into the sorted slots (the same values
// as moving the whole state from the random sampling order, at a fraction of
// the scattered writes).
int sort_species(fdf_ctx* c, const std::vector<SortPrediction>& pred, const std::vector<char>& due,
                 bool resample) {
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_SORT, &ev);
  for (size_t i = 0; i < c->species.size(); ++i) {
    if (!due[i]) continue;
    SpeciesRec& s = c->species[i];
    SortArgs a = sort_args(c, s, pred[i].tau, pred[i].a_mid);
    a.id_only = resample && s.pristine;
    launch_sort(a, stream_of(c));
    if (a.id_only) {
      SampleArgs sa{};
      sa.seg = s.seg[s.cur ^ 1];
      sa.fp64 = c->cfg.precision == FDF_PREC_FP64;
      sa.by_id = 1;
      sa.seed = s.seed;
      sa.box = c->cfg.box_mpc;
      sa.t_nu = t_nu_ev();
      launch_sample_species(sa, stream_of(c));
    }
    s.cur ^= 1;
  }
  timing_end(c, FDF_KERNEL_SORT, ev);
  return launched(c, "sort");
}

// A re-sort carried out by the push of the step: the due species in batches
// of up to kMaxSortJobs (as many as the bucket-count buffer holds), each
// batch ranked by one launch and scanned together, then pushed by one launch
// that writes the updated state in sorted order into the other copy (pa
// describes the step's push).  The rank passes are timed as sorting, the
// pushes on their own.  keyed: the push of the previous step has written the
// (single) due species' sort keys.
int sort_push_species(fdf_ctx* c, const std::vector<SortPrediction>& pred, const std::vector<char>& due,
                      const PushArgs& pa, size_t table, bool keyed) {
  const size_t ns = c->species.size();
  const int tiles = sort_tiles_of(c);
  const int64_t nkeys = (int64_t)tiles * tiles * tiles;
  const int64_t max_jobs = std::min<int64_t>(kMaxSortJobs, std::max<int64_t>(1, c->lay.sort_keys_max / nkeys));
  const Segment* tables[2] = {(const Segment*)(c->ws + c->lay.seg), (const Segment*)(c->ws + c->lay.seg + table)};
  size_t i = 0;
  while (true) {
    while (i < ns && !due[i]) ++i;
    if (i >= ns) break;
    SpeciesRec& s0 = c->species[i];
    SortArgs a = sort_args(c, s0, pred[i].tau, pred[i].a_mid);
    SortBatch& b = a.batch;
    b = SortBatch{};
    b.tables[0] = tables[0];
    b.tables[1] = tables[1];
    int64_t blocks = 0, base = 0;
    std::vector<size_t> members;
    std::vector<char> mesh(c->fields.size(), 0);
    for (; i < ns && b.njobs < max_jobs; ++i) {
      if (!due[i]) continue;
      const SpeciesRec& s = c->species[i];
      const int j = b.njobs++;
      b.job_species[j] = (int32_t)i;
      b.job_cur[j] = s.cur;
      b.job_block[j] = blocks;
      b.job_base[j] = base;
      b.job_tau[j] = pred[i].tau;
      b.job_ma[j] = s.m * pred[i].a_mid;
      blocks += (s.n + kSortBlock - 1) / kSortBlock;
      base += s.n;
      members.push_back(i);
      mesh[s.field] = 1;
    }
    b.job_block[b.njobs] = blocks;
    // keys written by the previous push (one species) sit in the rank array
    // itself: each rank block reads its keys before it writes its ranks
    if (keyed && b.njobs == 1) a.keys = a.rank;
    std::pair<hipEvent_t, hipEvent_t> ev;
    timing_begin(c, FDF_KERNEL_SORT, &ev);
    launch_sort_rank_batch(a, stream_of(c));
    timing_end(c, FDF_KERNEL_SORT, ev);
    PushArgs p = pa;
    p.seg = tables[0];
    p.seg_alt = tables[1];
    p.dseg = nullptr;
    p.alt_mask = p.skip_mask = 0;
    p.nseg = 1;
    p.total_chunks = blocks;
    p.xcd_blocks = 0;
    p.persistent = 0;
    p.ppt = c->sort_push_ppt;
    p.lds_reserve = 0;   // the cap on resident waves is the plain push's; this kernel runs at full occupancy
    p.sort_src = a.src;
    p.sort_rank = a.rank;
    p.sort_bucket = a.bucket;
    p.sort_start = a.count;
    p.sort_nkeys = nkeys;
    p.sort_batch = b;
    timing_begin(c, FDF_KERNEL_PUSH_SORT, &ev);
    launch_push_sort(p, stream_of(c));
    timing_end(c, FDF_KERNEL_PUSH_SORT, ev);
    int64_t meshes = 0;
    for (char r : mesh) meshes += r;
    timing_work(c, FDF_KERNEL_PUSH_SORT, base, 0,
                meshes * (int64_t)c->cfg.grid_n * c->cfg.grid_n * c->cfg.grid_n * (pa.blend ? 2 : 1));
    for (size_t m : members) c->species[m].cur ^= 1;
    const int rc = launched(c, "sort + push");
    if (rc) return rc;
  }
  return FDF_OK;
}

// Grid of the segment-balanced XCD mapping of a launch over every species
// (8 times the largest share of an XCD), or 0 for a single species.
int64_t xcd_blocks(fdf_ctx* c) {
  if (c->species.size() < 2) return 0;
  const int64_t per = push_chunk_particles(c->ppt);
  int64_t most = 0;
  for (int64_t x = 0; x < 8; ++x) {
    int64_t share = 0;
    for (auto& s : c->species) {
      const int64_t n = (s.n + per - 1) / per;
      share += n * (x + 1) / 8 - n * x / 8;
    }
    most = std::max(most, share);
  }
  return 8 * most;
}

int64_t total_chunks(fdf_ctx* c) {
  const int64_t per = push_chunk_particles(c->ppt);
  int64_t t = 0;
  for (auto& s : c->species) t += (s.n + per - 1) / per;
  return t;
}

OutputArgs output_args(fdf_ctx* c, const SpeciesRec& s) {
  OutputArgs o{};
  o.seg = s.seg[s.cur];
  o.fp64 = c->cfg.precision == FDF_PREC_FP64;
  o.G = c->cfg.grid_n;
  o.pre_ic = (s.flags & FDF_SPECIES_PRE_IC) != 0;
  o.seed = s.seed;
  o.t_nu = t_nu_ev();
  o.box = c->cfg.box_mpc;
  o.a = c->a[c->step_index];
  o.m = s.m;
  return o;
}

// Byte offset in the FFT scratch of the FP32 form's binary32 density halves:
// behind the four transform planes of the largest mesh (two halves and the
// momentum spectrum's two accumulators), 8 G^3 bytes, inside the scratch's
// 28 G^3 bytes.
size_t density_copy_offset(const fdf_ctx* c) {
  const size_t G = (size_t)c->cfg.grid_n;
  return 4 * (G * G * (G / 2)) * 8;
}

// First complex entry of the n-point table in the twiddle regions.
size_t twiddle_entry(int G, int n) { return 2 * (size_t)(G - n); }

void fill_twiddles(fdf_ctx* c) {
  const int G = c->cfg.grid_n;
  std::vector<double> td(4 * (size_t)G, 0.0);
  std::vector<float> tf(4 * (size_t)G, 0.0f);
  for (int n = G; n >= 8; n /= 2) {
    const size_t base = 2 * twiddle_entry(G, n);
    for (int m = 0; m < n; ++m) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * m / n;
      td[base + 2 * m] = (double)cosl(ang);
      td[base + 2 * m + 1] = (double)sinl(ang);
      tf[base + 2 * m] = (float)cosl(ang);
      tf[base + 2 * m + 1] = (float)sinl(ang);
    }
  }
  (void)hipMemcpy(c->ws + c->lay.twiddle_d, td.data(), td.size() * 8, hipMemcpyHostToDevice);
  (void)hipMemcpy(c->ws + c->lay.twiddle_f, tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
}

int add_field_slot(fdf_ctx* c, int32_t* id) {
  if ((int)c->fields.size() >= c->cfg.max_fields) return fail(c, FDF_ERR_CAPACITY, "max_fields reached");
  FieldRec f;
  char* base = c->ws + c->lay.fields + c->field_next;
  f.dk = base;
  f.grid = base + c->lay.field_dk_bytes;
  f.grid2 = c->lay.grid_sets > 1 ? base + c->lay.field_dk_bytes + c->lay.field_grid_bytes : nullptr;
  c->field_next += c->lay.field_dk_bytes + c->lay.grid_sets * c->lay.field_grid_bytes;
  c->fields.push_back(f);
  *id = (int32_t)c->fields.size() - 1;
  return FDF_OK;
}

int new_species(fdf_ctx* c, int32_t field_id, double m, int64_t n, uint64_t seed, int flags, int32_t* sid) {
  if (field_id < 0 || field_id >= (int)c->fields.size()) return fail(c, FDF_ERR_ARG, "bad field id");
  if (!(m >= 0) || !std::isfinite(m)) return fail(c, FDF_ERR_ARG, "mass must be finite and >= 0");
  if (n < 1) return fail(c, FDF_ERR_ARG, "need at least one particle");
  if (c->stepped) return fail(c, FDF_ERR_STATE, "species must be added before the first step");
  if ((int)c->species.size() >= c->cfg.max_species) return fail(c, FDF_ERR_CAPACITY, "max_species reached");
  int64_t tot = n;
  for (auto& s : c->species) tot += s.n;
  if (tot > c->cfg.max_particles) return fail(c, FDF_ERR_CAPACITY, "max_particles exceeded");
  SpeciesRec s;
  s.field = field_id; s.m = m; s.n = n; s.seed = seed; s.flags = flags;
  const size_t save = c->part_next;
  if (!carve_species(c, s.seg[0], n)) { c->part_next = save; return fail(c, FDF_ERR_CAPACITY, "workspace particles full"); }
  if (c->cfg.sort_every > 0 && !carve_species(c, s.seg[1], n)) {
    c->part_next = save;
    return fail(c, FDF_ERR_CAPACITY, "workspace particles full");
  }
  c->species.push_back(s);
  c->seg_dirty = true;
  *sid = (int32_t)c->species.size() - 1;
  return FDF_OK;
}

}  // namespace

// -------------------------------------------- static scratch (no allocation) --
// Device memory of fdf_power_spectrum_noalloc: one array per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel or a
// copy; it uses the address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
constexpr int kStaticMaxMesh = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The static scratch of the current device (resolved once per device).
int static_scratch(fdf_ctx* c, char** out) {
  int dev = -1;
  int rc = hip_check(c, hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(c, FDF_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    rc = hip_check(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return FDF_OK;
}

// Static scratch bytes of a spectrum on a G^3 mesh: bins, the maximum word,
// the deposit halves (8 bytes per cell each), four FFT planes and (FP32 form)
// the binary32 halves.
size_t static_scratch_bytes(bool f64, int G) {
  const size_t g3 = (size_t)G * G * G, plane = (size_t)G * G * (G / 2) * (f64 ? 16 : 8);
  return align_up(kBinsBytes) + kAlign + align_up(2 * g3 * 8) + align_up(4 * plane) +
         (f64 ? 0 : align_up(2 * g3 * 4));
}

}  // namespace

// ============================================================== C ABI ======
extern "C" {

const char* fdf_status_string(int s) {
  switch (s) {
    case FDF_OK: return "ok";
    case FDF_ERR_ARG: return "invalid argument";
    case FDF_ERR_STATE: return "invalid state";
    case FDF_ERR_WORKSPACE: return "workspace missing or too small";
    case FDF_ERR_HIP: return "HIP runtime error";
    case FDF_ERR_CAPACITY: return "capacity exceeded";
    case FDF_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* fdf_last_error(const fdf_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fdf_workspace_size(const fdf_config* cfg, size_t* bytes) {
  if (validate(cfg) || !bytes) return FDF_ERR_ARG;
  *bytes = plan(*cfg).total;
  return FDF_OK;
}

int fdf_create(const fdf_config* cfg, void* stream, fdf_ctx** out) {
  if (!out) return FDF_ERR_ARG;
  *out = nullptr;
  if (validate(cfg)) return FDF_ERR_ARG;
  fdf_ctx* c = new fdf_ctx();
  c->cfg = *cfg;
  c->cos = Cosmo{cfg->h, cfg->omega_m, cfg->omega_r, cfg->omega_l};
  c->stream = (hipStream_t)stream;
  c->lay = plan(*cfg);
  const int n = cfg->n_steps;
  const double lai = std::log(1.0 / (1.0 + cfg->z_begin)), laf = std::log(1.0 / (1.0 + cfg->z_end));
  const double dl = (laf - lai) / n;
  c->a.resize(n + 1);
  c->a_half.resize(n);
  c->kick1.resize(n);
  c->kick2.resize(n);
  c->drift.resize(n);
  for (int k = 0; k <= n; ++k) c->a[k] = std::exp(lai + dl * k);
  double max_drift = 0;
  for (int k = 0; k < n; ++k) {
    const double l0 = lai + dl * k, lh = lai + dl * (k + 0.5), l1 = lai + dl * (k + 1);
    c->a_half[k] = std::exp(lh);
    c->kick1[k] = dtau(c->cos, l0, lh);
    c->kick2[k] = dtau(c->cos, lh, l1);
    c->drift[k] = dtau(c->cos, l0, l1);
    max_drift = std::max(max_drift, std::fabs(c->drift[k]));
  }
  if (!(max_drift < 0.5 * cfg->box_mpc)) {   // fixed-point drift must stay below half a box
    delete c;
    return FDF_ERR_ARG;
  }
  c->amp = power_amplitude(cfg->sigma8, cfg->ns, cfg->gamma, cfg->h);
  c->sort_every = cfg->sort_every;
  if (cfg->potential_model == FDF_MODEL_RADMAT && cfg->superstep_tol > 0) {
    // Super-steps (sec. 2.1): a new anchor where phi or psi changed by more
    // than the tolerance since the last one (the model's transfer functions
    // are k-independent multiples of g(a), so the ratio test uses g alone).
    double g0, dg0, g, dg;
    radmat_factor(c->a[0], cfg->omega_m, cfg->omega_r, &g0, &dg0);
    c->anchors.push_back(0);
    for (int k = 1; k <= n; ++k) {
      radmat_factor(c->a[k], cfg->omega_m, cfg->omega_r, &g, &dg);
      if (std::fabs(g / g0 - 1.0) > cfg->superstep_tol) {
        c->anchors.push_back(k);
        g0 = g;
      }
    }
    if (c->anchors.back() != n) c->anchors.push_back(n);
  }
  c->tau_begin = conformal_time(c->cos, c->a[0]);
  *out = c;
  return FDF_OK;
}

int fdf_attach_workspace(fdf_ctx* c, void* dptr, size_t bytes) {
  if (!c) return FDF_ERR_ARG;
  if (!dptr || ((uintptr_t)dptr % kAlign) != 0) return fail(c, FDF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < c->lay.total) return fail(c, FDF_ERR_WORKSPACE, "workspace too small");
  c->ws = (char*)dptr;
  c->ws_bytes = bytes;
  fill_twiddles(c);
  char* st = nullptr;
  const int rc = static_scratch(c, &st);   // set-up of the no-allocation entry point's scratch
  if (rc) return rc;
  return fdf_reset(c);
}

int fdf_reset(fdf_ctx* c) {
  if (!c) return FDF_ERR_ARG;
  c->fields.clear();
  c->species.clear();
  c->field_next = 0;
  c->part_next = 0;
  c->step_index = 0;
  c->stepped = false;
  c->seg_dirty = true;
  c->have_density = false;
  c->sorted_once = false;
  return FDF_OK;
}

int fdf_destroy(fdf_ctx* c) {
  if (!c) return FDF_ERR_ARG;
  (void)hipStreamSynchronize(c->stream);
  clear_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& t : c->tim) {
    for (auto& e : t.pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : t.pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }
  delete c;
  return FDF_OK;
}

int fdf_add_field(fdf_ctx* c, uint64_t seed, int32_t fixed_amp, int32_t* field_id) {
  if (!c || !field_id) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  int rc = add_field_slot(c, field_id);
  if (rc) return rc;
  FieldRec& f = c->fields.back();
  f.seed = seed;
  FieldGenArgs g{};
  g.G = c->cfg.grid_n;
  g.fp64 = c->cfg.precision == FDF_PREC_FP64;
  g.fixed_amp = fixed_amp;
  g.seed = seed;
  g.box = c->cfg.box_mpc;
  g.amp = c->amp;
  g.ns = c->cfg.ns;
  g.gamma = c->cfg.gamma;
  g.h = c->cfg.h;
  g.out = f.dk;
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_INIT, &ev);
  launch_field_gen(g, c->stream);
  timing_end(c, FDF_KERNEL_INIT, ev);
  return launched(c, "field generation");
}

int fdf_set_field(fdf_ctx* c, const double* h, int32_t* field_id) {
  if (!c || !h || !field_id) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  int rc = add_field_slot(c, field_id);
  if (rc) return rc;
  const int G = c->cfg.grid_n, M = G / 2, H = G / 2 + 1;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  std::vector<double> d((size_t)G * G * M * 2);
  std::vector<float> f(f64 ? 0 : d.size());
  for (int ix = 0; ix < G; ++ix)
    for (int iy = 0; iy < G; ++iy)
      for (int iz = 0; iz < M; ++iz) {
        const size_t src = (((size_t)ix * G + iy) * H + iz) * 2, dst = (((size_t)ix * G + iy) * M + iz) * 2;
        const bool nyq = ix == M || iy == M;
        d[dst] = nyq ? 0.0 : h[src];
        d[dst + 1] = nyq ? 0.0 : h[src + 1];
      }
  if (!f64) for (size_t i = 0; i < d.size(); ++i) f[i] = (float)d[i];
  rc = hip_check(c, hipMemcpyAsync(c->fields.back().dk, f64 ? (void*)d.data() : (void*)f.data(),
                                   d.size() * (f64 ? 8 : 4), hipMemcpyHostToDevice, c->stream), "field upload");
  if (rc) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "field upload");
}

int fdf_init_species(fdf_ctx* c, int32_t field_id, double m, int64_t n, uint64_t seed, int32_t flags,
                     int32_t* species_id) {
  if (!c || !species_id) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  if (flags & ~FDF_SPECIES_PRE_IC) return fail(c, FDF_ERR_ARG, "unknown species flag");
  int rc = new_species(c, field_id, m, n, seed, flags, species_id);
  if (rc) return rc;
  SpeciesRec& s = c->species.back();
  SampleArgs sa{};
  sa.seg = s.seg[0];
  sa.fp64 = c->cfg.precision == FDF_PREC_FP64;
  sa.seed = seed;
  sa.box = c->cfg.box_mpc;
  sa.t_nu = t_nu_ev();
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_INIT, &ev);
  launch_sample_species(sa, c->stream);
  if (flags & FDF_SPECIES_PRE_IC) {
    c->have_density = false;
    GridBuildArgs g = grid_recipe(c, c->fields[field_id], c->a[0], true);
    launch_build_grids(g, c->stream);
    PreIcArgs p{};
    p.seg = s.seg[0];
    p.fp64 = sa.fp64;
    p.G = c->cfg.grid_n;
    p.box = c->cfg.box_mpc;
    p.m = m;
    p.a = c->a[0];
    p.tau = c->tau_begin;
    p.grid = g.out;
    launch_pre_ic(p, c->stream);
  }
  timing_end(c, FDF_KERNEL_INIT, ev);
  s.pristine = !(flags & FDF_SPECIES_PRE_IC);
  return launched(c, "species sampling");
}

int fdf_set_species_state(fdf_ctx* c, int32_t field_id, double m, int64_t n, const uint32_t* xu,
                          const float* q, int32_t* species_id) {
  if (!c || !xu || !q || !species_id) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  int rc = new_species(c, field_id, m, n, 0, 0, species_id);
  if (rc) return rc;
  Segment& s = c->species.back().seg[0];
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  std::vector<uint32_t> ids(n);
  for (int64_t i = 0; i < n; ++i) ids[i] = (uint32_t)i;
  std::vector<double> dd(f64 ? n : 0);
  std::vector<float> ff(f64 ? 0 : n), zero(f64 ? 0 : n, 0.0f);
  std::vector<uint32_t> uu(f64 ? 0 : n);
  auto put = [&](void* dst, const void* src, size_t bytes) {
    return hip_check(c, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "state upload");
  };
  for (int d = 0; d < 3 && !rc; ++d) {
    if (f64) {
      for (int64_t i = 0; i < n; ++i) dd[i] = (double)xu[3 * i + d] * (c->cfg.box_mpc * 0x1p-32);
      rc = put(s.xd[d], dd.data(), n * 8);
      for (int64_t i = 0; i < n; ++i) dd[i] = (double)q[3 * i + d];
      if (!rc) rc = put(s.qd[d], dd.data(), n * 8);
      if (!rc) rc = put(s.q0d[d], dd.data(), n * 8);
    } else {
      for (int64_t i = 0; i < n; ++i) { uu[i] = xu[3 * i + d]; ff[i] = q[3 * i + d]; }
      rc = put(s.xu[d], uu.data(), n * 4);
      if (!rc) rc = put(s.q0f[d], ff.data(), n * 4);
      if (!rc) rc = put(s.dqf[d], zero.data(), n * 4);
    }
  }
  if (!rc) rc = put(s.id, ids.data(), n * 4);
  return rc;
}

int fdf_build_potential_grids(fdf_ctx* c, int32_t field_id, double a) {
  if (!c) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  if (field_id < 0 || field_id >= (int)c->fields.size()) return fail(c, FDF_ERR_ARG, "bad field id");
  if (!(a > 0) || !std::isfinite(a)) return fail(c, FDF_ERR_ARG, "a must be positive");
  c->fields[field_id].tag[0] = -1;   // buffer 0 no longer holds a super-step anchor
  return build_grid(c, field_id, a);   // graphs are keyed on grid_a, so replays stay consistent
}

}  // extern "C"

namespace {

// Enqueue the launches of n steps (grid rebuilds, re-sorts, pushes) on the
// current launch stream and advance the host-side state.
int enqueue_steps(fdf_ctx* c, int32_t n) {
  const int k0 = c->step_index, nabs = std::abs(n);
  const bool tdep = c->cfg.potential_model == FDF_MODEL_RADMAT;
  int rc = FDF_OK;
  std::vector<int> used(c->fields.size(), 0);
  for (auto& s : c->species) used[s.field] = 1;
  const size_t table = align_up((size_t)c->cfg.max_species * sizeof(Segment));
  const int sort_every = c->sort_every;
  PushArgs pa{};
  pa.nseg = (int)c->species.size();
  pa.total_chunks = total_chunks(c);
  pa.xcd_blocks = xcd_blocks(c);
  pa.fp64 = c->cfg.precision == FDF_PREC_FP64;
  pa.nslot = c->lay.nslot;
  pa.G = c->cfg.grid_n;
  pa.log2g = ilog2(c->cfg.grid_n);
  pa.box = c->cfg.box_mpc;
  pa.ppt = c->ppt;
  pa.persistent = c->persistent;
  pa.do_kick = 1;
  pa.eom = c->cfg.eom;
  pa.tsc = c->cfg.interp_order == 2;
  pa.lds_reserve = push_lds_reserve(c->push_waves);
  // The species the launch at integer time u re-sorts first.  Adaptive
  // cadence: each species once its own typical drift since its last sort
  // reaches sort_cells (all of them at the first sort, and all together when
  // there are too many species for the per-species masks); fixed cadence:
  // every sort_every steps.
  const size_t ns = c->species.size();
  double m_fast = 1e300;
  for (auto& sp : c->species) m_fast = std::min(m_fast, sp.m);
  auto cadence_mass = [&](size_t i) { return per_species_sorting(c) ? c->species[i].m : m_fast; };
  auto sorts_due = [&](int u, std::vector<char>* due) {
    bool any = false;
    for (size_t i = 0; i < ns; ++i) {
      bool d;
      if (c->sort_cells > 0) {
        const double dc = per_species_sorting(c) ? c->species[i].drift_cells : c->species[0].drift_cells;
        d = !c->sorted_once || dc >= c->sort_cells;
      } else {
        d = sort_every > 0 && u % sort_every == 0;
      }
      (*due)[i] = d;
      any = any || d;
    }
    if (any && !per_species_sorting(c)) std::fill(due->begin(), due->end(), 1);
    return any;
  };
  // the interval until the species' next re-sort after one at u0 (as the
  // cadence will decide it): half its conformal time and the scale factor at
  // its middle
  auto sort_prediction = [&](int u0, double m) {
    double span = 0.0, cells = 0.0;
    int steps = 0;
    std::vector<std::pair<double, double>> iv;   // (drift, a) of the steps in the interval
    const bool fwd = n > 0;
    for (int u = u0; ; u += fwd ? 1 : -1) {
      if (fwd ? u >= c->cfg.n_steps : u <= 0) break;
      const double dr = fwd ? c->drift[u] : -c->drift[u - 1];
      const double ah = fwd ? c->a_half[u] : c->a_half[u - 1];
      iv.push_back({dr, ah});
      span += dr;
      cells += typical_drift_cells(c, dr, ah, m);
      ++steps;
      if (c->sort_cells > 0 ? cells >= c->sort_cells : steps >= std::max(sort_every, 1)) break;
    }
    SortPrediction p;
    p.a_mid = c->a[u0];
    double half = 0.0;
    for (const auto& e : iv) {
      if (std::fabs(half + e.first) > 0.5 * std::fabs(span)) { p.a_mid = e.second; break; }
      half += e.first;
      p.a_mid = e.second;
    }
    p.tau = c->sort_predict ? 0.5 * span : 0.0;
    return p;
  };
  std::vector<char> due(ns, 0), due_next(ns, 0);
  std::vector<SortPrediction> pred(ns);
  // the plain push before a re-sort may write the sort keys (one species)
  const bool key_fusable = c->sort_keys_push && c->sort_fused && !pa.fp64 && pa.eom == FDF_EOM_SEPARABLE &&
                           !pa.tsc && c->anchors.empty() && !c->use_graph && ns == 1 && n > 0;
  bool keyed = false;           // this step's re-sort reads keys written by the previous push
  for (int j = 0; j <= nabs; ++j) {
    int t;            // integer time of this launch's kick
    double kclose = 0, kopen = 0, drift = 0, a_drift = 0;   // half-kicks ending / starting at t
    if (n > 0) {
      t = k0 + j;
      if (j > 0) kclose = c->kick2[t - 1];
      if (j < nabs) { kopen = c->kick1[t]; drift = c->drift[t]; a_drift = c->a_half[t]; }
    } else {
      t = k0 - j;
      if (j > 0) kclose = -c->kick1[t];
      if (j < nabs) { kopen = -c->kick2[t - 1]; drift = -c->drift[t - 1]; a_drift = c->a_half[t - 1]; }
    }
    // the separable force does not depend on q: both halves as one kick
    const double kick = pa.eom == FDF_EOM_SEPARABLE ? kclose + kopen : kclose;
    const double a_kick = c->a[t];
    pa.blend = 0;
    if (!c->anchors.empty()) {
      // super-steps: grids at the anchors around t, interpolated linearly in a
      const auto& an = c->anchors;
      size_t iv = 0;
      while (iv + 2 < an.size() && an[iv + 1] <= t) ++iv;
      const int kA = an[iv], kB = an[iv + 1];
      int fsel_all = -1;
      for (size_t f = 0; f < c->fields.size(); ++f) {
        if (!used[f]) continue;
        FieldRec& fr = c->fields[f];
        int fsel;
        if (fr.tag[0] == kA && fr.tag[1] == kB) fsel = 0;
        else if (fr.tag[1] == kA && fr.tag[0] == kB) fsel = 1;
        else if (fr.tag[0] == kA) { rc = build_grid(c, (int)f, c->a[kB], 1); fr.tag[1] = kB; fsel = 0; }
        else if (fr.tag[1] == kA) { rc = build_grid(c, (int)f, c->a[kB], 0); fr.tag[0] = kB; fsel = 1; }
        else if (fr.tag[0] == kB) { rc = build_grid(c, (int)f, c->a[kA], 1); fr.tag[1] = kA; fsel = 1; }
        else if (fr.tag[1] == kB) { rc = build_grid(c, (int)f, c->a[kA], 0); fr.tag[0] = kA; fsel = 0; }
        else {
          rc = build_grid(c, (int)f, c->a[kA], 0);
          if (!rc) rc = build_grid(c, (int)f, c->a[kB], 1);
          fr.tag[0] = kA;
          fr.tag[1] = kB;
          fsel = 0;
        }
        if (rc) return rc;
        if (fsel_all >= 0 && fsel != fsel_all) return fail(c, FDF_ERR_STATE, "grid sets of fields out of step");
        fsel_all = fsel;
      }
      pa.blend = 1;
      pa.grid_sel = fsel_all < 0 ? 0 : fsel_all;
      pa.blend_t = (a_kick - c->a[kA]) / (c->a[kB] - c->a[kA]);
    } else {
      for (size_t f = 0; f < c->fields.size(); ++f) {
        if (!used[f]) continue;
        if (!c->fields[f].has_grid || (tdep && c->fields[f].grid_a != a_kick)) {
          rc = build_grid(c, (int)f, a_kick);
          if (rc) return rc;
        }
      }
    }
    bool fused_sort = false;    // this step's push also performs the re-sort of the due species
    std::fill(due.begin(), due.end(), 0);
    if (j < nabs) {
      if (sorts_due(t, &due)) {
        for (size_t i = 0; i < ns; ++i)
          if (due[i]) pred[i] = sort_prediction(t, cadence_mass(i));
        // the first sort takes two passes (the second orders cells in buckets)
        const int passes = c->sorted_once ? 1 : 2;
        fused_sort = c->sort_fused && !pa.fp64 && pa.eom == FDF_EOM_SEPARABLE;
        for (int pass = 0; pass < passes - (fused_sort ? 1 : 0) && !rc; ++pass)
          rc = sort_species(c, pred, due, pass == 0);
        if (rc) return rc;
        c->sorted_once = true;
        for (size_t i = 0; i < ns; ++i)
          if (due[i]) c->species[i].drift_cells = 0;
      }
      for (size_t i = 0; i < ns; ++i)
        c->species[i].drift_cells += typical_drift_cells(c, drift, a_drift, cadence_mass(i));
    }
    // each species' state sits in its own copy: table 0 or 1 per species
    pa.seg = (const Segment*)(c->ws + c->lay.seg);
    pa.seg_alt = (const Segment*)(c->ws + c->lay.seg + table);
    pa.alt_mask = 0;
    pa.skip_mask = 0;
    if (per_species_sorting(c)) {
      for (size_t i = 0; i < ns; ++i) if (c->species[i].cur) pa.alt_mask |= 1ull << i;
    } else {
      pa.seg = (const Segment*)(c->ws + c->lay.seg + c->species[0].cur * table);
    }
    pa.kick = kick;
    pa.kick_open = pa.eom == FDF_EOM_SEPARABLE ? 0.0 : kopen;
    pa.a_kick = a_kick;
    pa.do_drift = j < nabs;
    pa.drift = drift;
    pa.a_drift = a_drift;
    int64_t pushed = 0;           // particles of the plain launch, and the meshes it reads
    std::vector<char> mesh_read(c->fields.size(), 0);
    if (fused_sort) {
      rc = sort_push_species(c, pred, due, pa, table, keyed && due[0]);
      if (rc) return rc;
      for (size_t i = 0; i < ns; ++i) if (due[i]) pa.skip_mask |= 1ull << i;   // pushed already
    }
    keyed = false;
    // write the sort keys in this push when the next launch of this call
    // re-sorts the species and this launch pushes it (the keys are those of
    // the state the rank pass would read)
    pa.key_out = nullptr;
    if (key_fusable && c->sorted_once && j + 1 < nabs && !(fused_sort && due[0]) &&
        sorts_due(t + 1, &due_next) && due_next[0]) {
      const SortPrediction pn = sort_prediction(t + 1, cadence_mass(0));
      const SortArgs sa = sort_args(c, c->species[0], pn.tau, pn.a_mid);
      pa.key_out = sa.rank;
      pa.key_fine_bits = sa.fine_bits;
      pa.key_tau = pn.tau;
      pa.key_ma = sa.ma;
      keyed = true;
    }
    for (size_t i = 0; i < ns; ++i) {
      if (fused_sort && due[i]) continue;
      pushed += c->species[i].n;
      mesh_read[c->species[i].field] = 1;
    }
    if (pushed > 0) {
      std::pair<hipEvent_t, hipEvent_t> ev;
      timing_begin(c, FDF_KERNEL_PUSH, &ev);
      launch_push(pa, stream_of(c));
      timing_end(c, FDF_KERNEL_PUSH, ev);
      int64_t meshes = 0;
      for (char r : mesh_read) meshes += r;
      timing_work(c, FDF_KERNEL_PUSH, pa.do_drift ? pushed : 0, pa.do_drift ? 0 : pushed,
                  meshes * (int64_t)c->cfg.grid_n * c->cfg.grid_n * c->cfg.grid_n * (pa.blend ? 2 : 1));
      rc = launched(c, "push");
      if (rc) return rc;
    }
    pa.key_out = nullptr;
    for (auto& s : c->species) s.pristine = false;
  }
  c->step_index = k0 + n;
  c->stepped = true;
  return FDF_OK;
}

// The workspace is carved deterministically, so fields and species added in
// the same order with the same sizes sit at the same device addresses: a graph
// captured for one such layout replays correctly after fdf_reset + re-adding.
std::vector<double> layout_signature(fdf_ctx* c) {
  std::vector<double> v;
  v.push_back((double)c->fields.size());
  for (auto& s : c->species) {
    v.push_back(s.field);
    v.push_back(s.m);
    v.push_back((double)s.n);
    v.push_back((double)s.flags);
  }
  return v;
}

HostStepState host_state(fdf_ctx* c) {
  HostStepState h;
  h.step_index = c->step_index;
  h.sorted_once = c->sorted_once;
  for (auto& s : c->species) {
    h.cur.push_back(s.cur);
    h.drift_cells.push_back(s.drift_cells);
    h.pristine.push_back(s.pristine ? 1 : 0);
  }
  for (auto& f : c->fields) {
    h.grid_a.push_back(f.has_grid ? f.grid_a : NAN);
    h.tags.push_back(f.tag[0]);
    h.tags.push_back(f.tag[1]);
  }
  return h;
}

void apply_state(fdf_ctx* c, const HostStepState& h) {
  c->step_index = h.step_index;
  c->sorted_once = h.sorted_once;
  for (size_t i = 0; i < c->species.size() && i < h.cur.size(); ++i) {
    c->species[i].cur = h.cur[i];
    c->species[i].drift_cells = h.drift_cells[i];
    c->species[i].pristine = h.pristine[i];
  }
  for (size_t i = 0; i < c->fields.size() && i < h.grid_a.size(); ++i) {
    c->fields[i].has_grid = !std::isnan(h.grid_a[i]);
    c->fields[i].grid_a = h.grid_a[i];
    c->fields[i].tag[0] = h.tags[2 * i];
    c->fields[i].tag[1] = h.tags[2 * i + 1];
  }
  c->stepped = true;
}

// Graph mode: the launches of step(n) from a given host state are captured
// once (on a private stream) and replayed on the context stream afterwards.
int step_graph(fdf_ctx* c, int32_t n) {
  const HostStepState before = host_state(c);
  const std::vector<double> layout = layout_signature(c);
  for (auto& g : c->graphs) {
    if (g.n == n && g.before == before && g.layout == layout) {
      int rc = hip_check(c, hipGraphLaunch(g.exec, c->stream), "graph launch");
      if (!rc) apply_state(c, g.after);
      return rc;
    }
  }
  if (!c->cap_stream) {
    int rc = hip_check(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
    if (rc) return rc;
  }
  if (c->graphs.size() >= 16) clear_graphs(c);   // bounded cache
  GraphRec g;
  g.n = n;
  g.before = before;
  g.layout = layout;
  int rc = hip_check(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc) return rc;
  c->launch_stream = c->cap_stream;
  const int rc_enq = enqueue_steps(c, n);
  c->launch_stream = nullptr;
  rc = hip_check(c, hipStreamEndCapture(c->cap_stream, &g.graph), "end capture");
  if (rc_enq || rc) {
    if (g.graph) (void)hipGraphDestroy(g.graph);
    apply_state(c, before);
    return rc_enq ? rc_enq : rc;
  }
  rc = hip_check(c, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "graph instantiate");
  if (rc) {
    (void)hipGraphDestroy(g.graph);
    apply_state(c, before);
    return rc;
  }
  g.after = host_state(c);
  rc = hip_check(c, hipGraphLaunch(g.exec, c->stream), "graph launch");
  c->graphs.push_back(g);
  return rc;
}

}  // namespace

extern "C" {

int fdf_step(fdf_ctx* c, int32_t n) {
  if (!c) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  if (c->species.empty()) return fail(c, FDF_ERR_STATE, "no species");
  if (n == 0) return FDF_OK;
  const int k0 = c->step_index;
  if (k0 + n < 0 || k0 + n > c->cfg.n_steps) return fail(c, FDF_ERR_ARG, "step range outside the schedule");
  int rc = upload_segments(c);
  if (rc) return rc;
  if (c->use_graph) return step_graph(c, n);
  return enqueue_steps(c, n);
}

int fdf_force_terms(fdf_ctx* c, int32_t sid, double* h_rms) {
  if (!c || !h_rms) return FDF_ERR_ARG;
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  if (sid < 0 || sid >= (int)c->species.size()) return fail(c, FDF_ERR_ARG, "bad species id");
  const int s_gpsi = grid_slot(c->cfg, 0), s_gphi = grid_slot(c->cfg, 3), s_dot = grid_slot(c->cfg, 6);
  if (s_gpsi < 0 || s_gphi < 0 || s_dot == -2)
    return fail(c, FDF_ERR_UNSUPPORTED, "grad psi, grad phi and phi-dot are not all stored for this equation of motion");
  SpeciesRec& sp = c->species[sid];
  FieldRec& f = c->fields[sp.field];
  const double a = c->a[c->step_index];
  const bool tdep = c->cfg.potential_model == FDF_MODEL_RADMAT;
  if (!f.has_grid || (tdep && f.grid_a != a) || !c->anchors.empty()) {
    f.tag[0] = -1;   // buffer 0 no longer holds a super-step anchor
    const int rc = build_grid(c, sp.field, a);
    if (rc) return rc;
  }
  TermArgs t{};
  t.seg = sp.seg[sp.cur];
  t.fp64 = c->cfg.precision == FDF_PREC_FP64;
  t.G = c->cfg.grid_n;
  t.nslot = c->lay.nslot;
  t.slot_gpsi = s_gpsi;
  t.slot_gphi = s_gphi;
  t.slot_phidot = s_dot;
  t.box = c->cfg.box_mpc;
  t.ma = sp.m * a;
  t.grid = f.grid;
  t.out = (double*)(c->ws + c->lay.bins);
  launch_fill_zero(t.out, align_up(3 * kMaxBins * sizeof(double)), c->stream);
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_OUTPUT, &ev);
  launch_force_terms(t, c->stream);
  timing_end(c, FDF_KERNEL_OUTPUT, ev);
  int rc = launched(c, "force terms");
  double sums[4];
  if (!rc) rc = hip_check(c, hipMemcpyAsync(sums, t.out, sizeof(sums), hipMemcpyDeviceToHost, c->stream), "terms");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "terms");
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) h_rms[k] = sp.n ? std::sqrt(sums[k] / (double)sp.n) : 0.0;
  return FDF_OK;
}

int fdf_weights(fdf_ctx* c, int32_t sid, double* d_w) {
  if (!c || !d_w) return FDF_ERR_ARG;
  if (sid < 0 || sid >= (int)c->species.size()) return fail(c, FDF_ERR_ARG, "bad species id");
  OutputArgs o = output_args(c, c->species[sid]);
  o.w_out = d_w;
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_OUTPUT, &ev);
  launch_weights(o, c->stream);
  timing_end(c, FDF_KERNEL_OUTPUT, ev);
  return launched(c, "weights");
}

// Device buffers of one spectrum: the deposit halves (8 bytes per cell),
// the fixed-point deposit's largest |value|, the FFT planes (halves and the
// momentum spectrum's two accumulators), the FP32 form's binary32 halves and
// the bin accumulators.
struct PkBuffers {
  char* dens;
  uint32_t* max_bits;
  void* scratch;
  float* real32;
  double* bins;
};

// Arguments shared by both spectrum entry points; *G receives the mesh.
static int pk_validate(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                       int32_t analysis_n, int* G) {
  if (!needs_ws(c)) return fail(c, FDF_ERR_WORKSPACE, "no workspace attached");
  if (nbins < 1 || nbins > kMaxBins) return fail(c, FDF_ERR_ARG, "n_bins must be in [1, 256]");
  if (mode != FDF_PK_CROSS && mode != FDF_PK_AUTO) return fail(c, FDF_ERR_ARG, "unknown mode");
  for (int i = 0; i < ns; ++i) {
    if (sp[i] < 0 || sp[i] >= (int)c->species.size()) return fail(c, FDF_ERR_ARG, "bad species id");
    // a total contrast only means something for species that see one field
    if (c->species[sp[i]].field != c->species[sp[0]].field)
      return fail(c, FDF_ERR_ARG, "the species of one spectrum must share a field");
    for (int j = 0; j < i; ++j)
      if (sp[j] == sp[i]) return fail(c, FDF_ERR_ARG, "a species is listed twice");
  }
  const int Gm = c->cfg.grid_n;
  if (analysis_n != 0 && (!is_pow2(analysis_n) || analysis_n < 8 || analysis_n > Gm))
    return fail(c, FDF_ERR_ARG, "analysis_n must be 0 or a power of two in [8, grid_n]");
  *G = analysis_n ? analysis_n : Gm;
  return FDF_OK;
}

// Binned spectrum of the energy-density contrast, or (momentum) of
// Theta = sum_a i k_a J_a with J the deposit of w q: the three axes are
// deposited and transformed one after the other and summed in Fourier space.
// Enqueues the work on the context stream; the bins end in b.bins as
// [count][sum |k|][sum P] per bin, from exact (order-independent) sums.
static void pk_enqueue(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                       bool momentum, int G, const PkBuffers& b) {
  const int Gm = c->cfg.grid_n;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  const size_t cells = (size_t)G * G * G;
  const double a = c->a[c->step_index];
  double esum = 0;
  for (int i = 0; i < ns; ++i) esum += mean_energy(c->species[sp[i]].m, a);
  // FP32 form: fixed-point halves in dens (int64 per cell), converted to
  // binary32 meshes for the transform
  int64_t n_all = 0;
  for (int i = 0; i < ns; ++i) n_all += c->species[sp[i]].n;
  int fixed_bits = 62;
  while (fixed_bits > 20 && ((int64_t)1 << (62 - fixed_bits)) < n_all) --fixed_bits;
  launch_fill_zero(b.bins, align_up(kBinsBytes), c->stream);
  PkArgs pk{};
  pk.G = G;
  pk.fp64 = f64;
  pk.nbins = nbins;
  pk.auto_mode = mode == FDF_PK_AUTO;
  pk.volume = c->cfg.box_mpc * c->cfg.box_mpc * c->cfg.box_mpc;
  pk.grid_a = f64 ? (void*)b.dens : (void*)b.real32;
  pk.grid_b = f64 ? (void*)(b.dens + cells * 8) : (void*)(b.real32 + cells);
  pk.scratch = b.scratch;
  pk.twiddle = c->ws + (f64 ? c->lay.twiddle_d + twiddle_entry(Gm, G) * 16
                            : c->lay.twiddle_f + twiddle_entry(Gm, G) * 8);
  pk.bins = b.bins;
  pk.acc = (unsigned long long*)(b.bins + 3 * kMaxBins);
  pk.max_bits = (uint32_t*)(b.bins + 8 * kMaxBins);
  pk.bin_plane = momentum ? 2 : 0;
  pk.kf = 2.0 * kPi / c->cfg.box_mpc;
  pk.deriv_axis = -1;
  for (int axis = momentum ? 0 : -1; axis < (momentum ? 3 : 0); ++axis) {
    launch_fill_zero(b.dens, align_up(2 * cells * 8), c->stream);
    if (!f64) launch_fill_zero(b.max_bits, kAlign, c->stream);
    for (int pass = f64 ? 1 : 0; pass < 2; ++pass)
    for (int i = 0; i < ns; ++i) {
      const SpeciesRec& s = c->species[sp[i]];
      OutputArgs o = output_args(c, s);
      o.auto_mode = mode == FDF_PK_AUTO;
      const double g3 = (double)cells;
      if (o.auto_mode) {
        o.norm[0] = o.norm[1] = g3 / ((double)s.n * esum);
      } else {
        const int64_t ne = (s.n + 1) / 2, no = s.n / 2;
        o.norm[0] = g3 / ((double)ne * esum);
        o.norm[1] = no ? g3 / ((double)no * esum) : 0.0;
      }
      o.G = G;
      o.dens[0] = b.dens;
      o.dens[1] = b.dens + cells * 8;
      o.quantity = axis;
      o.max_bits = b.max_bits;
      o.fixed_bits = fixed_bits;
      if (pass == 0) launch_deposit_max(o, c->stream);
      else launch_deposit(o, c->stream);
    }
    if (!f64) {
      FixedToRealArgs fr{};
      fr.src[0] = (const long long*)b.dens;
      fr.src[1] = (const long long*)(b.dens + cells * 8);
      fr.dst[0] = b.real32;
      fr.dst[1] = b.real32 + cells;
      fr.n_half = cells;
      fr.G = G;
      fr.n = (mode == FDF_PK_AUTO ? 1 : 2) * cells;
      fr.max_bits = b.max_bits;
      fr.fixed_bits = fixed_bits;
      launch_fixed_to_real(fr, c->stream);
    }
    pk.deriv_axis = axis;
    pk.accum_first = axis == 0;
    launch_power_spectrum(pk, c->stream);
  }
  launch_bin(pk, c->stream);
}

static int power_spectrum(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                          bool momentum, int32_t analysis_n, double* hk, double* hp, double* hn) {
  if (!c || !sp || ns < 1 || !hk || !hp || !hn) return FDF_ERR_ARG;
  int G = 0;
  int rc = pk_validate(c, sp, ns, nbins, mode, analysis_n, &G);
  if (rc) return rc;
  PkBuffers b{};
  b.dens = c->ws + c->lay.dens;
  b.max_bits = (uint32_t*)(c->ws + c->lay.dep);
  b.scratch = c->ws + c->lay.scratch;
  b.real32 = (float*)(c->ws + c->lay.scratch + density_copy_offset(c));
  b.bins = (double*)(c->ws + c->lay.bins);
  std::pair<hipEvent_t, hipEvent_t> ev;
  timing_begin(c, FDF_KERNEL_OUTPUT, &ev);
  pk_enqueue(c, sp, ns, nbins, mode, momentum, G, b);
  timing_end(c, FDF_KERNEL_OUTPUT, ev);
  rc = launched(c, "power spectrum");
  if (rc) return rc;
  std::vector<double> hb(3 * nbins);
  rc = hip_check(c, hipMemcpyAsync(hb.data(), b.bins, hb.size() * 8, hipMemcpyDeviceToHost, c->stream), "bins");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "bins");
  if (rc) return rc;
  for (int i = 0; i < nbins; ++i) {
    const double cnt = hb[i];
    hn[i] = cnt;
    hk[i] = cnt > 0 ? hb[nbins + i] / cnt : NAN;
    hp[i] = cnt > 0 ? hb[2 * nbins + i] / cnt : NAN;
  }
  c->have_density = !momentum && G == c->cfg.grid_n;   // else the buffers hold another quantity or mesh
  c->density_auto = mode == FDF_PK_AUTO;
  return FDF_OK;
}

int fdf_density_power_spectrum(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                               double* hk, double* hp, double* hn) {
  return power_spectrum(c, sp, ns, nbins, mode, false, 0, hk, hp, hn);
}

int fdf_momentum_power_spectrum(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                                double* hk, double* hp, double* hn) {
  return power_spectrum(c, sp, ns, nbins, mode, true, 0, hk, hp, hn);
}

int fdf_power_spectrum(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                       int32_t quantity, int32_t analysis_n, double* hk, double* hp, double* hn) {
  if (quantity != FDF_PK_DENSITY && quantity != FDF_PK_MOMENTUM)
    return c ? fail(c, FDF_ERR_ARG, "unknown quantity") : FDF_ERR_ARG;
  return power_spectrum(c, sp, ns, nbins, mode, quantity == FDF_PK_MOMENTUM, analysis_n, hk, hp, hn);
}

int fdf_power_spectrum_noalloc(fdf_ctx* c, const int32_t* sp, int32_t ns, int32_t nbins, int32_t mode,
                               int32_t quantity, int32_t analysis_n, double* d_out) {
  if (!c || !sp || ns < 1 || !d_out) return FDF_ERR_ARG;
  if (quantity != FDF_PK_DENSITY && quantity != FDF_PK_MOMENTUM) return fail(c, FDF_ERR_ARG, "unknown quantity");
  int G = 0;
  int rc = pk_validate(c, sp, ns, nbins, mode, analysis_n, &G);
  if (rc) return rc;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  if (G > kStaticMaxMesh || static_scratch_bytes(f64, G) > kStaticScratchBytes)
    return fail(c, FDF_ERR_ARG, "the no-allocation spectrum needs an analysis mesh of at most 64^3 "
                                "(analysis_n in [8, 64]): its static scratch holds 16 MiB");
  char* st = nullptr;
  rc = static_scratch(c, &st);
  if (rc) return rc;
  const size_t g3 = (size_t)G * G * G, plane = (size_t)G * G * (G / 2) * (f64 ? 16 : 8);
  PkBuffers b{};
  size_t off = 0;
  b.bins = (double*)(st + off); off += align_up(kBinsBytes);
  b.max_bits = (uint32_t*)(st + off); off += kAlign;
  b.dens = st + off; off += align_up(2 * g3 * 8);
  b.scratch = st + off; off += align_up(4 * plane);
  b.real32 = f64 ? nullptr : (float*)(st + off);
  pk_enqueue(c, sp, ns, nbins, mode, quantity == FDF_PK_MOMENTUM, G, b);
  launch_bins_finalize(b.bins, nbins, d_out, c->stream);
  return launched(c, "power spectrum (static scratch)");
}

int fdf_read_state(fdf_ctx* c, int32_t sid, double* hx, double* hq) {
  if (!c) return FDF_ERR_ARG;
  if (sid < 0 || sid >= (int)c->species.size()) return fail(c, FDF_ERR_ARG, "bad species id");
  const SpeciesRec& s = c->species[sid];
  const Segment& g = s.seg[s.cur];
  const int64_t n = s.n;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (rc) return rc;
  std::vector<uint32_t> id(n);
  rc = hip_check(c, hipMemcpy(id.data(), g.id, n * 4, hipMemcpyDeviceToHost), "read ids");
  if (rc) return rc;
  std::vector<double> bd(f64 ? n : 0);
  std::vector<float> bf(f64 ? 0 : n), bc(f64 ? 0 : n);
  std::vector<uint32_t> bu(f64 ? 0 : n);
  for (int d = 0; d < 3; ++d) {
    if (hx) {
      if (f64) {
        rc = hip_check(c, hipMemcpy(bd.data(), g.xd[d], n * 8, hipMemcpyDeviceToHost), "read x");
        for (int64_t i = 0; i < n && !rc; ++i) hx[3 * (size_t)id[i] + d] = bd[i];
      } else {
        rc = hip_check(c, hipMemcpy(bu.data(), g.xu[d], n * 4, hipMemcpyDeviceToHost), "read x");
        for (int64_t i = 0; i < n && !rc; ++i) hx[3 * (size_t)id[i] + d] = (double)bu[i] * (c->cfg.box_mpc * 0x1p-32);
      }
    }
    if (rc) return rc;
    if (hq) {
      if (f64) {
        rc = hip_check(c, hipMemcpy(bd.data(), g.qd[d], n * 8, hipMemcpyDeviceToHost), "read q");
        for (int64_t i = 0; i < n && !rc; ++i) hq[3 * (size_t)id[i] + d] = bd[i];
      } else {
        rc = hip_check(c, hipMemcpy(bf.data(), g.q0f[d], n * 4, hipMemcpyDeviceToHost), "read q0");
        if (!rc) rc = hip_check(c, hipMemcpy(bc.data(), g.dqf[d], n * 4, hipMemcpyDeviceToHost), "read dq");
        for (int64_t i = 0; i < n && !rc; ++i) hq[3 * (size_t)id[i] + d] = (double)bf[i] + (double)bc[i];
      }
    }
    if (rc) return rc;
  }
  return FDF_OK;
}

int fdf_read_grid(fdf_ctx* c, int32_t field_id, int32_t slot, double* h) {
  if (!c || !h) return FDF_ERR_ARG;
  if (field_id < 0 || field_id >= (int)c->fields.size()) return fail(c, FDF_ERR_ARG, "bad field id");
  if (slot < 0 || slot > 9) return fail(c, FDF_ERR_ARG, "quantity must be in [0, 9]");
  const FieldRec& f = c->fields[field_id];
  if (!f.has_grid) return fail(c, FDF_ERR_STATE, "grid not built");
  const int ns = c->lay.nslot;
  const int s = grid_slot(c->cfg, slot);
  if (s == -2) return fail(c, FDF_ERR_UNSUPPORTED, "quantity not stored for this equation of motion");
  if (s == -1) {
    std::fill(h, h + (size_t)c->cfg.grid_n * c->cfg.grid_n * c->cfg.grid_n, 0.0);
    return FDF_OK;
  }
  const size_t cells = (size_t)c->cfg.grid_n * c->cfg.grid_n * c->cfg.grid_n;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (rc) return rc;
  // the device mesh is bricked (mesh_x/y/z); the host array is x-major
  const uint32_t G = (uint32_t)c->cfg.grid_n;
  std::vector<size_t> where(cells);
  for (uint32_t ix = 0; ix < G; ++ix)
    for (uint32_t iy = 0; iy < G; ++iy)
      for (uint32_t iz = 0; iz < G; ++iz)
        where[((size_t)ix * G + iy) * G + iz] = (size_t)mesh_x(ix, G) + mesh_y(iy, G) + mesh_z(iz);
  if (f64) {
    std::vector<double> all(cells * ns);
    rc = hip_check(c, hipMemcpy(all.data(), f.grid, all.size() * 8, hipMemcpyDeviceToHost), "read grid");
    for (size_t i = 0; i < cells && !rc; ++i) h[i] = all[where[i] * ns + s];
  } else {
    std::vector<uint16_t> all(cells * ns);
    rc = hip_check(c, hipMemcpy(all.data(), f.grid, all.size() * 2, hipMemcpyDeviceToHost), "read grid");
    for (size_t i = 0; i < cells && !rc; ++i) {
      uint32_t u = (uint32_t)all[where[i] * ns + s] << 16;
      float v;
      std::memcpy(&v, &u, 4);
      h[i] = v;
    }
  }
  return rc;
}

int fdf_read_field(fdf_ctx* c, int32_t field_id, double* h) {
  if (!c || !h) return FDF_ERR_ARG;
  if (field_id < 0 || field_id >= (int)c->fields.size()) return fail(c, FDF_ERR_ARG, "bad field id");
  const int G = c->cfg.grid_n, M = G / 2, H = M + 1;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  const size_t n = (size_t)G * G * M * 2;
  std::vector<double> d(n);
  std::vector<float> f(f64 ? 0 : n);
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (!rc) rc = hip_check(c, hipMemcpy(f64 ? (void*)d.data() : (void*)f.data(), c->fields[field_id].dk,
                                       n * (f64 ? 8 : 4), hipMemcpyDeviceToHost), "read field");
  if (rc) return rc;
  if (!f64) for (size_t i = 0; i < n; ++i) d[i] = f[i];
  for (int ix = 0; ix < G; ++ix)
    for (int iy = 0; iy < G; ++iy)
      for (int iz = 0; iz < H; ++iz) {
        const size_t dst = (((size_t)ix * G + iy) * H + iz) * 2;
        if (iz == M) { h[dst] = 0; h[dst + 1] = 0; continue; }
        const size_t src = (((size_t)ix * G + iy) * M + iz) * 2;
        h[dst] = d[src];
        h[dst + 1] = d[src + 1];
      }
  return FDF_OK;
}

int fdf_read_density(fdf_ctx* c, int32_t half, double* h) {
  if (!c || !h) return FDF_ERR_ARG;
  if (!c->have_density) return fail(c, FDF_ERR_STATE, "no density deposited yet");
  if (half < 0 || half > 1) return fail(c, FDF_ERR_ARG, "half must be 0 or 1");
  const size_t cells = (size_t)c->cfg.grid_n * c->cfg.grid_n * c->cfg.grid_n;
  const bool f64 = c->cfg.precision == FDF_PREC_FP64;
  const char* src = f64 ? c->ws + c->lay.dens + half * cells * 8
                        : c->ws + c->lay.scratch + density_copy_offset(c) + half * cells * 4;
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (rc) return rc;
  if (f64) return hip_check(c, hipMemcpy(h, src, cells * 8, hipMemcpyDeviceToHost), "read density");
  std::vector<float> f(cells);
  rc = hip_check(c, hipMemcpy(f.data(), src, cells * 4, hipMemcpyDeviceToHost), "read density");
  for (size_t i = 0; i < cells && !rc; ++i) h[i] = f[i];
  return rc;
}

int fdf_read_schedule(const fdf_ctx* c, double* h) {
  if (!c || !h) return FDF_ERR_ARG;
  const int n = c->cfg.n_steps;
  std::copy(c->a.begin(), c->a.end(), h);
  std::copy(c->a_half.begin(), c->a_half.end(), h + n + 1);
  std::copy(c->kick1.begin(), c->kick1.end(), h + 2 * n + 1);
  std::copy(c->kick2.begin(), c->kick2.end(), h + 3 * n + 1);
  std::copy(c->drift.begin(), c->drift.end(), h + 4 * n + 1);
  return FDF_OK;
}

int fdf_get_info(const fdf_ctx* c, fdf_info* info) {
  if (!c || !info) return FDF_ERR_ARG;
  std::memset(info, 0, sizeof(*info));
  info->step_index = c->step_index;
  info->n_steps = c->cfg.n_steps;
  info->a_current = c->a[c->step_index];
  info->amplitude = c->amp;
  info->tau_begin = c->tau_begin;
  info->n_fields = (int32_t)c->fields.size();
  info->n_species = (int32_t)c->species.size();
  for (auto& s : c->species) info->n_particles += s.n;
  info->workspace_used = c->lay.total;
  return FDF_OK;
}

int fdf_get_tuning(const fdf_ctx* c, fdf_tuning* t) {
  if (!c || !t) return FDF_ERR_ARG;
  std::memset(t, 0, sizeof(*t));
  t->particles_per_thread = c->ppt;
  t->sort_tiles = c->sort_tiles;
  t->sort_every = c->sort_every;
  t->sort_cells = c->sort_cells;
  t->persistent_blocks = c->persistent;
  t->use_graph = c->use_graph ? 1 : 0;
  t->sort_predict = c->sort_predict ? 1 : 0;
  t->sort_fused = c->sort_fused ? 1 : 0;
  t->push_waves = c->push_waves;
  t->sort_push_ppt = c->sort_push_ppt;
  t->sort_keys_push = c->sort_keys_push ? 1 : 0;
  return FDF_OK;
}

int fdf_set_tuning(fdf_ctx* c, const fdf_tuning* t) {
  if (!c || !t) return FDF_ERR_ARG;
  const int p = t->particles_per_thread;
  if (p != 1 && p != 2 && p != 4 && p != 8) return fail(c, FDF_ERR_ARG, "particles_per_thread must be 1, 2, 4 or 8");
  const int tmax = std::min(c->cfg.grid_n, 256);
  if (t->sort_tiles != 0 && (!is_pow2(t->sort_tiles) || t->sort_tiles > tmax))
    return fail(c, FDF_ERR_ARG, "sort_tiles must be 0 or a power of two <= min(G, 256)");
  if (t->sort_every < 0 || (t->sort_every > 0 && c->cfg.sort_every == 0))
    return fail(c, FDF_ERR_ARG, "sorting needs a context created with sort_every > 0");
  if (!(t->sort_cells >= 0) || (t->sort_cells > 0 && c->cfg.sort_every == 0))
    return fail(c, FDF_ERR_ARG, "sort_cells must be >= 0 (and > 0 needs sort_every > 0 at create)");
  if (t->persistent_blocks < 0 || t->persistent_blocks % 8 != 0 || t->persistent_blocks > (1 << 20))
    return fail(c, FDF_ERR_ARG, "persistent_blocks must be 0 or a positive multiple of 8");
  if (t->use_graph != 0 && t->use_graph != 1) return fail(c, FDF_ERR_ARG, "use_graph must be 0 or 1");
  if (t->sort_predict != 0 && t->sort_predict != 1) return fail(c, FDF_ERR_ARG, "sort_predict must be 0 or 1");
  if (t->sort_fused != 0 && t->sort_fused != 1) return fail(c, FDF_ERR_ARG, "sort_fused must be 0 or 1");
  if (t->push_waves != 0 && (t->push_waves < 2 || t->push_waves > 8))
    return fail(c, FDF_ERR_ARG, "push_waves must be 0 or in [2, 8]");
  if (t->sort_push_ppt != 0 && t->sort_push_ppt != 1 && t->sort_push_ppt != 2 && t->sort_push_ppt != 4)
    return fail(c, FDF_ERR_ARG, "sort_push_ppt must be 0, 1, 2 or 4");
  if (t->sort_keys_push != 0 && t->sort_keys_push != 1) return fail(c, FDF_ERR_ARG, "sort_keys_push must be 0 or 1");
  if (p != c->ppt) c->seg_dirty = true;   // chunk boundaries depend on the block size
  clear_graphs(c);
  c->persistent = t->persistent_blocks;
  c->use_graph = t->use_graph != 0;
  c->ppt = p;
  c->sort_tiles = t->sort_tiles;
  c->sort_every = t->sort_every;
  c->sort_cells = t->sort_cells;
  c->sort_predict = t->sort_predict != 0;
  c->sort_fused = t->sort_fused != 0;
  c->push_waves = t->push_waves;
  c->sort_push_ppt = t->sort_push_ppt ? t->sort_push_ppt : 4;
  c->sort_keys_push = t->sort_keys_push != 0;
  return FDF_OK;
}

int fdf_sync(fdf_ctx* c) {
  if (!c) return FDF_ERR_ARG;
  return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

int fdf_timing_enable(fdf_ctx* c, int32_t on) {
  if (!c) return FDF_ERR_ARG;
  c->timing = on != 0;
  return FDF_OK;
}

int fdf_read_timing(fdf_ctx* c, int32_t cls, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return FDF_ERR_ARG;
  if (cls < 0 || cls >= FDF_KERNEL_COUNT) return fail(c, FDF_ERR_ARG, "bad kernel class");
  timing_collect(c);
  *ms = c->tim[cls].total_ms;
  *launches = c->tim[cls].launches;
  return FDF_OK;
}

int fdf_timing_reset(fdf_ctx* c) {
  if (!c) return FDF_ERR_ARG;
  timing_collect(c);
  for (auto& t : c->tim) { t.total_ms = 0; t.launches = 0; t.work[0] = t.work[1] = t.work[2] = 0; }
  return FDF_OK;
}

int fdf_read_work(fdf_ctx* c, int32_t cls, int64_t* work) {
  if (!c || !work) return FDF_ERR_ARG;
  if (cls < 0 || cls >= FDF_KERNEL_COUNT) return fail(c, FDF_ERR_ARG, "bad kernel class");
  for (int k = 0; k < 3; ++k) work[k] = c->tim[cls].work[k];
  return FDF_OK;
}

}  // extern "C"
