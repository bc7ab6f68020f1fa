/*
 * fastdf.h -- C ABI of the MI355X (gfx950) FastDF neutrino push.
 *
 * Method: W. Elbers, "Geodesic motion and phase-space evolution of massive
 * neutrinos" (arXiv:2207.14256).  Neutrino tracers move through linear
 * Newtonian-gauge potentials phi, psi (sec. 2, eq. metric) on a periodic mesh
 * with the separable equations of motion eq. releq_approx / eq.
 * geodesic_approx, integrated by the kick-drift-kick leapfrog of sec. 3.3 with
 * constant Delta log a.  The delta-f weights of sec. 2.2 and the binned
 * energy-density power spectrum of sec. 4 are the outputs.
 *
 * Units: lengths and conformal time in Mpc (c = 1); momenta, energies and
 * masses in eV; the neutrino temperature is 1.95 K (sec. 2).
 *
 * Conventions shared by every call:
 *   - Every function returns an fdf_status: 0 on success, a negative code on
 *     failure.  Nothing throws across the ABI.  fdf_last_error() gives a
 *     human-readable reason for the last failure on a context.
 *   - "device pointer" means memory on the HIP device of the context
 *     (for example a torch tensor's data_ptr()); "host pointer" means
 *     ordinary CPU memory.  The caller owns all memory it passes in.  The
 *     context owns only host tables; all of its device buffers are carved
 *     from the one workspace the caller attaches.
 *   - Calls enqueue work on the context's stream and return.  Calls that
 *     copy to host memory (fdf_read_*, fdf_*_power_spectrum,
 *     fdf_read_timing) and fdf_sync block until the stream has drained;
 *     device faults surface there as FDF_ERR_HIP.
 *   - A context is not thread-safe: use it from one host thread at a time.
 *
 * Particle ids: species i with N particles has ids 0..N-1.  Arrays exchanged
 * with the host are indexed by id, whatever order the device keeps them in.
 */
#ifndef FASTDF_H
#define FASTDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDF_ABI_VERSION 1

typedef struct fdf_ctx fdf_ctx;

typedef enum fdf_status {
  FDF_OK = 0,
  FDF_ERR_ARG = -1,          /* invalid argument or configuration */
  FDF_ERR_STATE = -2,        /* call not valid in the current state */
  FDF_ERR_WORKSPACE = -3,    /* no workspace, or too small / misaligned */
  FDF_ERR_HIP = -4,          /* a HIP runtime call failed */
  FDF_ERR_CAPACITY = -5,     /* more fields / species / particles than configured */
  FDF_ERR_UNSUPPORTED = -6   /* valid request that this build does not implement */
} fdf_status;

/* Arithmetic of the push (sec. 3.3 integrator):
 *   FP64: positions, momenta and grids in binary64.
 *   FP32: positions as 32-bit fixed-point fractions of the box (periodic wrap
 *         is the integer overflow), momenta as the binary32 initial momentum
 *         q0 plus the binary32 sum of the kicks dq (so rounding scales with
 *         dq, not q), gradient grids in bfloat16; schedule and weights in
 *         binary64. */
enum { FDF_PREC_FP64 = 0, FDF_PREC_FP32 = 1 };

/* Linear potentials (see fdf_config.potential_model):
 *   POISSON: phi_k = -(3/2) H0^2 Omega_m D(a) delta_0(k) / (a k^2), D = a
 *            (constant in time, phi-dot = 0);
 *   RADMAT : the same shape times the super-horizon radiation-to-matter
 *            factor g(a) in (1, 10/9), so phi-dot != 0 (a synthetic time-dependent
 *            model; the paper takes transfer functions from a Boltzmann code).
 * In both, psi = phi (1 - slip_amp exp(-k / slip_k)). */
enum { FDF_MODEL_POISSON = 0, FDF_MODEL_RADMAT = 1 };

/* Equations of motion of the push (fdf_config.eom).  With eps = sqrt(q^2 + m^2 a^2):
 *   SEPARABLE: eq. releq_approx / geodesic_approx (sec. 3.3), the force taken at
 *              the initial momentum q0, velocity q/eps: the fast default.
 *   EXACT:     eq. releq / geodesic (sec. 3.1) at the current q, with the drift
 *              factor (1 + phi + psi).
 *   CANONICAL: eq. releq_lag / geodesic_lag (sec. 3.2) in the canonical momentum
 *              P, which then takes the place of q everywhere (sampling, weights):
 *              the substitution of P for q that sec. 4 shows to be biased.
 *   SR_NEWTON: eq. p_eq (sec. 5), Newtonian gravity with special-relativistic
 *              velocities in P.
 *   SIMPLE_Q:  eq. q_eq (sec. 5), F = -eps grad psi.
 *   NEWTONIAN: F = -m a grad psi with the relativistic velocity (sec. 5).
 * The non-separable forms integrate an explicit kick-drift-kick whose
 * half-kicks use the momentum they start from (one mesh gather per step). */
enum {
  FDF_EOM_SEPARABLE = 0, FDF_EOM_EXACT = 1, FDF_EOM_CANONICAL = 2,
  FDF_EOM_SR_NEWTON = 3, FDF_EOM_SIMPLE_Q = 4, FDF_EOM_NEWTONIAN = 5
};

/* Power-spectrum estimator (sec. 4): CROSS = cross spectrum of the even-id and
 * odd-id halves (no shot-noise plateau); AUTO = auto spectrum of all particles. */
enum { FDF_PK_CROSS = 0, FDF_PK_AUTO = 1 };

/* Quantity of fdf_power_spectrum: the energy-density contrast (eq.
 * empirical_rho) or the momentum perturbation (1 + delta) theta (sec. 4). */
enum { FDF_PK_DENSITY = 0, FDF_PK_MOMENTUM = 1 };

/* fdf_init_species flags */
enum {
  /* apply the pre-initial conditions of sec. 2.1, eq. transform, with the
   * super-horizon moments delta = -2 psi and theta = k^2 tau psi / 2 */
  FDF_SPECIES_PRE_IC = 1
};

/* Kernel classes for fdf_read_timing */
enum {
  FDF_KERNEL_PUSH = 0,       /* gather + kick-drift-kick, one launch per step  */
  FDF_KERNEL_SORT = 1,       /* spatial bucket sort of the particle state      */
  FDF_KERNEL_GRID = 2,       /* Fourier stage + 3-D C2R FFT of the potentials  */
  FDF_KERNEL_INIT = 3,       /* field generation and particle sampling          */
  FDF_KERNEL_OUTPUT = 4,     /* weights, deposit, forward FFT and binning       */
  FDF_KERNEL_PUSH_SORT = 5,  /* push launches that also carry out a re-sort
                                (their rank passes count as SORT)               */
  FDF_KERNEL_COUNT = 6
};

typedef struct fdf_config {
  int32_t abi_version;     /* must equal FDF_ABI_VERSION */
  int32_t grid_n;          /* G: mesh points per side, a power of two in [8, 1024] */
  double box_mpc;          /* L: periodic box side [Mpc], > 0 */
  double h;                /* H0 = 100 h km/s/Mpc */
  double omega_m, omega_r, omega_l;   /* background densities, H(a) = H0 sqrt(...) */
  double z_begin, z_end;   /* integration range; z_end > z_begin integrates backward */
  int32_t n_steps;         /* number of constant-Delta-log-a steps, >= 1 */
  int32_t precision;       /* FDF_PREC_* */
  int32_t potential_model; /* FDF_MODEL_* */
  int32_t eom;             /* FDF_EOM_* */
  double slip_amp, slip_k; /* psi = phi (1 - slip_amp exp(-k/slip_k)); slip_k in 1/Mpc */
  double ns, sigma8, gamma;/* P(k) = A k^ns T_BBKS(k/(gamma h))^2, sigma(8 Mpc/h) = sigma8 */
  int32_t sort_every;      /* spatial re-sort of particles every this many steps (0: never) */
  int32_t max_fields;      /* capacity: number of seeded fields (each owns one grid set) */
  int32_t max_species;     /* capacity: number of species */
  int32_t interp_order;    /* force interpolation order r (sec. 4): 0 or 1 CIC (8 points),
                              2 TSC (27 points); deposits stay CIC */
  int64_t max_particles;   /* capacity: total particles over all species */
  double superstep_tol;    /* time-dependent potentials only.  0: rebuild the grids at
                              every kick time.  > 0: super-steps (sec. 2.1) -- grids are
                              built at anchor times where the transfer functions have
                              changed by more than this fraction since the previous
                              anchor, and linearly interpolated in a in between */
  int32_t pad_mesh;        /* FP32 form with psi != phi and phi-dot identically zero (POISSON):
                              0 stores the six gradient slots in 12-byte bfloat16 cells (the
                              default: 25 % less mesh traffic), 1 in 16-byte cells with a zero
                              slot and a pad (aligned, never across a cache line).  No effect
                              otherwise; results are bit for bit the same */
} fdf_config;

typedef struct fdf_info {
  int32_t step_index;      /* current integer time k: the state is at a_k */
  int32_t n_steps;
  double a_current;        /* a_k */
  double amplitude;        /* A of P(k) = A k^ns T^2 [Mpc^(3+ns)] */
  double tau_begin;        /* conformal time at z_begin [Mpc] */
  int32_t n_fields, n_species;
  int64_t n_particles;     /* total over species */
  size_t workspace_used;   /* bytes of the workspace in use */
} fdf_info;

/* Launch and sort parameters (picked by the autotuner or set by hand).  None
 * changes results: the push is per particle and the sort only permutes. */
typedef struct fdf_tuning {
  int32_t particles_per_thread;  /* push: 1, 2, 4 or 8 */
  int32_t sort_tiles;            /* sort buckets per axis: a power of two <= min(G, 256);
                                    particles are ordered by the Morton index of
                                    their bucket, then of their cell inside it;
                                    0 selects G/4 (4^3 cells per bucket) */
  int32_t sort_every;            /* re-sort cadence in steps; 0 never.  Values > 0
                                    need a context created with sort_every > 0 */
  float sort_cells;              /* > 0: adaptive cadence instead -- re-sort once the
                                    typical drift since the last sort (mean-momentum
                                    particle of the fastest species, in mesh cells)
                                    reaches this value; 0: use sort_every */
  int32_t persistent_blocks;     /* push launch: 0 = one block per particle chunk;
                                    > 0 = a persistent grid of this many blocks
                                    (a multiple of 8) striding over the chunks */
  int32_t use_graph;             /* 1: fdf_step captures its launch sequence into
                                    a hipGraph (once per distinct starting state)
                                    and replays it; per-kernel timing is then off */
  int32_t sort_predict;          /* 1: order by the positions extrapolated to the
                                    middle of the interval until the next re-sort
                                    (halves the spread of neighbours); 0: by the
                                    current positions */
  int32_t sort_fused;            /* 1: FP32 separable form -- a re-sort after the
                                    first is carried out by the push of that step,
                                    which writes the updated state in sorted order
                                    (no separate move pass; results bit-identical;
                                    the default); 0: rank + move passes, then
                                    the push */
  int32_t push_waves;            /* plain push launch (not one that carries out a
                                    re-sort): at most this many resident waves per
                                    SIMD (2-8; enforced by reserving LDS per block),
                                    fewer waves keeping more of each block's mesh
                                    neighbourhood in cache; 0: as many as the
                                    registers allow */
  int32_t sort_push_ppt;         /* push that carries out a re-sort: particles per
                                    thread (1, 2 or 4; 0 selects 4) of its
                                    1024-particle blocks */
  int32_t sort_keys_push;        /* 1 (the default): with one species, CIC, no
                                    super-steps and no graph, the plain push of the
                                    step before a re-sort in the same fdf_step call
                                    also writes the particles' sort keys, which the
                                    rank pass then reads instead of the state (4
                                    instead of 36 bytes per particle; results
                                    bit-identical); 0: the rank pass computes them */
} fdf_tuning;

/* ---- lifetime -------------------------------------------------------------- */

/* Bytes of device workspace a context with this configuration needs (host only;
 * callable without a GPU).  Returns FDF_ERR_ARG for an invalid configuration. */
int fdf_workspace_size(const fdf_config* cfg, size_t* bytes);

/* Validate cfg, build the FP64 schedule (sec. 3.3: constant Delta log a,
 * Delta tau = int dlog a / (a H)) and the sigma_8 normalisation; no device
 * memory is touched.  stream: a hipStream_t (NULL = the default stream).
 * *out receives the new context.  Errors: FDF_ERR_ARG. */
int fdf_create(const fdf_config* cfg, void* stream, struct fdf_ctx** out);

/* Attach the caller-owned device workspace (>= fdf_workspace_size bytes,
 * 256-byte aligned).  The memory must stay valid until fdf_destroy. */
int fdf_attach_workspace(struct fdf_ctx* ctx, void* device_ptr, size_t bytes);

/* Forget all fields and species (the workspace is reused), rewind to step 0. */
int fdf_reset(struct fdf_ctx* ctx);

/* Release the context's host resources.  Does not free the workspace. */
int fdf_destroy(struct fdf_ctx* ctx);

/* ---- inputs ---------------------------------------------------------------- */

/* Generate the seeded Gaussian field delta_0(k) on the device (one Philox4x64
 * draw per mode; fixed_amp != 0: |delta_k| = sqrt(P/V), the fixed initial
 * conditions of sec. 4).  *field_id receives its index. */
int fdf_add_field(struct fdf_ctx* ctx, uint64_t seed, int32_t fixed_amp, int32_t* field_id);

/* Upload delta_0(k) from the host: host pointer to G*G*(G/2+1) complex values
 * as interleaved (re, im) doubles in the half-complex layout [ix][iy][iz].
 * Modes with a Nyquist component are ignored (taken as zero). */
int fdf_set_field(struct fdf_ctx* ctx, const double* h_delta_k, int32_t* field_id);

/* Sample N particles of mass m_ev for field field_id (sec. 2.1: uniform
 * positions, Fermi-Dirac momenta; pdf of |q| proportional to q^2 fbar(q)),
 * all draws from Philox4x64(seed, id).  flags: FDF_SPECIES_PRE_IC applies
 * eq. transform at a_begin (builds a psi grid internally).  Only before the
 * first fdf_step.  *species_id receives its index. */
int fdf_init_species(struct fdf_ctx* ctx, int32_t field_id, double m_ev, int64_t n,
                     uint64_t seed, int32_t flags, int32_t* species_id);

/* Hand-placed particles: host arrays indexed by id, h_xu[n][3] uint32 fixed
 * point positions (x = L u / 2^32) and h_q[n][3] binary32 momenta [eV];
 * q0 = p = q.  Only before the first fdf_step. */
int fdf_set_species_state(struct fdf_ctx* ctx, int32_t field_id, double m_ev, int64_t n,
                          const uint32_t* h_xu, const float* h_q, int32_t* species_id);

/* ---- hot path -------------------------------------------------------------- */

/* Fourier stage + 3-D C2R FFT: gradient grids of psi and phi and the phi-dot
 * grid of field field_id at scale factor a (sec. 2.1: potentials from linear
 * transfer functions on a shared mesh).  fdf_step calls it by itself when the
 * grids are missing or the model is time dependent. */
int fdf_build_potential_grids(struct fdf_ctx* ctx, int32_t field_id, double a);

/* Advance every species n steps of the schedule (sec. 3.3 leapfrog; adjacent
 * half-kicks of consecutive steps are fused into one launch).  n < 0 walks
 * the same schedule backward.  Returns with positions and momenta at a
 * schedule point.  Errors: FDF_ERR_ARG when the step range leaves [0, n_steps]. */
int fdf_step(struct fdf_ctx* ctx, int32_t n);

/* delta-f weights (sec. 2.2): w = 1 - fbar(|q|)/fbar(|p|), p the sampled
 * momentum, evaluated without cancellation in binary64.  d_w: device pointer
 * to N doubles, written by id. */
int fdf_weights(struct fdf_ctx* ctx, int32_t species_id, double* d_w);

/* Energy-density contrast of eq. empirical_rho (CIC deposit of w eps with the
 * normalisation G^3 / (N <eps>)), forward FFT and log-binned spectrum over
 * [2 pi/L, pi G/L) (sec. 4).  Several species give their total contrast: the
 * relic species share one temperature (sec. 2) and so one number density, and
 * each species' contrast (normalised by its own count and <eps>) enters with
 * the weight <eps>_s(a) / sum_s <eps>_s.  The species must share one field and
 * appear once each (FDF_ERR_ARG otherwise).  Host outputs of n_bins doubles:
 * mean |k| [1/Mpc], P(k) [Mpc^3] (NaN for an empty bin) and the number of
 * modes.  The bin sums are exact fixed-point sums in both forms, and the FP32
 * form also deposits in fixed point, so its spectrum is the same bit for bit
 * from run to run, whatever the launch shape, sort cadence or particle
 * order. */
int fdf_density_power_spectrum(struct fdf_ctx* ctx, const int32_t* species, int32_t n_species,
                               int32_t n_bins, int32_t mode,
                               double* h_k, double* h_p, double* h_nmodes);

/* Power spectrum of the momentum perturbation (1 + delta) theta (sec. 4): the
 * delta-f deposit J of w q = w eps v per axis, normalised as the density
 * contrast, and Theta(k) = sum_a i k_a J_a(k); binned as
 * fdf_density_power_spectrum (same modes, CROSS or AUTO) in Mpc^3 / Mpc^2.
 * Uses the density buffers as scratch: fdf_read_density fails afterwards
 * until the next fdf_density_power_spectrum. */
int fdf_momentum_power_spectrum(struct fdf_ctx* ctx, const int32_t* species, int32_t n_species,
                                int32_t n_bins, int32_t mode,
                                double* h_k, double* h_p, double* h_nmodes);

/* Either spectrum (quantity FDF_PK_DENSITY or FDF_PK_MOMENTUM) estimated on an
 * analysis mesh of analysis_n points per side instead of G: a power of two in
 * [8, G], or 0 for G.  The bins then span [2 pi/L, pi analysis_n/L).  Runs on
 * different meshes G compared on one analysis mesh differ only through the
 * force resolution (sec. 4, the mesh-size study), not through the estimator.
 * fdf_read_density afterwards needs analysis_n = G (or 0) and the density. */
int fdf_power_spectrum(struct fdf_ctx* ctx, const int32_t* species, int32_t n_species,
                       int32_t n_bins, int32_t mode, int32_t quantity, int32_t analysis_n,
                       double* h_k, double* h_p, double* h_nmodes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * spectrum of fdf_power_spectrum on an analysis mesh of analysis_n points per
 * side, a power of two in [8, min(64, G)] (0 means G and is accepted only when
 * G <= 64), computed without any allocation.  Its temporaries (deposit
 * halves, FFT planes, bin sums) live in a static 16 MiB device array of the
 * library, one per GPU, held until the process ends; a larger mesh returns
 * FDF_ERR_ARG.  d_out: device pointer to 3 * n_bins doubles, written as
 * [mean |k|][P(k)][modes] (NaN means for an empty bin).  Enqueued on the
 * context stream; nothing is copied to the host and nothing waits.  Every
 * call on one GPU uses the same array, so calls that overlap on one GPU (two
 * streams, two threads, two contexts) race; calls in stream order do not.
 * Other errors as fdf_power_spectrum. */
int fdf_power_spectrum_noalloc(struct fdf_ctx* ctx, const int32_t* species, int32_t n_species,
                               int32_t n_bins, int32_t mode, int32_t quantity, int32_t analysis_n,
                               double* d_out);

/* Fig. 2 diagnostic (sec. 3.1): root mean square over the species' particles
 * of the magnitude of each term of eq. releq at the current state and a_k --
 * h_rms[0] = |eps grad psi|, [1] = |(q^2/eps) grad phi|, [2] = |q (q.grad phi)/eps|,
 * [3] = |q phidot| [eV/Mpc] -- with eps from the current momentum and the
 * mesh values interpolated by CIC.  Builds the grids at a_k when they are not
 * current (with super-steps this replaces the first grid set).  Blocking.
 * FDF_ERR_UNSUPPORTED when the equation of motion's layout lacks grad phi or
 * phi-dot (canonical, SR-Newtonian, simple-q and Newtonian forms). */
int fdf_force_terms(struct fdf_ctx* ctx, int32_t species_id, double* h_rms);

/* ---- read-back (blocking) -------------------------------------------------- */

/* Current state in binary64, indexed by id: h_x[n][3] in [0, L) Mpc,
 * h_q[n][3] eV (any pointer may be NULL to skip it). */
int fdf_read_state(struct fdf_ctx* ctx, int32_t species_id, double* h_x, double* h_q);

/* One slot of a field's grid set as G^3 doubles [ix][iy][iz]: slots 0-2 grad psi,
 * 3-5 grad phi, 6 phi-dot. */
int fdf_read_grid(struct fdf_ctx* ctx, int32_t field_id, int32_t slot, double* h_grid);

/* delta_0(k) as G*G*(G/2+1) interleaved complex doubles. */
int fdf_read_field(struct fdf_ctx* ctx, int32_t field_id, double* h_delta_k);

/* The last density contrast deposited by fdf_density_power_spectrum: half 0 or 1
 * (AUTO mode: half 0), G^3 doubles. */
int fdf_read_density(struct fdf_ctx* ctx, int32_t half, double* h_grid);

/* The FP64 schedule: five arrays of n_steps (+1 for a) doubles written back to
 * back: a[n+1], a_half[n], kick1[n], kick2[n], drift[n]. */
int fdf_read_schedule(const struct fdf_ctx* ctx, double* h_table);

int fdf_get_info(const struct fdf_ctx* ctx, fdf_info* info);

/* Read or replace the launch and sort parameters.  Errors: FDF_ERR_ARG for a
 * value outside the ranges documented in fdf_tuning. */
int fdf_get_tuning(const struct fdf_ctx* ctx, fdf_tuning* tuning);
int fdf_set_tuning(struct fdf_ctx* ctx, const fdf_tuning* tuning);
int fdf_sync(struct fdf_ctx* ctx);

/* Per-kernel-class timing with HIP events on the context stream. */
int fdf_timing_enable(struct fdf_ctx* ctx, int32_t enable);
int fdf_read_timing(struct fdf_ctx* ctx, int32_t kernel_class, double* total_ms, int64_t* launches);
int fdf_timing_reset(struct fdf_ctx* ctx);

/* Work done by the timed launches of a kernel class since the last
 * fdf_timing_reset (counted while timing is enabled; the push classes only):
 * work[0] particle-updates with a drift, work[1] kick-only particle-updates,
 * work[2] mesh cells read (one per cell of each field mesh a launch gathers
 * from, two with super-step blending).  Host pointer to 3 int64. */
int fdf_read_work(struct fdf_ctx* ctx, int32_t kernel_class, int64_t* work);

const char* fdf_status_string(int status);
const char* fdf_last_error(const struct fdf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FASTDF_H */
