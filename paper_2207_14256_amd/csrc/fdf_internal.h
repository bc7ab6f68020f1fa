// Internal interface between the host runtime (fdf_host.cpp) and the HIP
// kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fdf {

// ----------------------------------------------------------------------------
// Layout of the gradient meshes: 4 x 4 x 4-cell bricks, bricks in x, y, z
// order and cells inside a brick in x, y, z order, so that the CIC or TSC
// corners of a particle lie in one or two kilobyte-sized bricks instead of
// rows a whole x-plane apart.  The index of cell (ix, iy, iz) on a G^3 mesh
// (G a power of two >= 8) is mesh_x(ix) + mesh_y(iy) + mesh_z(iz).
// ----------------------------------------------------------------------------
// (G is a power of two: the brick strides are shifts, not multiplications)
__host__ __device__ inline uint32_t log2_pow2(uint32_t G) { return 31u - (uint32_t)__builtin_clz(G); }
__host__ __device__ inline uint32_t mesh_x(uint32_t i, uint32_t G) {
  return ((i >> 2) << (2u * log2_pow2(G) + 2u)) + (i & 3u) * 16u;
}
__host__ __device__ inline uint32_t mesh_y(uint32_t i, uint32_t G) { return ((i >> 2) << (log2_pow2(G) + 4u)) + (i & 3u) * 4u; }
__host__ __device__ inline uint32_t mesh_z(uint32_t i) { return (i >> 2) * 64u + (i & 3u); }

// ----------------------------------------------------------------------------
// Grid recipe: which potential-derived quantity each output slot carries.
// ----------------------------------------------------------------------------
enum SlotKind : int32_t {
  SK_ZERO = 0,
  SK_DX_PSI = 1, SK_DY_PSI = 2, SK_DZ_PSI = 3,
  SK_DX_PHI = 4, SK_DY_PHI = 5, SK_DZ_PHI = 6,
  SK_PHIDOT = 7,
  SK_PSI = 8,
  SK_PHI = 9,
  SK_PHI_PSI = 10,         // phi + psi
};

// Transfer functions at one scale factor (host evaluates the time factors):
//   T_phi(k)    = c_phi / k^2
//   T_psi(k)    = T_phi(k) (1 - slip_amp exp(-k / slip_k))
//   T_phidot(k) = c_phidot / k^2
struct Transfer {
  double c_phi, c_phidot, slip_amp, slip_k;
};

// Output element type of a grid set.
enum GridType : int32_t { GT_BF16 = 0, GT_F32 = 1, GT_F64 = 2 };

struct GridBuildArgs {
  int32_t G;
  int32_t fp64;            // 1: FFT in binary64, 0: binary32
  int32_t nslot;           // 4 or 8 slots per cell in the output
  int32_t nfft;            // number of non-zero slots (FFTs to run)
  int32_t kind[8];         // SlotKind of FFT i
  int32_t slot[8];         // output slot of FFT i
  int32_t out_type;        // GridType
  double kf;               // 2 pi / L
  Transfer tr;
  const void* delta_k;     // complex [G][G][G/2]
  void* scratch;           // complex [nfft][G][G][G/2]
  const void* twiddle;     // complex [G], e^{-2 pi i m / G}, same precision as the FFT
  void* out;               // [G^3][nslot] of out_type
};

struct PkArgs {
  int32_t G;
  int32_t fp64;
  int32_t nbins;
  int32_t auto_mode;       // 1: only grid a is transformed, P = |a|^2
  double volume;           // L^3
  const void* grid_a;      // real [G^3]
  const void* grid_b;
  void* scratch;           // complex [2][G][G][G/2]
  const void* twiddle;
  double* bins;            // [3][nbins]: count, sum |k|, sum P, written by the binning
  unsigned long long* acc; // [5][nbins] exact bin sums: count, sum |n| (128-bit fixed point,
                           // lo and hi words), sum P (128-bit fixed point, lo and signed hi)
                           // (zeroed by the caller, with *max_bits)
  uint32_t* max_bits;      // binary32 bits of the largest |P| of a mode (the P quantum)
  double kf;
  int32_t deriv_axis;      // -1: transform the halves in place (planes 0, 1); 0-2: multiply by
                           // i k_axis and add into scratch planes 2 (and 3)
  int32_t accum_first;     // 1: the first term of the sum (store instead of add)
  int32_t bin_plane;       // first plane the binning reads: 0 (density) or 2 (momentum)
};

// Segment of the batched particle state: one species.
struct Segment {
  // FP32 form: positions as uint32 fixed point; the momentum is q0 + dq with
  // q0 the momentum at the start (binary32) and dq the accumulated kicks
  uint32_t* xu[3];
  float* q0f[3];
  float* dqf[3];
  // FP64 form
  double* xd[3];
  double* qd[3];
  double* q0d[3];
  uint32_t* id;
  const void* grid;        // [G^3][nslot]
  const void* grid2;       // second grid set (super-steps), or null
  double m;                // mass [eV]
  int64_t n;               // particles
  int64_t chunk_begin;     // first chunk of this segment in the launch
};

// Particles per block of the sort's rank pass.
constexpr int kSortBlock = 1024;

// A batched re-sort (FP32 separable form): the species due at one step are
// ranked by one launch, scanned together and moved by one fused push launch.
// Job j is species job_species[j], whose current state is in copy
// job_cur[j] of the segment tables; its rank blocks (kSortBlock particles
// each) are [job_block[j], job_block[j + 1]); its bucket counts are
// count + j nkeys, scanned together with the other jobs' so that its bucket
// starts are offset by job_base[j] (the particles of the jobs before it), and
// its rank-pass outputs are rank, bucket and src + job_base[j].
constexpr int kMaxSortJobs = 16;
struct SortBatch {
  int32_t njobs;           // 0: not batched (SortArgs.seg, one species)
  int32_t job_species[kMaxSortJobs];
  int32_t job_cur[kMaxSortJobs];
  int64_t job_block[kMaxSortJobs + 1];
  int64_t job_base[kMaxSortJobs];
  double job_tau[kMaxSortJobs];   // predict_tau of the job's species
  double job_ma[kMaxSortJobs];    // m a of the job's species
  const Segment* tables[2];       // device segment tables, copies 0 and 1
};

// Block b of a batched launch: each XCD (b mod 8) takes a contiguous eighth
// of every job's blocks.  Returns the job and (*local) the block inside it,
// or -1 for a block past its XCD's share (the grid is 8 times the largest).
__device__ inline int batch_block(const SortBatch& sb, int64_t b, int64_t* local) {
  const int64_t x = b & 7;
  int64_t l = b >> 3;
  for (int j = 0; j < sb.njobs; ++j) {
    const int64_t n = sb.job_block[j + 1] - sb.job_block[j];
    const int64_t lo = n * x / 8, hi = n * (x + 1) / 8;
    if (l < hi - lo) { *local = lo + l; return j; }
    l -= hi - lo;
  }
  return -1;
}

// Grid of a batched launch (host).
inline int64_t batch_grid(const SortBatch& sb) {
  int64_t most = 0;
  for (int64_t x = 0; x < 8; ++x) {
    int64_t share = 0;
    for (int j = 0; j < sb.njobs; ++j) {
      const int64_t n = sb.job_block[j + 1] - sb.job_block[j];
      share += n * (x + 1) / 8 - n * x / 8;
    }
    most = most > share ? most : share;
  }
  return 8 * most;
}

struct PushArgs {
  const Segment* seg;      // device array: each species' segment in copy 0 of its state
  const Segment* seg_alt;  // the same in copy 1 (the other buffer of a sorting species)
  uint64_t alt_mask;       // species whose current state is in copy 1 (species index < 64)
  uint64_t skip_mask;      // species this launch leaves alone (pushed by a fused re-sort)
  int32_t nseg;
  int64_t total_chunks;
  int32_t fp64;
  int32_t nslot;
  int32_t log2g;
  int32_t G;
  int32_t do_kick, do_drift;
  int32_t eom;             // 0: separable form (fdf_config.eom), else a form of fdf_push_eom.hip
  double kick;             // separable: fused kick coefficient [Mpc]; other forms: closing half-kick
  double kick_open;        // other forms: opening half-kick of the next step (applied second)
  double a_kick;           // a at the kick
  double drift;            // Delta tau of the drift [Mpc]
  double a_drift;          // a_{k+1/2}
  double box;              // L
  int32_t ppt;             // particles per thread (fused re-sort push: 1, 2 or 4)
  int32_t persistent;      // 0: one block per chunk; > 0: this many blocks (a multiple of 8) loop
  int32_t tsc;             // 1: TSC (r = 2) force interpolation, 0: CIC
  int32_t blend;           // 1: interpolate two grid sets (super-steps)
  int32_t grid_sel;        // which set holds the earlier anchor: 0 = grid, 1 = grid2
  double blend_t;          // interpolation weight of the later anchor
  int32_t lds_reserve;     // bytes of LDS reserved per block (caps resident waves), or 0
  int64_t xcd_blocks;      // > 0: grid of the segment-balanced XCD mapping (several segments)
  // push fused with the move of a re-sort (launch_push_sort; FP32 separable
  // form, one species: seg and dseg point at its entry in the two tables,
  // total_chunks counts its kSortBlock-particle rank blocks)
  const Segment* dseg;     // destination copy
  const uint32_t* sort_src;     // rank pass outputs (SortArgs::src, rank, bucket)
  const uint32_t* sort_rank;
  const uint32_t* sort_bucket;
  const uint32_t* sort_start;   // bucket starts (the scanned counts)
  int64_t sort_nkeys;           // buckets per job (batched re-sort)
  SortBatch sort_batch;         // batched re-sort: njobs > 0 (seg / seg_alt are the two tables)
  // sort keys of the next step's re-sort, written by this (plain, FP32,
  // one-species) push from the state it leaves: key_out[i] for particle slot i
  uint32_t* key_out;            // or null
  int32_t key_fine_bits;        // log2 of the bucket tile side in cells
  double key_tau;               // predict_tau of the next re-sort
  double key_ma;                // m a at the middle of its interval
};

struct SortArgs {
  Segment seg;             // source copy
  Segment dst;             // destination copy
  double predict_tau;      // order by x + v * predict_tau (conformal time, Mpc; 0: by x)
  double ma;               // m a for the velocity v = q / sqrt(q^2 + (m a)^2)
  int32_t fp64;
  int32_t grid_n;          // G
  int32_t cell_shift;      // 32 - log2(G): cell index of a fixed-point position
  int32_t fine_bits;       // log2 of the bucket tile side in cells
  double box;
  int64_t nkeys;           // number of buckets, (G >> fine_bits)^3
  uint32_t* count;         // [nkeys] bucket counts, scanned in place into bucket starts
  uint32_t* scan_scratch;  // sort_scan_scratch_words(nkeys) words
  uint32_t* rank;          // [n] per sorted element of each 1024-block: rank inside its bucket
  uint32_t* bucket;        // [n] per sorted element: bucket
  uint32_t* src;           // [n] per sorted element: source slot inside the block
  int32_t id_only;         // move pass: move the ids alone (the caller re-samples the state by id)
  SortBatch batch;         // rank pass over several species (batch.njobs > 0; seg, dst unused)
  const uint32_t* keys;    // rank pass: keys written by the previous push (one species), or null
};

struct SampleArgs {
  Segment seg;
  int32_t fp64;
  int32_t by_id;           // 1: slot i takes the particle seg.id[i] (ids kept); 0: slot i is id i
  uint64_t seed;
  double box;
  double t_nu;             // k_B T [eV]
};

struct FieldGenArgs {
  int32_t G;
  int32_t fp64;
  int32_t fixed_amp;
  uint64_t seed;
  double box, amp, ns, gamma, h;
  void* out;               // complex [G][G][G/2]
};

struct PreIcArgs {
  Segment seg;
  int32_t fp64;
  int32_t G;
  double box, m, a, tau;
  const void* grid;        // [G^3][4] f64: dpsi/dx, dpsi/dy, dpsi/dz, psi
};

struct OutputArgs {
  Segment seg;
  int32_t fp64;
  int32_t G;
  int32_t pre_ic;          // p regenerated from (seed, id) instead of q0
  uint64_t seed;
  double t_nu;
  double box, a, m;
  double norm[2];          // deposit normalisation per half (even / odd id)
  int32_t auto_mode;
  int32_t quantity;        // -1: deposit w eps (energy density); 0-2: w q_axis (momentum density)
  double* w_out;           // weights by id (may be null)
  void* dens[2];           // per half, [G^3]: f64 (FP64 form) or int64 fixed point (FP32 form)
  uint32_t* max_bits;      // FP32 form: binary32 bits of the largest |deposited value|
  int32_t fixed_bits;      // FP32 form: the quantum is 2^(e - fixed_bits), max |value| < 2^e
};

// Fixed-point deposit halves (bricked cell order) -> x-major binary32 meshes
// (n cells in all, n_half = G^3 per half).
struct FixedToRealArgs {
  const long long* src[2];
  float* dst[2];
  size_t n, n_half;
  int32_t G;
  const uint32_t* max_bits;
  int32_t fixed_bits;
};

// Acceleration terms of eq. releq (Fig. 2 diagnostic): sums over particles of
// the squared magnitude of each of the four terms.
struct TermArgs {
  Segment seg;
  int32_t fp64;
  int32_t G;
  int32_t nslot;
  int32_t slot_gpsi;       // first of three slots of grad psi
  int32_t slot_gphi;       // first of three slots of grad phi
  int32_t slot_phidot;     // slot of phi-dot, or -1 when it is zero
  double box, ma;
  const void* grid;        // [G^3][nslot], bf16 (FP32 form) or f64
  double* out;             // [4], zeroed by the caller
};

void launch_field_gen(const FieldGenArgs& a, hipStream_t s);
void launch_force_terms(const TermArgs& a, hipStream_t s);
void launch_sample_species(const SampleArgs& a, hipStream_t s);
void launch_pre_ic(const PreIcArgs& a, hipStream_t s);
void launch_build_grids(const GridBuildArgs& a, hipStream_t s);
void launch_push(const PushArgs& a, hipStream_t s);
void launch_push_eom(const PushArgs& a, hipStream_t s);
void launch_weights(const OutputArgs& a, hipStream_t s);
void launch_deposit(const OutputArgs& a, hipStream_t s);
void launch_deposit_max(const OutputArgs& a, hipStream_t s);   // FP32 form, before launch_deposit
void launch_fixed_to_real(const FixedToRealArgs& a, hipStream_t s);
void launch_bins_finalize(const double* bins, int nbins, double* out, hipStream_t s);
void launch_power_spectrum(const PkArgs& a, hipStream_t s);
void launch_bin(const PkArgs& a, hipStream_t s);   // bins planes bin_plane (and + 1) into a.bins
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t s);
int push_chunk_particles(int ppt);
void launch_sort(const SortArgs& a, hipStream_t s);
void launch_sort_rank(const SortArgs& a, hipStream_t s);   // counts, rank pass and scan, no move
void launch_sort_rank_batch(const SortArgs& a, hipStream_t s);   // the same over a SortBatch
void launch_push_sort(const PushArgs& a, hipStream_t s);
size_t sort_scan_scratch_words(int64_t nkeys);

}  // namespace fdf
