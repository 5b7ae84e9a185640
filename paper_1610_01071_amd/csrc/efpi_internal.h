// Internal definitions shared by the HIP kernels and the host side of libefpi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "efpi.h"

namespace efpi {

constexpr double kFxScale = 1099511627776.0;     // 2^40: fixed-point charge unit 2^-40
constexpr double kFxInv = 1.0 / 1099511627776.0;

// The fixed-point charge of an ion and its CIC split, shared by every kernel that
// deposits (the particle pass and the lift), so that all deposits are the same
// integers: q = rint(w 2^40) as an exact binary64 integer, the right-node share
// rint(theta q) (one rounded product, ties to even) and the left share q - rint(theta q).
__device__ __forceinline__ double fx_charge(float w) {
  return __builtin_rint((double)w * kFxScale);
}
__device__ __forceinline__ double fx_share(float theta, double q) {
  return __builtin_rint((double)theta * q);
}
// rint(x) as int64 for |x| < 2^51: adding 1.5 * 2^52 leaves the integer part
// rounded to nearest (ties to even, the IEEE default) in the low mantissa bits.
__device__ __forceinline__ long long rint_i64(double x) {
  const double magic = 6755399441055744.0;
  return (long long)(__double_as_longlong(x + magic) - __double_as_longlong(magic));
}
constexpr int kWave = 64;

#define EFPI_GLOBAL __attribute__((address_space(1)))

// Global-memory view of an array address taken from a descriptor.  Accesses
// through it compile to global_* instructions; through the plain (generic)
// pointer they become flat_* ones, which also count against the LDS wait
// counter, so every later LDS wait would wait for the memory access as well.
template <class T>
__device__ __forceinline__ EFPI_GLOBAL T* gmem(T* p) {
  return (EFPI_GLOBAL T*)p;
}

// Element i of a global array addressed as a 32-bit byte offset (i * sizeof(T)
// below 2^32) from a base that is the same in every lane: the access takes the
// base from scalar registers and one vector offset, with no 64-bit address
// arithmetic per lane.
template <class T>
__device__ __forceinline__ EFPI_GLOBAL T* at(EFPI_GLOBAL T* base, unsigned i) {
  return (EFPI_GLOBAL T*)((EFPI_GLOBAL const char*)base + i * (unsigned)sizeof(T));
}

// Per-replica descriptor in device memory: sizes, parameters and the addresses
// of the replica's arrays inside the workspace.
struct RepDev {
  int32_t n_cells, n_nodes, bc, closure;
  int32_t ppc, levels, n_coarse, burst_steps;
  int32_t coevolving, lift_linear, log2n;
  int32_t field_m;       // rows per thread of the field solve (N / field_m <= 512 threads)
  int32_t moments;       // coarse moments: 2 (n, j) or 3 (n, j, s: EFREE)
  double h, inv_h, length, vth, dt, macro_dt, n_floor;
  int64_t capacity;
  int64_t item_begin;    // first particle work item of this replica
  int64_t block_begin;   // first coarse-block work item of this replica
  // particle store (SoA) and its sort copy
  int16_t* cell;
  float* frac;
  float* v;
  float* w;
  int16_t* cell2;
  float* frac2;
  float* v2;
  float* w2;
  int64_t* np;           // live particle slots
  // grid
  int64_t* q[2];         // fixed-point node charge, double-buffered
  double* phi;
  float* e;              // node field E^p
  float* en;             // field stored at the start of the burst (App. B step 1)
  // coarse
  int64_t* rbins;        // [K+1][moments][N_c] fixed-point block sums of the snapshots
  double* snap;          // [K+1][moments][N_c] snapshots (internal macro step)
  double* coarse_tmp;    // [moments][N_c]
  // lift
  double* prof_n;        // [N+1] fine density
  double* prof_u;        // [N+1] fine mean velocity
  double* prof_t;        // [N+1] fine temperature (three moments only)
  int32_t* cell_of_rank; // [N] occupied cells in order
  int32_t* block_rank;   // [N_c + 1] first occupied-cell rank of every block
  int64_t* aux;          // [4] per-replica scratch: [0] absorbed ions of a sort, [1] lift rotation
  // species of the store above: charge-to-mass ratio (1 for ions).  The
  // electron descriptor of a kinetic replica is a copy of the ion one with the
  // electron store, count, profile, rank arrays, aux, ppc, vth, capacity and qm.
  double qm;
  int64_t* jfx;          // kinetic ions: fixed-point node momentum of an electron reset
};

// Rotation of the electron quiet start relative to the ions' of the same lift.
constexpr uint32_t kElectronShiftXor = 0x9E3779B9u;

// Kernel flags of the particle pass.
enum : int {
  kFresh = 1,      // velocities are at an integer time level (first pass after load)
  kRestrict = 2,   // deposit snapshot p along the approximate characteristics
  kPush = 4,       // leapfrog step and deposit of the new charge
  kDepositOnly = 8, // deposit the charge of the current positions
  kMoment3 = 16      // the snapshot also restricts the second velocity moment
};

// Launchers (defined in the kernel sources), all asynchronous on `stream`.
constexpr int kMaxShiftReplicas = 256;
struct ShiftArg {
  uint32_t s[kMaxShiftReplicas];
};

// d_status receives EFPI_DEV_WEIGHT when an ion's |w| reaches the bound that
// keeps the exact charge sums exact.
void launch_particles(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                      int64_t total_items, int tile, int grid_blocks, int p, int flags,
                      int qsel, uint32_t* d_status, hipStream_t stream, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
// Newton solves of every replica in one launch, one workgroup each (R.field_m
// rows per thread).
void launch_newton(const RepDev* d_reps, int n_reps, int iters, int cold, int qsel, int save_en,
                   int zero_bins, double tol, uint32_t* d_status, hipStream_t stream);
void launch_prep_burst(const RepDev* d_reps, int n_reps, hipStream_t stream);
// Kinetic electrons (electrons.hip, field.hip).  d_ereps: electron descriptors.
// Push (gather, leapfrog with R.qm, periodic wrap) and deposit -charge into
// R.q[qsel]; with push == 0 only the deposit of the current positions.
void launch_electrons(const RepDev* d_ereps, int n_reps, int push, int fresh, int qsel,
                      int max_nodes, hipStream_t stream, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
// Linear periodic Poisson solve from R.q[qsel] of every replica in one launch
// (Newton's shape: R.field_m rows per thread): phi, E (and E_n with save_en), the
// other charge buffer cleared, the snapshot bins with zero_bins.
// Storage slot of node k's potential.  A field-solve thread keeps its M consecutive
// nodes in registers; the pair (2j, 2j + 1) of thread t is stored at pair slot
// j T + t (T = N / M threads), so that the solve's loads and stores of phi are
// coalesced across the threads.  Node N (walls) and M = 1 keep the natural order
// (with M = 2 the two orders coincide).
__host__ __device__ __forceinline__ int64_t phi_slot(int k, int n_cells, int m) {
  if (m < 2 || k >= n_cells) return k;
  const int t = k / m, r = k - t * m;
  return 2 * ((int64_t)(r >> 1) * (n_cells / m) + t) + (r & 1);
}
// Clear q[which] of every replica (one launch).
void launch_zero_charge(const RepDev* d_reps, int n_reps, int which, hipStream_t stream);
// Copy a replica's potential between the natural node order (the caller's) and the
// solve's storage order: to_natural != 0 reads the store into dst[0..n_nodes).
void launch_phi_copy(const RepDev* d_reps, int rep, const double* d_src, double* d_dst,
                     int to_natural, hipStream_t stream);
void launch_poisson(const RepDev* d_reps, int n_reps, int qsel, int save_en, int zero_bins,
                    uint32_t* d_status, hipStream_t stream);
// Electron loading profile of every replica: density exp(phi), mean velocity the
// ions' fine profile u (from_moments == 0) or the ion node momentum R.jfx over the
// ion node charge R.q[qsel] (from_moments != 0), and the rotation (ion rotation
// XOR kElectronShiftXor).
void launch_electron_profile(const RepDev* d_reps, const RepDev* d_ereps, int n_reps,
                             int from_moments, int qsel, hipStream_t stream);
// Fixed-point CIC momentum of the ions into R.jfx (cleared first), with
// velocities v + half_kick dt E at the ion (time-centred after a burst).
void launch_ion_momentum(const RepDev* d_reps, int n_reps, int half_kick, int max_nodes,
                         hipStream_t stream);
void launch_set_profile(const RepDev* d_reps, int rep, const double* d_n, const double* d_u,
                        hipStream_t stream);
// Fine profile and occupied-cell ranks of every replica before a lift; with
// shifts != nullptr also the lift rotations (as launch_set_shifts).
void launch_lift_prep(const RepDev* d_reps, int n_reps, const double* d_coarse,
                      const int64_t* d_coff, uint32_t* d_status, const ShiftArg* shifts,
                      hipStream_t stream);
void launch_occupancy(const RepDev* d_reps, int n_reps, int only_rep, uint32_t* d_status,
                      hipStream_t stream);
// Store each replica's lift rotation (R.aux[1]) for the next lift.
void launch_set_shifts(const RepDev* d_reps, int n_reps, int only_rep, const ShiftArg& shifts,
                       hipStream_t stream);
// Lift; with shifts == nullptr the rotations stored by launch_set_shifts are used.
// qsel >= 0: also deposit the lifted ions' charge into R.q[qsel] (zeroed before),
// which needs every replica's coarse blocks to be at most 64 cells wide
// (lift_can_deposit); d_status receives EFPI_DEV_WEIGHT then.  third (with
// d_coarse): three coarse moments, thermal speeds from the temperature profile
// and the second-moment stretch of the block correction.
constexpr int kLiftMaxDepositLevels = 6;
void launch_lift_particles(const RepDev* d_reps, const int64_t* d_block_prefix, int n_reps,
                           int64_t total_blocks, int only_rep, const double* d_coarse,
                           const int64_t* d_coff, const ShiftArg* shifts, int grid_blocks,
                           hipStream_t stream, int qsel = -1, uint32_t* d_status = nullptr,
                           bool third = false);
void launch_restrict(const RepDev* d_reps, int n_reps, int steps, double* d_snap,
                     const int64_t* d_soff, hipStream_t stream);
void launch_project(const RepDev* d_reps, int n_reps, const double* d_snap,
                    const int64_t* d_soff, double* d_out, const int64_t* d_coff,
                    uint32_t* d_status, hipStream_t stream);
// launch_restrict of all burst_steps + 1 snapshots followed by launch_project, in one launch.
void launch_restrict_project(const RepDev* d_reps, int n_reps, double* d_snap,
                             const int64_t* d_soff, double* d_out, const int64_t* d_coff,
                             uint32_t* d_status, hipStream_t stream);
// Slope, forward-Euler and second-order projections (d_slope_prev may be NULL).
void launch_project2(const RepDev* d_reps, int n_reps, const double* d_snap,
                     const int64_t* d_soff, const double* d_slope_prev, double gap,
                     double* d_slope, double* d_euler, double* d_out, const int64_t* d_coff,
                     uint32_t* d_status, hipStream_t stream);
void launch_ensemble_mean(const RepDev* d_reps, int n_reps, const int32_t* d_group,
                          double* d_coarse, const int64_t* d_coff, hipStream_t stream);
void launch_fill_u8(void* d_ptr, size_t bytes, hipStream_t stream);
// Phase-space coarse coefficients of replica rep's ions (phase.hip): the int64
// restricted histogram into d_hist [n_cells >> levels_x][2^jf], then the column
// transforms into d_out [n_cells >> levels_x][2^jc].
void launch_phase_restrict(const RepDev* d_reps, int rep, int n_cells, int levels_x, double v_min,
                           double v_max, int jf, int jc, const double* h_taps, int n_taps,
                           double tau, int fresh, int stored_field, double h, long long* d_hist,
                           double* d_out, hipStream_t stream);
// Ions of replica rep lifted from phase-space coefficients d_coarse [nxc][2^jc]:
// columns refined into d_cols [nxc][2^jf], CDFs repaired into d_cdf
// [n_cells][2^jf + 1], node densities in R.prof_n, ranks by the occupancy, load.
void launch_phase_lift(const RepDev* d_reps, int rep, int n_cells, int levels_x, double v_min,
                       double v_max, int jf, int jc, const double* h_taps, int n_taps,
                       const double* d_coarse, double* d_cols, double* d_cdf,
                       uint32_t* d_status, uint32_t shift, hipStream_t stream);
void launch_phase_project(const double* d_snap, int64_t count, int ne, double dt, double macro_dt,
                          double* d_out, hipStream_t stream);
void launch_copy_particles(const RepDev* d_reps, int rep, const int16_t* cell, const float* frac,
                           const float* v, const float* w, int64_t n, int to_store,
                           int16_t* ocell, float* ofrac, float* ov, float* ow,
                           hipStream_t stream);
void launch_sort(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                 int64_t total_items, int tile, int32_t* d_hist, int64_t* d_base,
                 int grid_blocks, hipStream_t stream);

// Learned projection network (nn.hip).
constexpr int kNnCin = EFPI_NN_CIN;
constexpr int kNnHidden = EFPI_NN_HIDDEN;
constexpr int kNnCout = EFPI_NN_COUT;
constexpr int kNnParams = EFPI_NN_PARAMS;
constexpr int kNnPackForward = 29696;  // bf16 elements of the four forward packs
constexpr int kNnPackElems = EFPI_NN_PACK_BYTES / 2;

namespace nn {
size_t workspace_floats(int batch, int nc);
void launch_pack(const float* params, uint16_t* pack, hipStream_t stream);
void launch_forward(const float* params, const uint16_t* pack, const float* x, float* y,
                    int batch, int nc, int periodic, float* ws, hipStream_t stream);
void launch_backward(const uint16_t* pack, const float* x, const float* dy, float* grad,
                     int batch, int nc, int periodic, float* ws, hipStream_t stream);
void launch_mse(const float* y, const float* t, float* dy, float* loss, int64_t count,
                hipStream_t stream);
void launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                 float b1, float b2, float eps, uint16_t* pack, hipStream_t stream);
void launch_features(const double* states, int n_states, const int32_t* index, int batch, int nc,
                     const efpi_nn_norm& nm, float noise, uint32_t seed, float* x, float* t,
                     hipStream_t stream);
void launch_step(const double* cn, const float* y, int batch, int nc, const efpi_nn_norm& nm,
                 double* out, hipStream_t stream);
void launch_predict_step(const float* params, const uint16_t* pack, const double* states, int nc,
                         int periodic, const efpi_nn_norm& nm, double* out, float* ws,
                         hipStream_t stream);
void launch_rel_l2(const double* a, const double* b, int64_t n, double* out, hipStream_t stream);
}  // namespace nn

}  // namespace efpi
