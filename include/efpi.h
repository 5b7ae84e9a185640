/*
 * efpi.h - C ABI of the MI355X EFPI / PIC-burst library (libefpi.so).
 *
 * The library advances electrostatic 1D1V particle-in-cell ions with Boltzmann
 * electrons and couples them to coarse Haar coefficients of the density and
 * momentum moments through the equation-free projective integration cycle of
 * Cazeaux & Hesthaven (arXiv:1610.01071), Sec. 3.1 and 3.3:
 *
 *   lift (App. C)  ->  N_e fine PIC steps, restricting after each (Sec. 2.2,
 *   App. B)  ->  least-squares slope (eq. 3.18)  ->  projection (eq. 3.17).
 *
 * Units: length in Debye lengths, time in inverse ion plasma frequencies,
 * potential in T_e/e, density in n_0; the ion charge-to-mass ratio is 1 and the
 * field equation is -phi'' + exp(phi) = n_i (eq. 3.15).
 *
 * Conventions that hold for every entry point:
 *  - Pointers named d_* are device pointers, h_* are host pointers.
 *  - Device memory is owned by the caller.  efpi_init binds one caller-owned
 *    workspace; the library never allocates or frees device memory.  Its one
 *    device array of its own is the static scratch of
 *    efpi_phase_restrict_static, which the loaded code object holds on each GPU.
 *  - Every call that touches the device only enqueues work on the context's
 *    HIP stream and returns; results are visible after the stream synchronises.
 *    Calls documented as synchronous say so.
 *  - Argument checks happen before anything is enqueued; a rejected call
 *    returns a negative efpi_status, enqueues nothing and leaves the context
 *    unchanged.  efpi_last_error() then describes the failure.
 *  - Device-side conditions (Newton not converged, non-finite values,
 *    particle capacity exceeded, negative projected mass) set bits of a device
 *    status word; efpi_sync returns them.
 *  - A context is used from one host thread at a time.
 *
 * Particle store (structure of arrays, cell order after a lift): per ion an
 * int16 cell index c (-1 marks an absorbed ion), an FP32 offset frac in [0,1)
 * inside the cell (position x = (c + frac) h), an FP32 velocity and an FP32
 * weight.  Grid charge is accumulated as int64 fixed point in units of 2^-40,
 * so it is independent of summation order.
 */
#ifndef EFPI_H
#define EFPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EFPI_ABI_VERSION 2u

typedef enum {
  EFPI_OK = 0,
  EFPI_EINVAL = -1,    /* invalid argument or configuration                     */
  EFPI_ENOMEM = -2,    /* workspace smaller than efpi_workspace_size            */
  EFPI_EHIP = -3,      /* a HIP runtime call failed                             */
  EFPI_ENEWTON = -4,   /* Newton iteration did not reach its tolerance          */
  EFPI_ENUMERIC = -5,  /* non-finite value in potential or coarse state         */
  EFPI_ESTATE = -6,    /* call not valid in the current state                   */
  EFPI_EOVERFLOW = -7  /* particle capacity exceeded at load or lift            */
} efpi_status;

/* Device status bits returned by efpi_sync. */
#define EFPI_DEV_NEWTON 1u   /* max |Newton update| above newton_tol             */
#define EFPI_DEV_NAN 2u      /* non-finite potential or coarse value             */
#define EFPI_DEV_OVERFLOW 4u /* lift wanted more particles than capacity         */
#define EFPI_DEV_NEGMASS 8u  /* projected block mass below zero (clipped at lift) */
#define EFPI_DEV_WEIGHT 16u  /* an ion weight |w| (or snapshot moment |w V|, or
                                |w V^2| with EFPI_FLAG_PRESSURE) >= 16: the exact
                                per-lane sums of the particle pass need values
                                below 16                                         */

/* Boundary conditions and closures. */
#define EFPI_BC_PERIODIC 0
#define EFPI_BC_WALLS 1      /* absorbing walls, Neumann potential (phi' = 0)    */
#define EFPI_CLOSURE_BOLTZMANN 0 /* Newton solve of eq. 3.15                      */
#define EFPI_CLOSURE_KINETIC 1   /* kinetic electrons (particles, eq. 2.5) and the
                                    linear Poisson equation -phi'' = n_i - n_e
                                    (eq. 2.2); periodic only, n_cells <= 8192, and
                                    every replica of the context kinetic          */
#define EFPI_CLOSURE_NOFIELD 2   /* E = 0 (free streaming; test closure)          */

/* One replica (an independent plasma).  Ensembles pass several. */
typedef struct {
  int32_t n_cells;      /* N: power of two in [8, 16384]                          */
  int32_t bc;           /* EFPI_BC_*                                              */
  int32_t closure;      /* EFPI_CLOSURE_*                                         */
  int32_t ppc;          /* ions per occupied cell at load and lift, >= 1          */
  int32_t haar_levels;  /* l: coarse blocks of 2^l cells; N_c = N >> l, l <= log2 N */
  int32_t burst_steps;  /* N_e: fine steps per burst (Sec. 3.1), >= 1            */
  int32_t coevolving;   /* 1: restriction along approximate characteristics (App. B) */
  int32_t lift_linear;  /* 1: linear interpolation of block means at lift        */
  double length;        /* L, with h = L / N                                      */
  double vth;           /* thermal speed sqrt(T_i/T_e) of the lifted Maxwellian   */
  double dt;            /* fine step delta t > 0                                  */
  double macro_dt;      /* projective step Delta t >= N_e dt (eq. 3.17)           */
  double n_floor;       /* density below which a cell is empty at lift (> 0)     */
  int64_t capacity;     /* particle slots reserved for this replica               */
  /* kinetic electrons (EFPI_CLOSURE_KINETIC only; ignored otherwise).  Units are
   * the ions' (length lambda_D, time 1/omega_pi, potential T_e/e): with
   * mu = m_i/m_e the electrons have q/m = -mu, omega_pe = sqrt(mu) and thermal
   * speed sqrt(mu) at T_e0. */
  double qm_e;          /* electron charge-to-mass ratio, < 0 (-m_i/m_e)         */
  double vth_e;         /* electron thermal speed at loading, >= 0               */
  int32_t ppc_e;        /* electrons per occupied cell at loading, >= 1          */
  int32_t pad_e;        /* must be 0                                              */
  int64_t capacity_e;   /* electron slots reserved for this replica               */
} efpi_replica;

typedef struct {
  uint32_t abi_version;              /* EFPI_ABI_VERSION                          */
  uint32_t n_replicas;               /* R >= 1                                    */
  const efpi_replica* replicas;      /* host array of R replicas, copied at init  */
  int32_t newton_iters;              /* Newton iterations per fine step, >= 1     */
  int32_t newton_iters_start;        /* iterations after a load, lift or set      */
  double newton_tol;                 /* status threshold on max |last Newton update|;
                                        convergence is quadratic, so the remaining
                                        error is about its square                 */
  int32_t tile;                      /* particles per work item: 0 (default, 4096)
                                        or a multiple of 1024 up to 16384         */
  int32_t grid_blocks;               /* persistent grid size of the particle, lift
                                        and sort passes; 0 = one workgroup per
                                        work item                                 */
  uint32_t flags;                    /* EFPI_FLAG_*                               */
} efpi_config;

/* Reserve a second particle store so that efpi_sort can reorder out of place. */
#define EFPI_FLAG_SORT_BUFFER 1u
/* EFREE coarse variables (Sec. 3.2): three moments per replica instead of two.
 * Besides the density n and the momentum density j = nV, the coarse state carries
 * the second velocity moment s = nV^2 + P (P = nT, the ion pressure), restricted
 * along the co-evolving frame like the others (sum w V~^2 by CIC at X~).  The lift
 * loads each ion with the local thermal speed sqrt(T(X)), T = s/n - u^2 at the
 * fine nodes (clipped at 0, 0 below n_floor) linear in the cell, instead of vth,
 * and the block correction also stretches velocities about the block's mean so
 * that sum w v^2 meets the block's second moment.  Every coarse and snapshot
 * array of a context (efpi_lift, efpi_restrict, efpi_project, efpi_project2,
 * efpi_macro_step, efpi_macro_step_graph, efpi_restrict_state,
 * efpi_ensemble_mean) then holds three moments n, j, s where it reads [2]
 * below: [R][3][N_c] and [R][K+1][3][N_c].  The learned-projection calls keep
 * two.  Not with EFPI_CLOSURE_KINETIC. */
#define EFPI_FLAG_PRESSURE 2u

typedef struct efpi_ctx efpi_ctx; /* opaque host object owned by the library */

/* ---------------------------------------------------------------- set-up -- */

/* Bytes of device workspace the configuration needs (synchronous, host only). */
efpi_status efpi_workspace_size(const efpi_config* cfg, size_t* h_bytes);

/* Validate cfg, bind the caller's workspace (>= efpi_workspace_size bytes,
 * 256-byte aligned) and the caller's HIP stream (hipStream_t, may be NULL for
 * the null stream), clear the workspace on that stream and return a context in
 * *out.  The workspace must stay allocated until efpi_destroy. */
efpi_status efpi_init(const efpi_config* cfg, void* d_workspace, size_t bytes,
                      void* hip_stream, efpi_ctx** out);

/* Wait for the work the context queued on its stream, then release the host
 * context (the workspace stays the caller's and may be freed afterwards). */
void efpi_destroy(efpi_ctx* ctx);

/* Change the stream later calls enqueue on. */
efpi_status efpi_set_stream(efpi_ctx* ctx, void* hip_stream);

/* Number of Haar coarse coefficients per moment of replica r (host only). */
efpi_status efpi_n_coarse(efpi_ctx* ctx, int32_t replica, int32_t* h_nc);

/* ------------------------------------------------------- particle state -- */

/* Copy n particles (int16 cell, FP32 frac, v, w) into replica r.  v is at an
 * integer time level; the next burst starts the leapfrog from it.  Cells must
 * lie in [0, N) or be -1; frac in [0, 1).  n <= capacity. */
efpi_status efpi_set_particles(efpi_ctx* ctx, int32_t replica, const int16_t* d_cell,
                               const float* d_frac, const float* d_v, const float* d_w,
                               int64_t n);

/* Copy replica r's particles out (any pointer may be NULL).  Synchronous: waits
 * for the stream, then writes the particle count to *h_n.  Velocities are at
 * the half step after a burst and at the integer step after a load or lift. */
efpi_status efpi_get_particles(efpi_ctx* ctx, int32_t replica, int16_t* d_cell, float* d_frac,
                               float* d_v, float* d_w, int64_t* h_n);

/* Copy replica r's last deposited fixed-point charge (int64, N or N+1 nodes,
 * units 2^-40), potential (FP64) and node field (FP32).  Any pointer may be NULL. */
efpi_status efpi_get_grid(efpi_ctx* ctx, int32_t replica, int64_t* d_q, double* d_phi,
                          float* d_e);

/* Set replica r's potential (warm start of the next Newton solve).  Without it,
 * or a solve, the first field solve of a context after a load or lift starts cold
 * from phi = ln max(rho, 1e-8); once any replica's potential is set or solved,
 * burst starts are warm for every replica.  A cold first solve takes
 * max(newton_iters_start, 40) iterations. */
efpi_status efpi_set_potential(efpi_ctx* ctx, int32_t replica, const double* d_phi);

/* ------------------------------------------------------------- hot path -- */

/* Quiet-start load of replica r from fine node profiles of density d_n and mean
 * velocity d_u (FP64, N or N+1 nodes): App. C particle loading with uniform
 * in-cell offsets (m+1/2)/ppc, Maxwellian velocities by the inverse normal CDF at
 * the Hammersley coordinate b_i = ((bitrev32(c ppc + m) + shift) mod 2^32 + 1/2)/2^32,
 * and weights n(X) h / ppc.  Cells whose nodes are all below n_floor stay empty.
 * The thermal speed is the configured vth, also with EFPI_FLAG_PRESSURE. */
efpi_status efpi_load_profile(efpi_ctx* ctx, int32_t replica, const double* d_n,
                              const double* d_u, uint32_t shift);

/* Lifting operator (Sec. 3.3 "Lifting", App. C): for every replica, coarse
 * coefficients d_coarse[r][2][N_c] (density, momentum; FP64) -> fine profile by
 * inverse Haar (and linear interpolation of block means when lift_linear) ->
 * quiet-start ions as in efpi_load_profile with rotation h_shifts[r] -> per
 * coarse block, weights rescaled to the block mass and velocities shifted to
 * the block momentum.  With EFPI_FLAG_PRESSURE (d_coarse[r][3][N_c]) the thermal
 * speed is sqrt(T) of the fine temperature profile and velocities are also
 * stretched about the block mean to the block's second moment.  d_coarse must
 * stay valid until the work has run. */
efpi_status efpi_lift(efpi_ctx* ctx, const double* d_coarse, const uint32_t* h_shifts);

/* Deposit the fixed-point CIC charge of the current particles (Sec. 2.2): ion
 * charge, minus the electron charge in kinetic contexts (each electron deposits
 * -q_L, -q_R with the ions' fixed-point split). */
efpi_status efpi_deposit(efpi_ctx* ctx);

/* Solve -phi'' + exp(phi) = rho (eq. 3.15) by `iters` Newton iterations from the
 * current potential (cold != 0: from ln max(rho, 1e-8)), then set the node field
 * E_k = -(phi_{k+1} - phi_{k-1}) / 2h.  Requires a deposit since the last state change.
 * Kinetic contexts instead solve the periodic linear Poisson equation
 * -phi'' = rho - mean(rho) (eq. 2.2) exactly, with mean(phi) = 0 (iters and cold
 * are checked but not used). */
efpi_status efpi_solve_field(efpi_ctx* ctx, int32_t iters, int32_t cold);

/* ---------------------------------------------------- kinetic electrons -- */
/* Contexts whose replicas use EFPI_CLOSURE_KINETIC hold a second particle store
 * per replica for the electrons (same SoA layout as the ions).  Every burst
 * step pushes both species with the same field (electrons with q/m = qm_e,
 * time step dt) and deposits both charges; the field is the linear Poisson
 * solution.  Lifts (efpi_lift, efpi_macro_step, captured graphs) load the
 * electrons in Boltzmann equilibrium with the lifted ions, as
 * efpi_boltzmann_electrons.  All four calls return EFPI_ESTATE in contexts
 * without kinetic electrons. */

/* Copy n electrons into replica r's electron store (layout of efpi_set_particles;
 * n <= capacity_e).  Their velocities are taken at the current integer time level
 * (their next push is a half step); the ions are left as they are. */
efpi_status efpi_set_electrons(efpi_ctx* ctx, int32_t replica, const int16_t* d_cell,
                               const float* d_frac, const float* d_v, const float* d_w,
                               int64_t n);

/* Copy replica r's electrons out (as efpi_get_particles; synchronous). */
efpi_status efpi_get_electrons(efpi_ctx* ctx, int32_t replica, int16_t* d_cell, float* d_frac,
                               float* d_v, float* d_w, int64_t* h_n);

/* Quiet-start electrons of replica r from node profiles d_n (density) and d_u
 * (mean velocity), FP64, N nodes: the loading of efpi_load_profile (App. C) with
 * ppc_e electrons per occupied cell and thermal speed vth_e, rotation `shift`,
 * at the current time level (as efpi_set_electrons). */
efpi_status efpi_load_electrons(efpi_ctx* ctx, int32_t replica, const double* d_n,
                                const double* d_u, uint32_t shift);

/* Electrons in Boltzmann equilibrium with the current ions of every replica
 * (the passive electron variables of Sec. 3.3, eqs. 3.15-3.16): deposit the ion
 * charge, solve -phi'' + exp(phi) = n_i by newton_iters_start Newton iterations
 * from ln max(n_i, 1e-8), and load electrons with density exp(phi), mean velocity
 * the ions' fine velocity profile of their last lift or load, thermal speed
 * vth_e and Hammersley rotation h_shifts[r] XOR 0x9E3779B9.  The ions must be at
 * an integer time level (EFPI_ESTATE otherwise). */
efpi_status efpi_boltzmann_electrons(efpi_ctx* ctx, const uint32_t* h_shifts);

/* Reset the electrons of every replica to the Boltzmann equilibrium of the
 * current ions, at any point of a run (the control run of Sec. 4.1 that resets
 * the electrons periodically from the ion density): deposit the ion charge n_i
 * and the ion momentum with time-centred velocities (v + dt/2 E at the ions
 * after a burst), solve eq. 3.15 as efpi_boltzmann_electrons, and load
 * electrons with density exp(phi), mean velocity the ion node momentum over the
 * ion node charge (0 where the ion density is below n_floor), thermal speed
 * vth_e and rotation h_shifts[r] XOR 0x9E3779B9.  The ions are not changed; the
 * electrons start at the current time level (their next push is a half step).
 * After a burst the field must be current (it is after efpi_pic_burst). */
efpi_status efpi_reset_electrons(efpi_ctx* ctx, const uint32_t* h_shifts);

/* Fine burst on every replica: `steps` leapfrog steps (gather, push, boundary,
 * fixed-point deposit, Newton solve).  With restrict != 0 the burst starts by
 * storing the field E_n and restricts after every step: snapshots p = 0..steps
 * of the coarse (density, momentum) coefficients of the ions moved along the
 * approximate characteristics over Delta t - p dt (App. B, eq. B.4; plain
 * deposition when coevolving = 0).  steps <= burst_steps when restricting. */
efpi_status efpi_pic_burst(efpi_ctx* ctx, int32_t steps, int32_t restrict_);

/* Coarse snapshots of the last restricting burst: d_snap[r][p][2][N_c] (FP64)
 * for p = 0..steps, c_B = 2^{-l/2} (block mass) / h. */
efpi_status efpi_restrict(efpi_ctx* ctx, double* d_snap);

/* Least-squares slope of eq. 3.18 over the snapshots d_snap[r][0..N_e][2][N_c]
 * and forward-Euler projection over Delta t - N_e dt from the last snapshot
 * (eq. 3.17) -> d_coarse_next[r][2][N_c].  d_snap may be the output of
 * efpi_restrict; snapshots of every replica must hold burst_steps + 1 entries. */
efpi_status efpi_project(efpi_ctx* ctx, const double* d_snap, double* d_coarse_next);

/* Variable projective step: set Delta t of every replica to macro_dt (>= burst_steps
 * dt of each; EFPI_EINVAL otherwise, nothing changed).  Later bursts use it in the
 * co-evolving restriction (tau = Delta t - p dt, App. B) and later projections over
 * Delta t - N_e dt (eq. 3.17), eager or replayed from captured graphs.  Copies the
 * descriptors to the device on the context's stream and waits for the copy. */
efpi_status efpi_set_macro_dt(efpi_ctx* ctx, double macro_dt);

/* Step-size rule of the adaptive projective integrator (the paper's remark on
 * estimating the projection error, Sec. 3.1): err, the error of eq. 4.2 between the
 * second-order and the forward-Euler projections of the coarse density, estimates
 * the local error of a forward-Euler step, which grows as Delta t^2; so
 * *h_next = macro_dt * f with f = min(2, max(1/2, safety (tol / err)^{1/2})) (f = 2
 * when err = 0), then clamped to [dt_min, dt_max].  Host only and synchronous.
 * EFPI_EINVAL unless 0 < dt_min <= dt_max, macro_dt > 0, tol > 0, safety > 0,
 * err >= 0 (all finite) and h_next != NULL. */
efpi_status efpi_next_macro_dt(double macro_dt, double err, double tol, double dt_min,
                               double dt_max, double safety, double* h_next);

/* Second-order projective step (the higher-order projection the paper mentions
 * after eq. 3.17, read as Adams-Bashforth 2 on the burst slopes).  From the
 * snapshots d_snap[r][0..N_e][2][N_c] (as efpi_project):
 *   d_slope[r][2][N_c]   <- f, the LS slope of eq. 3.18 (keep it for the next step);
 *   d_euler[r][2][N_c]   <- c^{N_e} + (Delta t - N_e dt) f, eq. 3.17 (NULL: skipped;
 *                           the same bits as efpi_project);
 *   d_coarse_next[r][2][N_c] <- c^{N_e} + (Delta t - N_e dt) f*, with
 *     f* = f + (f - f_prev) Delta t / (2 gap)
 *   where f_prev = d_slope_prev (the previous step's d_slope) and gap the previous
 *   step's Delta t: f and f_prev estimate the derivative at the centres of two
 *   bursts gap apart, and f* extrapolates them to the middle of the projection leap.
 *   With d_slope_prev == NULL, f* = f (the forward-Euler step).  gap must be finite
 *   and > 0 when d_slope_prev is given. */
efpi_status efpi_project2(efpi_ctx* ctx, const double* d_snap, const double* d_slope_prev,
                          double gap, double* d_slope, double* d_euler, double* d_coarse_next);

/* One whole macro step for every replica: lift(d_coarse_in) -> restricting burst
 * of burst_steps -> restrict -> project -> d_coarse_out.  d_coarse_in and
 * d_coarse_out may alias.  The Newton solve after the lift starts from each
 * replica's current potential (newton_iters_start iterations, see
 * efpi_set_potential), so the result depends on that potential at the level of
 * the remaining Newton residual: equal inputs and equal potentials give equal
 * bits. */
efpi_status efpi_macro_step(efpi_ctx* ctx, const double* d_coarse_in, double* d_coarse_out,
                            const uint32_t* h_shifts);

/* efpi_macro_step replayed from a captured HIP graph.  The first call for a
 * given (d_coarse_in, d_coarse_out) pair and starting state captures the whole
 * macro step (lift, restricted burst, restriction, projection) on the
 * context's stream and instantiates it; later calls only upload the lift
 * rotations h_shifts and launch the graph, so the host enqueues two
 * operations per macro step instead of one per kernel.  Results are identical
 * to efpi_macro_step.  Needs a non-null stream and timing disabled
 * (EFPI_ESTATE otherwise).  A context keeps its 8 most recently captured
 * graphs (until efpi_destroy); the buffers they name must stay allocated while
 * they are used. */
efpi_status efpi_macro_step_graph(efpi_ctx* ctx, const double* d_coarse_in,
                                  double* d_coarse_out, const uint32_t* h_shifts);

/* ------------------------------------------------- phase-space restriction -- */
/* Phase-space coarse variables of the wavelet-based scheme (Sec. 3.3): the ion
 * distribution on nodes x_k (CIC) times 2^jf velocity bins over [v_min, v_max)
 * (nearest bin; ions outside are not counted), l = levels steps of the
 * full-weighting restriction in x (eq. 3.8), then per coarse x node the
 * periodized discrete wavelet transform of the velocity column down to 2^jc
 * scaling coefficients (App. A) with the caller's orthonormal low-pass filter
 * (for the paper's scheme, the 12-tap order-4 Coiflet). */
typedef struct {
  double v_min, v_max;   /* velocity window                                          */
  int32_t jf;            /* 2^jf fine velocity bins, 4 <= jf <= 11                    */
  int32_t jc;            /* 2^jc coarse coefficients per x node, jc <= jf, 2^jc >= n_taps */
  int32_t levels;        /* full-weighting levels in x, n_cells >> levels >= 1, and
                            h 4^levels < 2^18 (the int64 histogram holds node
                            densities up to 16 n_0 at that bound)                   */
  int32_t n_taps;        /* filter length, even, 2 <= n_taps <= 16                    */
  double taps[16];       /* low-pass filter h_0..h_{n_taps-1} (host copy)            */
} efpi_phase;

/* Order-2K Coiflet low-pass filter for efpi_phase (App. A: the wavelet has
 * vanishing moments 0 .. 2K-1 and the scaling function vanishing moments
 * 1 .. 2K-1 about the origin of its support [-2K, 4K-1], i.e. about tap 2K).
 * n_taps = 6K: 12 for the paper's order-4 filter, or 6.  Among the isolated
 * solutions of those conditions, the one most nearly symmetric about tap 2K is
 * returned.  Host only and synchronous (no context, no device work); writes
 * h_taps[n_taps] (sum sqrt 2, orthonormal even shifts).  EFPI_EINVAL for another
 * n_taps or a NULL pointer, EFPI_ENUMERIC if the solver finds no filter. */
efpi_status efpi_coiflet_taps(int32_t n_taps, double* h_taps);

/* Bytes of the caller-owned work buffer of efpi_phase_restrict for replica r:
 * the int64 intermediate histogram [n_cells >> levels][2^jf]. */
efpi_status efpi_phase_work_size(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                 size_t* h_bytes);

/* Phase-space coarse coefficients of replica r's current ions:
 * d_out[n_cells >> levels][2^jc] (FP64).  Each ion enters at X + tau v,
 * V = v + tau E(X) (the co-evolving frame of App. B with the current field; tau = 0:
 * plain), with time-centred velocities after a burst (v + dt/2 E).  Its charge is
 * quantised as in the deposit, q = rint(w 2^40) split rint(theta q) / rest over the
 * two nodes of X, and node i = 2^l K + d adds (2^l - d) and d times its share to
 * coarse nodes K and K + 1 (the composed full-weighting weights, denominator 4^l):
 * the histogram d_work[K][k_v] is exact int64 and order-free.  The column values
 * are H 2^-40 / (4^l h dv) (a phase-space density) times 2^{-jf/2} (v_max - v_min)
 * (App. A's finest scaling coefficients of the velocity rescaled to [0, 1)), then
 * jf - jc levels a_k = sum_m h_m x_{(2k + m) mod N}.  d_work: efpi_phase_work_size
 * bytes, 256-byte aligned.  EFPI_EINVAL on bad parameters. */
efpi_status efpi_phase_restrict(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                double tau, int32_t stored_field, void* d_work, double* d_out);

/* Size of the static scratch of efpi_phase_restrict_static (per GPU). */
#define EFPI_STATIC_SCRATCH_BYTES ((size_t)8 << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): efpi_phase_restrict
 * with its int64 histogram in a static device array of EFPI_STATIC_SCRATCH_BYTES
 * that the library's code object holds on each GPU until the process ends,
 * instead of a caller work buffer.  Same arguments, checks, kernels and results
 * as efpi_phase_restrict; allocates nothing.  The array's address on a device is
 * looked up at the first efpi_init with that device current; the context's
 * stream must belong to that device.  EFPI_EINVAL when the histogram
 * (efpi_phase_work_size bytes) exceeds EFPI_STATIC_SCRATCH_BYTES.  Every call on
 * one GPU uses the same array: each call clears the histogram before use, and
 * calls that can overlap on one GPU (other streams, other threads) race. */
efpi_status efpi_phase_restrict_static(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                       double tau, int32_t stored_field, double* d_out);

/* Bytes of the caller-owned work buffer of efpi_phase_lift for replica r: the
 * refined columns [n_cells >> levels][2^jf] and the repaired CDFs
 * [n_cells][2^jf + 1] (FP64). */
efpi_status efpi_phase_lift_work_size(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                      size_t* h_bytes);

/* Lifting from phase-space coefficients d_coarse[n_cells >> levels][2^jc] (App. C):
 * each column back to 2^jf values with zero details (inverse of the transform
 * above) and scaled to the phase-space density, l levels of midpoint interpolation
 * in x (eq. 3.7), per fine node the density n = (sum f) dv and the conditional CDF
 * at the bin edges (sums in index order), the CDF repair of App. C (edges below 0
 * and, reflected, above 1; interior ramps from the lower indexes and, reflected,
 * from the upper ones, averaged; a ramp is accepted when its last value stays at
 * or below F[k+]; where none fits below F[n] a straight line joins F[k-] to F[n]);
 * then ppc ions per occupied cell (a node density above n_floor) at offsets
 * (m + 1/2)/ppc with velocity the two nodes' inverse CDFs (lookup, linear within
 * the bin) at the Hammersley b with rotation `shift`, interpolated in x, and weight
 * n(X) h / ppc.  Kinetic electrons are left as they are: efpi_reset_electrons
 * then loads them in Boltzmann equilibrium with the lifted ions.  d_work:
 * efpi_phase_lift_work_size bytes, 256-byte aligned. */
efpi_status efpi_phase_lift(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                            const double* d_coarse, uint32_t shift, void* d_work);

/* Least-squares slope (eq. 3.18) of `snapshots` equally spaced (dt) snapshots
 * d_snap[snapshots][count] and forward-Euler projection over
 * macro_dt - (snapshots - 1) dt from the last one (eq. 3.17) -> d_out[count]. */
efpi_status efpi_phase_project(efpi_ctx* ctx, const double* d_snap, int64_t count,
                               int32_t snapshots, double dt, double macro_dt, double* d_out);

/* Make the field current (deposit and solve if needed) and store it as E_n, the
 * field of the burst start that the co-evolving frame uses (App. B); clears the
 * Haar snapshot bins. */
efpi_status efpi_store_field(efpi_ctx* ctx);

/* Plain restriction (no co-evolving frame) of the current particles of every
 * replica: d_coarse[r][2][N_c] = coarse (density, momentum) coefficients at the
 * current time, with time-centred velocities after a burst.  Overwrites the
 * snapshots of the last burst. */
efpi_status efpi_restrict_state(efpi_ctx* ctx, double* d_coarse);

/* Replace every replica's coarse state in d_coarse[r][2][N_c] by the mean over
 * the replicas with the same n_cells and length (replica-index order). */
efpi_status efpi_ensemble_mean(efpi_ctx* ctx, double* d_coarse);

/* Stable per-tile counting sort of every replica's particles by cell; absorbed
 * ions (cell -1) are dropped.  Needs EFPI_FLAG_SORT_BUFFER. */
efpi_status efpi_sort(efpi_ctx* ctx);

/* ------------------------------------------------- learned projection -- */
/*
 * A small network replaces the least-squares slope (eq. 3.18) in the
 * projective step (eq. 3.17) on macro steps that skip the fine burst:
 *   x = features(c_{n-2}, c_{n-1}, c_n),  y = net(x),  c_{n+1} = c_n + delta * y.
 * Features, per moment m (0 density, 1 momentum) and coarse index k:
 *   x[m]   = (c_n - mu_m) / sigma_m,
 *   x[2+m] = (c_n - c_{n-1}) / delta_m,   x[4+m] = (c_{n-1} - c_{n-2}) / delta_m.
 * Network: 1D convolutions over k, widths 6 -> 64 -> 64 -> 64 -> 2, kernel 3,
 * SiLU after the first three, circular padding (periodic) or zero padding
 * (walls).  Parameters: one FP32 vector of EFPI_NN_PARAMS values, per layer
 * W[c_out][c_in][3] followed by b[c_out].  The matrix cores take bfloat16
 * weights and activations with FP32 accumulation; efpi_nn_pack and
 * efpi_nn_adam keep the bfloat16 weight pack (EFPI_NN_PACK_BYTES, 16-byte
 * aligned, caller-owned) in step with the FP32 parameters.  Activations are
 * FP32 [batch][channel][n_c].  These calls take the HIP stream directly and
 * need no context; none allocates memory.
 */
#define EFPI_NN_CIN 6
#define EFPI_NN_HIDDEN 64
#define EFPI_NN_COUT 2
#define EFPI_NN_PARAMS 26306
#define EFPI_NN_PACK_BYTES 112640

typedef struct {
  float mu[2];     /* feature shift of c_n per moment                          */
  float sigma[2];  /* feature scale of c_n per moment                          */
  float delta[2];  /* scale of the increments (inputs 2..5 and the output)     */
} efpi_nn_norm;

/* Bytes of device workspace (activations, gradient partials) for `batch`
 * samples of n_c coarse points (host only). */
efpi_status efpi_nn_workspace_size(int32_t batch, int32_t n_c, size_t* h_bytes);

/* Write the bfloat16 weight pack from FP32 parameters. */
efpi_status efpi_nn_pack(const float* d_params, void* d_pack, void* hip_stream);

/* Forward pass: d_y[batch][2][n_c] = net(d_x[batch][6][n_c]).  Keeps the layer
 * activations in d_ws for a following efpi_nn_backward of the same batch. */
efpi_status efpi_nn_forward(const float* d_params, const void* d_pack, const float* d_x,
                            float* d_y, int32_t batch, int32_t n_c, int32_t periodic, void* d_ws,
                            size_t ws_bytes, void* hip_stream);

/* Backward pass of the last forward on d_ws: d_grad[EFPI_NN_PARAMS] = gradient
 * of sum(d_dy * y).  Summation order is fixed, so the result is deterministic. */
efpi_status efpi_nn_backward(const void* d_pack, const float* d_x, const float* d_dy,
                             float* d_grad, int32_t batch, int32_t n_c, int32_t periodic,
                             void* d_ws, size_t ws_bytes, void* hip_stream);

/* Mean squared error over `count` values: *d_loss = mean((y - t)^2) and
 * d_dy = 2 (y - t) / count (FP32; one workgroup, fixed order). */
efpi_status efpi_nn_mse(const float* d_y, const float* d_t, float* d_dy, float* d_loss,
                        int64_t count, void* hip_stream);

/* One Adam step (Kingma & Ba 2015; `step` counts from 1) on the FP32
 * parameters with moments d_m, d_v, then refresh the bfloat16 pack. */
efpi_status efpi_nn_adam(float* d_params, const float* d_grad, float* d_m, float* d_v,
                         int32_t step, float lr, float beta1, float beta2, float eps,
                         void* d_pack, void* hip_stream);

/* Features of `batch` samples from a state sequence d_states[n_states][2][n_c]
 * (FP64): sample b uses states n-2, n-1, n with n = d_index[b] (device int32,
 * clamped to [2, n_states - 1], or to [2, n_states - 2] when d_t is given).
 * Writes d_x[batch][6][n_c] and, when d_t is not NULL, the training target
 * d_t[batch][2][n_c] = (c_{n+1} - c_n) / delta.  With noise > 0 (training), the
 * three input states are first perturbed by noise * delta_m times a unit-
 * variance uniform variate (counter-based hash of seed and element), and the
 * target is taken from the perturbed c_n, so the network learns to steer back
 * toward the trajectory; noise = 0 gives the exact features. */
efpi_status efpi_nn_features(const double* d_states, int32_t n_states, const int32_t* d_index,
                             int32_t batch, int32_t n_c, const efpi_nn_norm* h_norm, float noise,
                             uint32_t seed, float* d_x, float* d_t, void* hip_stream);

/* Learned projective step: d_c_next = d_c_n + delta * d_y, all [batch][2][n_c]
 * (states FP64, d_y FP32).  d_c_next may alias d_c_n. */
efpi_status efpi_nn_step(const double* d_c_n, const float* d_y, int32_t batch, int32_t n_c,
                         const efpi_nn_norm* h_norm, double* d_c_next, void* hip_stream);

/* One learned projective step in one call: features of the three consecutive
 * states d_states[3][2][n_c] (c_{n-2}, c_{n-1}, c_n; FP64), forward pass, and
 * d_c_next[2][n_c] = c_n + delta * y, except outside the plasma's support: a
 * block whose density in c_n is exactly zero at itself and at every block within
 * two blocks (wrapping when periodic, only blocks inside the walls otherwise)
 * keeps c_n (both moments), as a plain EFPI step leaves empty blocks empty.
 * d_ws holds at least efpi_nn_workspace_size(1, n_c) bytes; d_c_next must not
 * overlap d_states. */
efpi_status efpi_nn_predict_step(const float* d_params, const void* d_pack,
                                 const double* d_states, int32_t n_c, int32_t periodic,
                                 const efpi_nn_norm* h_norm, double* d_c_next, void* d_ws,
                                 size_t ws_bytes, void* hip_stream);

/* Relative error of eq. 4.2 between two FP64 arrays of n values:
 * *d_eps = sqrt(sum (a - b)^2 / sum (a^2 + b^2)) (0 when both are zero), FP64,
 * one workgroup with a fixed summation order.  The learned projection's judge
 * compares a learned step with a fine-burst step by it. */
efpi_status efpi_rel_l2(const double* d_a, const double* d_b, int64_t n, double* d_eps,
                        void* hip_stream);

/* ---------------------------------------------------------------- status -- */

/* Wait for the stream, return the device status bits in *h_bits (may be NULL)
 * and clear them.  Returns EFPI_ENUMERIC / EFPI_ENEWTON / EFPI_EOVERFLOW when the
 * matching bit was set (first in that order), else EFPI_OK. */
efpi_status efpi_sync(efpi_ctx* ctx, uint32_t* h_bits);

/* Measurement aid: with enable != 0, every later burst-step particle launch (the
 * pass that pushes, deposits and restricts) is bracketed by a pair of HIP events
 * (extended launch), and efpi_timing_read returns their summed intervals.  The
 * events are created without the system-scope fence (timing only: recording
 * them writes back no caches).  Each interval also holds the processing of the
 * two event markers around the dispatch, a few microseconds more than the
 * kernel's execution as a kernel trace reports it.  Enabling resets the record. */
efpi_status efpi_timing(efpi_ctx* ctx, int32_t enable);

/* Synchronous: wait for the stream, then return the summed event time in ms and
 * the number of timed launches since the last read or enable, and reset them. */
efpi_status efpi_timing_read(efpi_ctx* ctx, double* h_total_ms, int64_t* h_launches);

/* As efpi_timing_read for the electron pass of kinetic contexts: with timing
 * enabled every burst-step electron launch (push and deposit) is bracketed by
 * its own pair of events as well.  EFPI_ESTATE without kinetic electrons. */
efpi_status efpi_timing_read_electrons(efpi_ctx* ctx, double* h_total_ms, int64_t* h_launches);

/* Message for the last failed call on this thread ("" when none). */
const char* efpi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EFPI_H */
