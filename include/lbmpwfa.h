/*
 * lbmpwfa.h -- C ABI of the MI355X lattice-Boltzmann plasma-wakefield step.
 *
 * The library advances the plasma-electron fluid of G. Parise et al., "Lattice Boltzmann
 * simulations of Plasma Wakefield Acceleration" (arXiv:2201.05473) on an axisymmetric (z, r)
 * grid: three D2Q9 lattices for A = (n, n p_z, n p_r) (Sec. III, Eqs. (6)-(14); BGK collision, or
 * one of the operators of lbm_config.collision) coupled to Maxwell's equations on a Yee grid
 * (Sec. II, Eq. (5)), driven by a rigid bi-Gaussian electron bunch moving at c or by a
 * macroparticle bunch, on a window that moves with the driver (Sec. II, last paragraph).
 *
 * Units are normalised plasma units: t omega_p, x k_p, n / n_0, p / (m_e c),
 * e E / (m_e c omega_p), e B / (m_e omega_p), c = 1.
 *
 * Grid and layout.  Fluid sites (i, j), i in [0, nz) along z, j in [0, nr) along r, at
 * z_i = (s + i) dz (s = window shift count) and r_j = (j + 1/2) dr.  E_z lives at (z_i + dz/2, r_j),
 * E_r at (z_i, (j + 1) dr), B_theta at (z_i + dz/2, (j + 1) dr).  Every array that crosses this
 * ABI is row-major [component][nr][nz] with z fastest and no padding.
 *
 * Memory and streams.  The caller owns every buffer: one device workspace of at least
 * lbm_workspace_bytes() bytes (the library never allocates device memory), the HIP stream
 * (hipStream_t passed as void*, NULL = default stream), and all output buffers.  Calls are
 * stream-ordered; only calls that return data to host memory synchronise the stream.
 *
 * Errors.  Every call returns LBM_OK or a negative LBM_E* code and records a message readable
 * with lbm_last_error() on the same thread.  No call throws across the ABI.  A context is
 * used by one host thread at a time.
 */
#ifndef LBMPWFA_H
#define LBMPWFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid configuration or argument */
  LBM_ENOMEM = -2,    /* workspace smaller than required */
  LBM_EHIP = -3,      /* a HIP runtime call failed */
  LBM_EUNSTABLE = -4, /* a stability check found a non-finite value */
  LBM_ESTATE = -5     /* call out of order (e.g. NULL or destroyed context) */
};

/* Storage precision of the populations.  F64: populations, fields and arithmetic in FP64.
 * F32: populations and fields in FP32, FP32 arithmetic; E_r and B_theta carry a bfloat16
 * residual each (one more 32-bit plane), so that the field update accumulates without an FP32
 * rounding per step (compensated fields: the FP32 rounding of the large driver fields would
 * otherwise set the E_z error near 1e-5).  F16: populations in FP16, fields and
 * arithmetic in FP32.  The density lattice is stored as the deviation from the rest equilibrium
 * w_i n_bg(z); diagnostics are always accumulated in FP64.  F16N: as F16, but each population
 * is stored as its part off the equilibrium (Eq. (9)) of the moments stored at its own site,
 * which are FP32: the same bytes as F16 with about a tenth of its error, for more arithmetic per
 * step.  The adjoint (lbm_adjoint, lbm_vjp_*) takes every storage (with fp64_math = 1 on F32,
 * F16 and F16N for the BGK collision only). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_F16N = 3 };

/* Collision operator of the three lattices.  The paper uses BGK (Eq. (7)) and notes (Sec. IV)
 * that BGK is the simplest choice and that other collision operators may stabilise the
 * non-linear regime.  Three are offered, each relaxing toward the equilibrium of Eq. (9), with
 * the source of Eq. (10) added unchanged:
 *   LBM_BGK  Eq. (7): one relaxation time tau for every population.
 *   LBM_TRT  two relaxation times: the part of f - f_eq that is even under xi -> -xi (pairs of
 *            opposite directions) relaxes with tau_plus, the odd part with tau.
 *   LBM_REG  regularised BGK: before relaxing with tau, f - f_eq is replaced by its projection
 *            on the first-order Hermite polynomials, w_i xi_i . j_neq / c_s^2 with
 *            j_neq = sum_i xi_i (f_i - f_eq_i); every non-equilibrium moment above the first is
 *            dropped.
 *   LBM_MRT  multiple relaxation times: f - f_eq is expanded in the nine orthogonal moments of
 *            D2Q9 (the polynomials 1, 3|xi|^2 - 4, (9|xi|^4 - 21|xi|^2 + 8)/2, xi_z,
 *            (3|xi|^2 - 5) xi_z, xi_r, (3|xi|^2 - 5) xi_r, xi_z^2 - xi_r^2, xi_z xi_r of the
 *            velocities) and each relaxes with its own rate: the fluxes xi_z, xi_r with 1/tau,
 *            the energy, energy square, heat fluxes and stresses with mrt_se, mrt_seps,
 *            mrt_sq, mrt_spi. */
enum { LBM_BGK = 0, LBM_TRT = 1, LBM_REG = 2, LBM_MRT = 3 };

/* Driver of the wake.  The paper drives the plasma with the electron bunch of its hybrid code:
 * macroparticles moved by the Lorentz force (Sec. II, Eq. (1)) whose current, projected on the
 * grid, enters Ampere's law.
 *   LBM_DRIVER_RIGID      a rigid bi-Gaussian bunch at c (its current and initial field are
 *                         closed forms);
 *   LBM_DRIVER_PARTICLES  macroparticles.  Each step moves them by dt p / gamma, projects their
 *                         current w beta at the midpoints (linear in z onto the field points,
 *                         linear in r between rows; the share below the axis folds onto row 0
 *                         for densities and J_z, and is dropped for J_r, which vanishes there) as
 *                         J_b(t_{k-1/2}) of Ampere's law (z and r components), and after the fields
 *                         and the fluid pushes the momenta with the Boris scheme in E^k and
 *                         B^k = (B^{k-1/2} + B^{k+1/2}) / 2 interpolated with the same weights.
 *                         A particle whose stencil leaves columns [1, nz - 2] or the rows is lost
 *                         (its weight set to zero, no longer moved).  Deposition uses atomic
 *                         additions, so sums over particles are not ordered: results agree with an
 *                         ordered sum to round-off, not bit for bit. */
enum { LBM_DRIVER_RIGID = 0, LBM_DRIVER_PARTICLES = 1 };

/* Run configuration.  Physical meaning (normalised units):
 *   nz, nr        grid size: both >= 3, nr <= 65535, nz nr <= 2^26 sites
 *   dz, dr        cell size; must be equal (the D2Q9 lattice is square)
 *   c_dt_over_dz  c dt / dz, in (0, 1/sqrt(3)); keeps the lattice velocity below c_s and the
 *                 Yee scheme stable.  With moving_window it must be 1/m for an integer m
 *   tau           BGK relaxation time in lattice units, > 1/2; D = (tau - 1/2)/3 dz^2/dt (Eq. (12))
 *   storage       LBM_F64, LBM_F32, LBM_F16 or LBM_F16N
 *   moving_window 1: shift the window one cell every m = 1/(c dt/dz) steps
 *   periodic      bit 0: periodic in z (excludes moving_window); bit 1: periodic in r
 *                 (requires fields_on = 0 and cyl_on = 0)
 *   fields_on     1: Maxwell update and Lorentz force; 0: fields stay zero
 *   cyl_on        1: axisymmetric source terms of Eq. (13)
 *   n0, ramp_kind, ramp_start, ramp_len
 *                 background density n_bg(z): 0 uniform n0; 1 linear n0 clamp((z-z_p)/L, 0, 1);
 *                 2 tanh n0 (1 + tanh(2 (z-z_p)/L - 1)) / 2; z_p = ramp_start, L = ramp_len > 0
 *   nb, sigma_z, sigma_r, zd0
 *                 driver density n_b exp(-(z - zd0 - t)^2 / 2 sigma_z^2 - r^2 / 2 sigma_r^2)
 *   n_floor       densities at or below it carry no momentum, current or force
 *   check_every   > 0: every that many steps lbm_step synchronises and checks for non-finite
 *                 values (LBM_EUNSTABLE); 0: no checks
 *   fp64_math     1: FP64 arithmetic in the step for FP32 / FP16 storage (storage unchanged);
 *                 0: arithmetic in FP32.  Ignored for LBM_F64 (always FP64).
 *   collision     LBM_BGK, LBM_TRT, LBM_REG or LBM_MRT (above).  All four conserve A + dt F and
 *                 relax the first moment with 1/tau, so D of Eq. (12) is the same for all four
 *   trt_magic     LBM_TRT only: Lambda = (tau_plus - 1/2)(tau - 1/2) > 0, which fixes the
 *                 relaxation time tau_plus of the symmetric part; Lambda = (tau - 1/2)^2 is BGK.
 *                 Ignored otherwise.
 *   driver        LBM_DRIVER_RIGID (nb, sigma_z, sigma_r, zd0 above) or LBM_DRIVER_PARTICLES
 *                 (a macroparticle bunch set with lbm_set_bunch; nb .. zd0 are then unused)
 *   max_particles LBM_DRIVER_PARTICLES: capacity of the bunch, in [0, 2^31); the workspace holds
 *                 128 bytes per particle (the 7 doubles twice, since a re-sort moves the bunch to
 *                 a second buffer, the caller's index of each stored particle twice, and the
 *                 re-sort's key and rank) besides the per-grid buffers of the driver (two J_b plane
 *                 pairs, a density plane, the re-sort's count per cell).  Ignored otherwise.
 *   mrt_se, mrt_seps, mrt_sq, mrt_spi
 *                 LBM_MRT only: relaxation rates (1 / relaxation time) of the energy, energy
 *                 square, heat-flux and stress moments, each in (0, 2); all four 1/tau is BGK,
 *                 mrt_se = mrt_seps = mrt_spi = 1/tau_plus with mrt_sq = 1/tau is TRT.  Ignored
 *                 otherwise.
 *   resort_every  LBM_DRIVER_PARTICLES: every that many steps lbm_step re-sorts the stored bunch
 *                 on the device by grid cell (column, then row), so that the particles of a
 *                 wavefront stay close together as the bunch disperses; 0 is 500, negative
 *                 values are rejected.  The caller's order is kept (lbm_get_bunch).  Ignored
 *                 otherwise.
 *   bunch_streaming
 *                 LBM_DRIVER_PARTICLES: 1 = the push and move read and write the bunch with
 *                 non-temporal accesses, which leave the GPU's caches to the step's own data.
 *                 That pays on a grid whose step traffic is about the size of the last-level
 *                 cache (256 MB): 2400 x 400 in FP32 (261 MB per step) goes from 68.7 to 62.8 us
 *                 per step with 200,000 particles; on a larger one it costs, since the bunch then
 *                 comes from HBM (2048 x 512: 70.6 against 73.2 us).  0 = cached accesses.  Only 0
 *                 and 1 are accepted.  Results are the same either way.  Ignored otherwise. */
typedef struct {
  int32_t nz, nr;
  double dz, dr, c_dt_over_dz, tau;
  int32_t storage;
  int32_t moving_window, periodic, fields_on, cyl_on;
  double n0;
  int32_t ramp_kind;
  double ramp_start, ramp_len;
  double nb, sigma_z, sigma_r, zd0;
  double n_floor;
  int32_t check_every;
  int32_t fp64_math;
  int32_t collision;
  double trt_magic;
  int32_t driver;
  int64_t max_particles;
  double mrt_se, mrt_seps, mrt_sq, mrt_spi;
  int32_t resort_every;
  int32_t bunch_streaming;
} lbm_config;

/* FP64 diagnostics of the current state (all sums over the window):
 *   charge        sum 2 pi r_j dz dr n          (electron number in the window)
 *   field_energy  1/2 sum 2 pi dz dr (r E_z^2 + r_edge E_r^2 + r_edge B^2)
 *   gauss_max     max over sites with i >= 1 of |div_h E - (n_bg - n - n_b)|
 *   umax          max lattice speed |u*| = (c dt/dz) |beta|
 *   nonfinite     number of non-finite values among the moments and fields */
typedef struct {
  double charge, field_energy, gauss_max, umax;
  int64_t step, shifts;
  int32_t nonfinite, reserved;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Device workspace needed by a configuration (bytes).  LBM_EINVAL for an invalid config. */
int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes);

/* Create a context and set the initial state (Sec. II/III set-up; the seeded density
 * perturbation is an input, and the initial field is the driver's discrete Gauss field):
 * populations at the local equilibrium of density n_bg(z_i) (1 + n_pert[j][i]) and momentum
 * p_init[c][j][i] (c = 0: p_z, 1: p_r); E_z = 0; E_r and B_theta = the driver's discrete Gauss
 * field at t = -dt and t = -dt/2.  n_pert (host, [nr][nz]) and p_init (host, [2][nr][nz]) may
 * be NULL (zero).  workspace: device pointer, 256-byte aligned, ws_bytes >= lbm_workspace_bytes.
 * The workspace must stay valid until lbm_destroy.  Synchronises the stream. */
int lbm_init(const lbm_config* cfg, const double* n_pert, const double* p_init,
             void* workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Advance nsteps >= 0 steps.  One step (Eqs. (5)-(10), (13), (14)): Ampere with the previous
 * step's post-kick current and the driver current, Faraday, pull-stream of the 27 populations,
 * moments, Lorentz and axisymmetric sources, collision (cfg.collision), window shift when due.  Stream-
 * ordered and asynchronous, except that it synchronises the stream at each diagnostic check
 * (cfg.check_every > 0) and, with LBM_DRIVER_PARTICLES and particles in the bunch, at each re-sort
 * (every cfg.resort_every steps), which reads back the bunch's extent. */
int lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Moments of the last step's post-collision state, [3][nr][nz]: n, J_z = n beta_z,
 * J_r = n beta_r.  n is the zeroth moment of the density lattice (Eq. (8)) after the source of the
 * step (A* = A + dt F); J = n beta is the electron current density J_e of Eq. (5), with
 * beta = p / gamma from the zeroth moments of the momentum lattices (Eq. (2); zero at or below
 * n_floor).  dtype LBM_F64 or LBM_F32.  dst on the device (stream-ordered) or on the host
 * (synchronising).  LBM_EINVAL for a NULL dst or another dtype. */
int lbm_moments(lbm_ctx* ctx, void* dst, int32_t dtype, int32_t dst_on_device);

/* Fields of the state, [3][nr][nz]: the E_z, E_r, B_theta of Maxwell's equations (Eq. (5)) on
 * the radially half-shifted Yee grid (the paper names an FDTD/Yee scheme without its layout):
 * E_z at (z_i + dz/2, r_j), E_r at (z_i, (j + 1) dr), B_theta at (z_i + dz/2, (j + 1) dr); E at
 * t_{k-1} and B_theta at t_{k-1/2} after k steps (LBM_F32 storage: each with its residual
 * added, in FP64).  dtype and placement as lbm_moments. */
int lbm_fields(lbm_ctx* ctx, void* dst, int32_t dtype, int32_t dst_on_device);

/* Full state in FP64 on the host: [27][nr][nz] populations (lattice-major, raw values, not
 * deviations), [3][nr][nz] post-collision moments, [3][nr][nz] E_z, E_r, B_theta; the step and
 * shift counters go to *step and *shifts (may be NULL).  dst holds 33 nr nz doubles.
 * Synchronising.  Used for checkpoints and checks. */
int lbm_get_state(lbm_ctx* ctx, double* dst, int64_t* step, int64_t* shifts);

/* Restore a state written by lbm_get_state (same layout, host memory) together with its step
 * and shift counters.  Values are rounded to the storage precision.  Synchronising. */
int lbm_set_state(lbm_ctx* ctx, const double* src, int64_t step, int64_t shifts);

/* Checkpoint in the native storage format, for exact resume:
 * a 64-byte header (magic, storage, nz, nr, row pitch, step, shift count, plane stride, driver,
 * particle count) followed by the active population, moment and field buffers as stored (with
 * LBM_F32 the field buffer includes the plane of residuals).  With LBM_DRIVER_PARTICLES a bunch
 * section follows: the extent that bounds the J_b region and its age in steps (24 bytes), the 7
 * coordinate arrays of the bunch in its stored order (FP64) and each particle's index in the
 * caller's order (int32).  lbm_checkpoint_bytes gives the size of the context's checkpoint, which
 * depends on the number of particles (it changes only with lbm_set_bunch and lbm_load).
 * dst/src may be host or device memory (flag); both calls synchronise the stream.  lbm_load
 * returns LBM_EINVAL, and leaves the context as it was, if the checkpoint was written for another
 * grid, storage precision or driver, holds more than max_particles particles or an index array
 * that is not a permutation.  It replaces the bunch and clears the J_b buffers.  A rigid-driver run
 * resumes bit for bit; a particle-driven one to round-off (the deposit adds in no fixed order). */
int lbm_checkpoint_bytes(lbm_ctx* ctx, size_t* bytes);
int lbm_save(lbm_ctx* ctx, void* dst, int32_t dst_on_device);
int lbm_load(lbm_ctx* ctx, const void* src, int32_t src_on_device);

/* ---------------------------------------------------------------------------------------------
 * Adjoint (differentiation of the step; not part of the paper's method).
 *
 * theta = (ramp_len, n0, sigma_r, nb).  The objective J is the witness field: E_z of the state
 * on row obj->row, linearly interpolated in z at z_d(t_{N-1}) - obj->z_behind after N steps
 * (the time level of E in the state).  On the device the adjoint computes and stores its
 * variables in the precision of the auxiliary planes (FP64 for LBM_F64, FP32 for LBM_F32,
 * LBM_F16 and LBM_F16N), reads the forward states in their storage precision, and sums the theta
 * partials in FP64; J and grad are FP64.  With LBM_F16N the state it differentiates is the state
 * view of lbm_get_state (the populations, not their stored parts off the equilibrium).  Host-side
 * adjoint arrays are FP64 in the layout of lbm_get_state: [27][nr][nz] populations,
 * [3][nr][nz] moments, [3][nr][nz] E_z, E_r, B_theta.  Every collision operator is covered:
 * each writes the post-collision populations as P f + (I - P) f_eq + w_i dt F with a fixed linear
 * map P of the pulled populations f (BGK: (1 - 1/tau) I), and the adjoint applies P^T.
 * ------------------------------------------------------------------------------------------- */
typedef struct { double z_behind; int32_t row; } lbm_objective;

/* Device scratch of lbm_vjp_step / lbm_vjp_init (bytes). */
int lbm_vjp_workspace_bytes(const lbm_config* cfg, size_t* bytes);

/* Vector-Jacobian product of one step at the current state x^k: lam_out = (dPhi/dx^k)^T lam_next
 * and grad[4] = (dPhi/dtheta)^T lam_next, where x^{k+1} = Phi(x^k; theta) is the next step.
 * lam_next and lam_out are host arrays in the lbm_get_state layout.  The state is unchanged.
 * Periodic dimensions need at least 5 cells.  Synchronising. */
int lbm_vjp_step(lbm_ctx* ctx, void* adj_ws, size_t adj_bytes, const double* lam_next,
                 double* lam_out, double grad[4]);

/* theta partials of the initial state: grad[4] = (dx^0/dtheta)^T lam0.  The context must hold
 * its initial state (step 0).  Synchronising. */
int lbm_vjp_init(lbm_ctx* ctx, void* adj_ws, size_t adj_bytes, const double* lam0, double grad[4]);

/* Device workspace of lbm_adjoint for nsteps steps with a checkpoint every ckpt_every steps. */
int lbm_adjoint_workspace_bytes(const lbm_config* cfg, int64_t nsteps, int32_t ckpt_every,
                                size_t* bytes);

/* Objective and its gradient dJ/d(ramp_len, n0, sigma_r, nb) over nsteps steps from the
 * initial state.  The context must be at step 0.  Forward pass with a stored checkpoint every
 * ckpt_every steps, then segment by segment in reverse: recompute the segment's states (and the
 * site record of each of its steps: the site-averaged fields and the moments of the pulled
 * populations, which is all the reverse step needs of the collision's input) from its
 * checkpoint, and run the reverse steps.
 * The last segment is kept from the forward pass (its states and site records go straight to a
 * segment buffer), so it is not recomputed.  The recompute of the next segment runs on a second
 * stream, created by the library on first use (default priority, released by lbm_destroy),
 * while the reverse steps run on the caller's stream; with more than one segment the workspace
 * holds two segment buffers.  On return the context holds the state after nsteps (on an error
 * it still holds the initial state).  cfg.check_every is not applied inside this call.
 * Synchronising.  Periodic dimensions need at least 5 cells. */
int lbm_adjoint(lbm_ctx* ctx, const lbm_objective* obj, int64_t nsteps, int32_t ckpt_every,
                void* adj_ws, size_t adj_bytes, double* J, double grad[4]);

/* Objective and gradient as lbm_adjoint, under a budget of `snapshots` stored states instead of
 * a checkpoint interval: binomial (revolve-type) checkpointing.  With s snapshots and every step
 * advanced at most t times, C(s + t, s) steps can be reversed; the recursion places each next
 * snapshot so that the later part of a range fits one snapshot fewer.  The workspace holds the
 * snapshots and the site record of one step.  The context's two state buffers serve as scratch;
 * on return the context holds its initial state (step 0) again.  steps_advanced (may be NULL)
 * receives the number of forward steps taken, including the one each reverse step recomputes.
 * Synchronising.  Periodic dimensions need at least 5 cells. */
int lbm_adjoint_revolve_workspace_bytes(const lbm_config* cfg, int32_t snapshots, size_t* bytes);
int lbm_adjoint_revolve(lbm_ctx* ctx, const lbm_objective* obj, int64_t nsteps, int32_t snapshots,
                        void* adj_ws, size_t adj_bytes, double* J, double grad[4],
                        int64_t* steps_advanced);

/* The objective J of lbm_adjoint for the current state, without its gradient: E_z of row obj->row
 * linearly interpolated in z at z_d(t_{k-1}) - obj->z_behind after k >= 1 steps (the time level of
 * E in the state), z_d the driver centre.  Equals the J that lbm_adjoint returns after the same
 * steps.  LBM_EINVAL for a row outside [0, nr) or a position outside the window, LBM_ESTATE before
 * the first step.  Synchronising. */
int lbm_witness(lbm_ctx* ctx, const lbm_objective* obj, double* J);

/* FP64 diagnostics of the current state (the sums of lbm_diag above; deterministic two-pass
 * reduction).  The charge is the electron number of the window, the quantity the moving-window
 * set-up of Sec. IV conserves apart from inflow and outflow; the field energy is that of the
 * fields of Eq. (5) on the Yee points; the Gauss residual checks Gauss's law, which the paper does
 * not state and the scheme keeps only at t = 0 (the initial field is the driver's discrete Gauss
 * field), since J_e = n beta of Eq. (5) leaves out the lattice's diffusive flux.  LBM_ESTATE for a
 * NULL context, LBM_EINVAL for a NULL out.  Synchronising. */
int lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out);

/* lbm_diagnostics for callers that cannot allocate device memory (harnesses that forbid hipMalloc,
 * tight loops that must not allocate; it copies its result to the host, so it is not for code
 * under HIP graph capture).  The same values, bit for bit, as
 * lbm_diagnostics on the same state: the same kernels, with their per-block partial sums in a
 * fixed array inside the library instead of the context's workspace.  That array holds the partials
 * of at most 2048 blocks plus the result (16,392 doubles, 131,136 bytes); the first pass strides
 * over the lattice, so every lattice that lbm_init accepts fits, and a larger need is refused with
 * LBM_EINVAL.  Each GPU holds one copy of the array from the first lbm_init on it until the
 * process ends, and every call on that GPU shares it: calls that overlap in time on one GPU (other
 * streams or host threads) race on it and must be serialised by the caller.  Makes no allocation
 * (no hipMalloc, hipFree or allocating library call).  LBM_ESTATE for a NULL context, LBM_EINVAL
 * for a NULL out.  Synchronising. */
int lbm_diagnostics_noalloc(lbm_ctx* ctx, lbm_diag* out);

/* Bubble length (Sec. IV, Fig. 4): the number of sites of row `row` at lab positions z in
 * [z_from, z_to] whose electron density is below n_star times the local background density
 * n_bg(z) (sites in vacuum, n_bg = 0, excluded; the paper uses n_star = 0.95), and that number
 * times dz (length may be NULL).  The comparison is made in FP64.  Synchronising.  LBM_EINVAL for
 * a row outside [0, nr), n_star <= 0 or a NaN bound. */
int lbm_bubble_length(lbm_ctx* ctx, int32_t row, double n_star, double z_from, double z_to,
                      int64_t* count, double* length);

/* Macroparticle bunch of LBM_DRIVER_PARTICLES (Sec. II, Eq. (1)), host memory, [7][n] row-major:
 * x, y, z (lab frame, z along the axis), p_x, p_y, p_z (units of m_e c), w (electrons, in units of
 * n_0 / k_p^3).  Positions are at t_{k-1} and momenta at t_{k-1/2} for a context after k steps
 * (after lbm_init: positions at t = -dt, momenta at t = -dt/2).  n <= cfg.max_particles.
 * init_fields = 1 (only at step 0) also sets the initial field from the bunch: E_z = 0, E_r and
 * B_theta from the discrete Gauss law of the bunch density deposited at t = -dt (E_r) and at
 * t = -dt/2 (B_theta, with B_theta = E_r as for a bunch at c); the fluid is not touched.
 * init_fields = 0 keeps the fields (to resume a run).  The library keeps its own copy, stored in
 * an order of its choosing (lbm_get_bunch returns the caller's order).  Synchronising.
 * LBM_EINVAL for another driver, n out of range, a non-finite value, a negative weight, or
 * init_fields at a step other than 0 (the previous bunch is kept); LBM_ENOMEM if host memory
 * runs out; LBM_EHIP if the upload fails, which leaves the context with no particles. */
int lbm_set_bunch(lbm_ctx* ctx, int64_t n, const double* bunch, int32_t init_fields);

/* Current bunch, [7][n] in the layout of lbm_set_bunch and in the caller's order (lbm_step
 * re-sorts the stored bunch; a device index array maps it back), into host memory of at least
 * 7 * n_max doubles; the number of particles goes to *n (lost particles included, with w = 0).
 * LBM_EINVAL if n_max is smaller; LBM_ESTATE (bunch left unwritten) if the index array read back
 * is not a permutation; LBM_EHIP if a download fails.  Synchronising. */
int lbm_get_bunch(lbm_ctx* ctx, double* bunch, int64_t n_max, int64_t* n);

/* Step and window-shift counters of the state. */
int lbm_counters(lbm_ctx* ctx, int64_t* step, int64_t* shifts);

/* Release the context (not the caller's workspace). */
int lbm_destroy(lbm_ctx* ctx);

/* Message of the last failed call on this thread ("" if none).  Valid until the next call. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMPWFA_H */
