// Internal declarations shared by the kernels and the host runtime of liblbmpwfa.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

// Tile of the fused step kernel: TZ sites along z (one wavefront) by TR rows.
constexpr int TZ = 64;
constexpr int TR = 4;
constexpr int NTHREADS = TZ * TR;
// Row pitch of every plane, in elements (keeps every row start 256-byte aligned in FP32).
constexpr int PITCH_ALIGN = 64;
// Blocks of the diagnostic reduction: threads per block, and the most blocks its first pass uses
// (each thread strides over the lattice).
constexpr int RED_THREADS = 256;
constexpr int DIAG_MAX_BLOCKS = 2048;
// Devices for which the library keeps per-device state (the scratch address of
// lbm_diagnostics_noalloc).
constexpr int MAX_DEVICES = 64;

// FP32 storage (1) keeps bfloat16 residuals of E_r and B_theta in a fourth field plane
// (compensated fields); the other storages have three field planes.
__host__ __device__ constexpr bool fields_lo(int storage) { return storage == 1; }
__host__ __device__ constexpr int field_planes(int storage) { return fields_lo(storage) ? 4 : 3; }

// Physical and grid parameters of a run (fixed for a context).
struct Physics {
  int nz, nr, pitch;
  long long plane;          // nr * pitch elements
  double h, dt, lam, tau, D, n_floor;
  double n0, ramp_start, ramp_len;
  int ramp_kind;
  double nb, sigma_z, sigma_r, zd0;
  int window, m, per_z, per_r, fields_on, cyl_on;
  int fp64_math;            // FP64 arithmetic for FP32 / FP16 storage
  int coll;                 // collision operator: 0 BGK, 1 TRT, 2 regularised, 3 MRT
  double tau_plus;          // TRT: relaxation time of the even part (tau otherwise)
  int driver;               // 0 rigid bi-Gaussian, 1 macroparticles
  long long cap;            // macroparticle capacity (driver 1)
  int bunch_nt;             // driver 1: non-temporal bunch accesses in the push and move
  double mrt_se, mrt_seps, mrt_sq, mrt_spi;   // MRT rates of energy, energy square, heat flux, stress
};

// One launch of the fused step: physics + time counters + buffers.
struct StepArgs {
  Physics p;
  long long k;      // index of the step being taken (state holds k completed steps)
  long long s;      // window shift count before this step
  int shift;        // 1 if the window moves at the end of this step
  const void* g_in;
  void* g_out;
  const void* M_in;
  void* M_out;
  const void* E_in;  // [3 planes] E_z, E_r, B_theta; FP32 storage: a fourth plane with the
                     // bfloat16 residuals of E_r (low half) and B_theta (high half) of each cell
  void* E_out;
  void* site_out;    // optional, for the reverse sweep: [6 planes] at the output index, E_z, E_r,
                     // B_theta averaged to the sites as used by the fluid (fields on; else left
                     // alone), then the moments n, n p_z, n p_r of the pulled populations (Eq. (8),
                     // ghosts included, before the forcing); nullptr to skip
  const void* jb_in; // particle driver: [2 planes] J_bz (E_z points), J_br (E_r points) at
                     // t_{k-1/2}, logical columns of x^k (auxiliary type)
  void* jb_zero;     // particle driver: [2 planes] cleared at the output index for the next step
  int jb_c0 = 0;     // particle driver: columns [jb_c0, jb_c1] (logical, frame s) and rows
  int jb_c1 = -1;    // [0, jb_r1] outside which J_b is zero in both buffers: blocks whose tile
  int jb_r1 = -1;    // misses them skip J_b (loads and clears)
};

// One reverse step of the adjoint at the state x^k (k, s, shift as for the forward step k).
// lam_next / lam: 33 pitched planes in the adjoint precision (FP64 for FP64 storage, FP32
// otherwise): 27 population planes, 3 moments, E_z, E_r, B_theta.  The population planes of lam
// (output) hold f_bar^k, the adjoint of the populations each site pulls in step k; those of
// lam_next hold f_bar^{k+1} (pull_in = 1) or the adjoint of the stored populations g^{k+1}
// (pull_in = 0).  work: 6 pitched planes (adjoint precision); partials: per-block theta partials.
struct AdjArgs {
  Physics p;
  long long k, s;
  int shift;
  int pull_in;
  const void* g;
  const void* M;
  const void* E;
  const void* lam_next;
  void* lam;
  void* work;
  const void* site;   // site record of step k (6 planes, auxiliary type, output index, as site_out)
  double* partials;
};

// The fields of AdjArgs that change from one reverse step to the next (everything but the
// physics), so that a launch covering two steps carries the physics once.
struct AdjStep {
  long long k, s;
  int shift;
  int pull_in;
  const void* g;
  const void* M;
  const void* E;
  const void* lam_next;
  void* lam;
  void* work;
  const void* site;
  double* partials;
};

// Launchers (defined in lbm_kernels.hip / lbm_adjoint.hip).  storage: 0 F64, 1 F32, 2 F16.
hipError_t launch_step(int storage, const StepArgs& a, hipStream_t st);
// Bubble length count of one row (single block) into *out (device).
// Particle driver (lbm_bunch.hip).  bunch: SoA [7][cap] doubles (x, y, z, p_x, p_y, p_z, w).
// Move to t_k and deposit J_b(t_{k-1/2}) (atomics, auxiliary type) into jb (2 planes).
hipError_t launch_bunch_move(int storage, const Physics& p, long long s, double* bunch, int n, long long cap,
                             void* jb, hipStream_t st);
// Boris push with E^k, B^{k+1/2} (Eout, frame s + shift) and B^{k-1/2} (Ein, frame s).
hipError_t launch_bunch_push(int storage, const Physics& p, long long s, int shift, const void* Ein,
                             const void* Eout, double* bunch, int n, long long cap, hipStream_t st);
// The push of step k (arguments as above) and the move of step k + 1 (frame s + shift, deposit into
// jb) in one launch.
hipError_t launch_bunch_push_move(int storage, const Physics& p, long long s, int shift, const void* Ein,
                                  const void* Eout, double* bunch, int n, long long cap, void* jb, hipStream_t st);
// Re-sort of the bunch by cell (column of z in frame s, then row; lost particles last): in -> out
// (SoA [7][cap] each, not overlapping) with the caller's indices pid_in -> pid_out; scratch holds
// bunch_sort_bytes(p) bytes (256-byte aligned), whose contents need not be kept between calls.
// rshift: rows are merged in groups of 2^rshift so that the nkeys keys stay within a bound.
void bunch_sort_shape(const Physics& p, int* rshift, long long* nkeys);
size_t bunch_sort_bytes(const Physics& p);
hipError_t launch_bunch_resort(const Physics& p, long long s, const double* in, const int32_t* pid_in, int n,
                               void* scratch, double* out, int32_t* pid_out, hipStream_t st);
// Extent of the live particles (lab frame, cells of dz), as partial extents of
// bunch_extent_blocks(n) <= EXTENT_BLOCKS blocks: out[3 b] = min floor(z / dz), out[3 b + 1] = max
// floor(z / dz), out[3 b + 2] = max floor(r / dr) over block b's particles (min > max when it has no
// live particle); the caller reduces them.
constexpr int EXTENT_BLOCKS = 128;
int bunch_extent_blocks(int n);
hipError_t launch_bunch_extent(const Physics& p, const double* bunch, int n, long long cap, int* out,
                               hipStream_t st);
// Bunch density (FP64, atomics) on the nodes z = (s + i + zoff) dz, rows (j + 1/2) dr, positions moved
// by t_ahead along the velocities; dens must be cleared first.
hipError_t launch_bunch_density(const Physics& p, long long s, double zoff, double t_ahead, const double* bunch,
                                int n, long long cap, double* dens, hipStream_t st);
// Discrete Gauss field of the density dens into plane comp (1 = E_r, 2 = B_theta) of E.
hipError_t launch_bunch_gauss(int storage, const Physics& p, const double* dens, void* E, int comp, hipStream_t st);
hipError_t launch_bubble(int storage, const Physics& p, long long s, const void* M, int row, double n_star,
                         double z0, double z1, long long* out, hipStream_t st);
hipError_t launch_init_fluid(int storage, const Physics& p, const double* n_pert,
                             const double* p_init, void* g, void* M, hipStream_t st);
hipError_t launch_init_fields(int storage, const Physics& p, void* E, hipStream_t st);
hipError_t launch_moments_out(int storage, const Physics& p, long long s, const void* M,
                              void* dst, int dst_f64, hipStream_t st);
hipError_t launch_fields_out(int storage, const Physics& p, const void* E, void* dst,
                             int dst_f64, hipStream_t st);
// One plane of the FP64 state view: component c in [0, 33) (27 populations, 3 moments,
// 3 fields) written unpadded to dst[nr][nz].
hipError_t launch_state_get(int storage, const Physics& p, long long s, const void* g,
                            const void* M, const void* E, int c, double* dst, hipStream_t st);
hipError_t launch_state_set(int storage, const Physics& p, long long s, void* g, void* M,
                            void* E, int c, const double* src, hipStream_t st);
// Diagnostics: partials[nblocks][8] then a single-block final pass into out[8].
int diag_blocks(const Physics& p);
// Device address of the library's fixed diagnostic scratch on the current device (partials of
// DIAG_MAX_BLOCKS blocks, then out[8]), and its size in doubles.
hipError_t diag_scratch(double** ptr);
size_t diag_scratch_doubles();
// drv: FP64 driver density at the nodes (z_i, r_j) and t_{k-1} (pitched plane), or nullptr for the
// rigid driver's closed form.
hipError_t launch_diagnostics(int storage, const Physics& p, long long k, long long s,
                              const void* M, const void* E, const double* drv, double* partials, double* out,
                              hipStream_t st);
// Adjoint: per-block accumulators (2 * adjoint_partial_blocks of 4 doubles, zeroed by the caller),
// one reverse step, the theta partials of the initial state (lam_next = lambda^0), and the final
// sum of the accumulators added into grad_acc[4].
int adjoint_partial_blocks(const Physics& p);
hipError_t launch_adjoint_step(int storage, const AdjArgs& a, hipStream_t st);
// The two halves of a reverse step (site part, then cell part), and the fused launch of the cell
// part of step k with the site part of step k - 1 (same partial accumulators as the site part).
hipError_t launch_adjoint_site(int storage, const AdjArgs& a, hipStream_t st);
hipError_t launch_adjoint_cell(int storage, const AdjArgs& a, hipStream_t st);
hipError_t launch_adjoint_fused(int storage, const AdjArgs& cell, const AdjArgs& site, hipStream_t st);
hipError_t launch_adjoint_init(int storage, const AdjArgs& a, hipStream_t st);
hipError_t adjoint_reduce(const Physics& p, const double* partials, double* grad_acc, hipStream_t st);
// lambda^k (a.lam) in the stored-state layout: 33 pitched FP64 planes written to out.
hipError_t launch_adjoint_state(int storage, const AdjArgs& a, double* out, hipStream_t st);
// 33 pitched FP64 planes (stored-state layout) into the adjoint precision.
hipError_t launch_adjoint_cast(int storage, const Physics& p, const double* in, void* out, hipStream_t st);

}  // namespace lbm
