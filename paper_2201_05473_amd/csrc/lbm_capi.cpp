// Host runtime and C ABI of liblbmpwfa (see include/lbmpwfa.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lbmpwfa.h"
#include "lbm_internal.h"

using lbm::Physics;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_CHECK(expr, what)                    \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t pop_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }
size_t aux_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }
// bytes of one group of field planes (E_z, E_r, B_theta, and the residual plane of FP32 storage)
size_t field_bytes(size_t plane, int storage) { return (size_t)lbm::field_planes(storage) * plane * aux_bytes(storage); }

// Validate a configuration; on success fill the derived physics.
int validate(const lbm_config* c, Physics* p) {
  if (!c) return fail(LBM_EINVAL, "config is NULL");
  if (c->nz < 3 || c->nr < 3) return fail(LBM_EINVAL, "nz and nr must be >= 3 (got %d, %d)", c->nz, c->nr);
  if ((long long)c->nz * c->nr > (1LL << 31) / 32)
    return fail(LBM_EINVAL, "grid too large (%d x %d)", c->nz, c->nr);
  if (c->nr > 65535) return fail(LBM_EINVAL, "nr must be <= 65535 (got %d)", c->nr);   // rows on grid y
  if (!(c->dz > 0.0) || !std::isfinite(c->dz)) return fail(LBM_EINVAL, "dz must be positive");
  if (std::fabs(c->dr - c->dz) > 1e-12 * c->dz) return fail(LBM_EINVAL, "dz and dr must be equal");
  const double lam = c->c_dt_over_dz;
  if (!(lam > 0.0) || !(lam < 1.0 / std::sqrt(3.0)))
    return fail(LBM_EINVAL, "c_dt_over_dz must lie in (0, 1/sqrt(3)) (got %g)", lam);
  if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_EINVAL, "tau must exceed 1/2 (got %g)", c->tau);
  if (c->storage != LBM_F64 && c->storage != LBM_F32 && c->storage != LBM_F16 && c->storage != LBM_F16N)
    return fail(LBM_EINVAL, "unknown storage %d", c->storage);
  if (c->periodic < 0 || c->periodic > 3) return fail(LBM_EINVAL, "periodic must be in [0, 3]");
  const int per_z = c->periodic & 1, per_r = (c->periodic >> 1) & 1;
  if (per_z && c->moving_window) return fail(LBM_EINVAL, "periodic z excludes the moving window");
  if (per_r && (c->fields_on || c->cyl_on))
    return fail(LBM_EINVAL, "periodic r needs fields_on = 0 and cyl_on = 0");
  int m = 0;
  if (c->moving_window) {
    m = (int)std::lround(1.0 / lam);
    if (m < 1 || std::fabs(m * lam - 1.0) > 1e-9)
      return fail(LBM_EINVAL, "the moving window needs 1/(c dt/dz) to be an integer (got %g)", 1.0 / lam);
  }
  if (c->ramp_kind < 0 || c->ramp_kind > 2) return fail(LBM_EINVAL, "unknown ramp_kind %d", c->ramp_kind);
  if (c->ramp_kind != 0 && !(c->ramp_len > 0.0)) return fail(LBM_EINVAL, "ramp_len must be positive");
  if (!std::isfinite(c->n0) || c->n0 < 0.0) return fail(LBM_EINVAL, "n0 must be finite and >= 0");
  if (!std::isfinite(c->nb)) return fail(LBM_EINVAL, "nb must be finite");
  if (c->nb != 0.0 && !(c->sigma_z > 0.0 && c->sigma_r > 0.0))
    return fail(LBM_EINVAL, "driver sizes must be positive");
  if (!(c->n_floor >= 0.0)) return fail(LBM_EINVAL, "n_floor must be >= 0");
  if (c->check_every < 0) return fail(LBM_EINVAL, "check_every must be >= 0");
  if (c->fp64_math != 0 && c->fp64_math != 1) return fail(LBM_EINVAL, "fp64_math must be 0 or 1");
  if (c->collision != LBM_BGK && c->collision != LBM_TRT && c->collision != LBM_REG && c->collision != LBM_MRT)
    return fail(LBM_EINVAL, "unknown collision operator %d", c->collision);
  if (c->collision == LBM_MRT)
    for (double v : {c->mrt_se, c->mrt_seps, c->mrt_sq, c->mrt_spi})
      if (!(v > 0.0 && v < 2.0)) return fail(LBM_EINVAL, "MRT rates must lie in (0, 2) (got %g)", v);
  if (c->collision == LBM_TRT && !(c->trt_magic > 0.0 && std::isfinite(c->trt_magic)))
    return fail(LBM_EINVAL, "trt_magic must be positive and finite (got %g)", c->trt_magic);
  if (c->driver != LBM_DRIVER_RIGID && c->driver != LBM_DRIVER_PARTICLES)
    return fail(LBM_EINVAL, "unknown driver %d", c->driver);
  if (c->driver == LBM_DRIVER_PARTICLES && (c->max_particles < 0 || c->max_particles > INT32_MAX))
    return fail(LBM_EINVAL, "max_particles must lie in [0, 2^31) (got %lld)", (long long)c->max_particles);
  if (c->driver == LBM_DRIVER_PARTICLES && c->resort_every < 0)
    return fail(LBM_EINVAL, "resort_every must be >= 0 (got %d)", c->resort_every);
  if (c->driver == LBM_DRIVER_PARTICLES && c->bunch_streaming != 0 && c->bunch_streaming != 1)
    return fail(LBM_EINVAL, "bunch_streaming must be 0 or 1 (got %d)", c->bunch_streaming);
  if (p) {
    Physics& q = *p;
    std::memset(&q, 0, sizeof q);
    q.nz = c->nz;
    q.nr = c->nr;
    q.pitch = (int)round_up((size_t)c->nz, lbm::PITCH_ALIGN);
    // Planes are 256 bytes (of the population type) longer than their nr pitched rows: with a
    // power-of-two plane (2048 x 512 FP32 is 4 MiB) the 27 loads of a site map to the same
    // memory channels, depending on where the buffer lands (measured on 2048 x 512 FP32:
    // 52.3 -> 51.0 us per step; 4096 x 1024: 220.5 -> 209.2 us).
    q.plane = (long long)q.nr * q.pitch + 256 / (long long)pop_bytes(c->storage);
    q.h = c->dz;
    q.lam = lam;
    q.dt = lam * c->dz;
    q.tau = c->tau;
    q.D = (c->tau - 0.5) / 3.0 * c->dz * c->dz / q.dt;   // Eq. (12) in normalised units
    q.n_floor = c->n_floor;
    q.n0 = c->n0;
    q.ramp_start = c->ramp_start;
    q.ramp_len = c->ramp_kind ? c->ramp_len : 1.0;
    q.ramp_kind = c->ramp_kind;
    q.nb = c->nb;
    q.sigma_z = c->nb != 0.0 ? c->sigma_z : 1.0;
    q.sigma_r = c->nb != 0.0 ? c->sigma_r : 1.0;
    q.zd0 = c->zd0;
    q.window = c->moving_window ? 1 : 0;
    q.m = m;
    q.per_z = per_z;
    q.per_r = per_r;
    q.fields_on = c->fields_on ? 1 : 0;
    q.cyl_on = c->cyl_on ? 1 : 0;
    q.fp64_math = c->fp64_math;
    q.coll = c->collision;
    q.tau_plus = c->collision == LBM_TRT ? 0.5 + c->trt_magic / (c->tau - 0.5) : c->tau;
    q.driver = c->driver;
    q.cap = c->driver == LBM_DRIVER_PARTICLES ? (long long)c->max_particles : 0;
    q.bunch_nt = c->driver == LBM_DRIVER_PARTICLES ? c->bunch_streaming : 0;
    q.mrt_se = c->mrt_se;
    q.mrt_seps = c->mrt_seps;
    q.mrt_sq = c->mrt_sq;
    q.mrt_spi = c->mrt_spi;
  }
  return LBM_OK;
}

// Workspace layout: two population buffers, two moment buffers, two field buffers, and the
// reduction scratch, each 256-byte aligned.
// The particle driver adds two bunch buffers (SoA [7][cap] doubles; a re-sort moves the bunch from
// one to the other) with the caller's index of each stored particle (int32 [cap] each), the
// scratch of the re-sort, a slot for the bunch's extent, two deposit buffers of J_bz, J_br (auxiliary type, alternating between
// steps) and an FP64 density plane (initial field, diagnostics); none of them for the rigid driver.
struct Layout {
  size_t g[2], M[2], E[2], partials, out, bunch[2], pid[2], sort, ext, jb[2], dens, total;
};

Layout layout(const Physics& p, int storage) {
  Layout L;
  const size_t plane = (size_t)p.plane;
  const size_t gb = round_up(27 * plane * pop_bytes(storage), 256);
  const size_t mb = round_up(3 * plane * aux_bytes(storage), 256);
  const size_t eb = round_up(field_bytes(plane, storage), 256);
  size_t off = 0;
  for (int b = 0; b < 2; ++b) { L.g[b] = off; off += gb; }
  for (int b = 0; b < 2; ++b) { L.M[b] = off; off += mb; }
  for (int b = 0; b < 2; ++b) { L.E[b] = off; off += eb; }
  L.partials = off;
  off += round_up((size_t)lbm::diag_blocks(p) * 8 * sizeof(double), 256);
  L.out = off;
  off += 256;
  L.bunch[0] = L.bunch[1] = L.pid[0] = L.pid[1] = L.sort = L.ext = L.jb[0] = L.jb[1] = L.dens = off;
  if (p.driver == 1) {
    for (int b = 0; b < 2; ++b) {
      L.bunch[b] = off;
      off += round_up(7 * (size_t)p.cap * sizeof(double), 256);
      L.pid[b] = off;
      off += round_up((size_t)p.cap * sizeof(int32_t), 256);
    }
    L.sort = off;
    off += round_up(lbm::bunch_sort_bytes(p), 256);
    L.ext = off;
    off += round_up(3 * lbm::EXTENT_BLOCKS * sizeof(int), 256);
    for (int b = 0; b < 2; ++b) {
      L.jb[b] = off;
      off += round_up(2 * plane * aux_bytes(storage), 256);
    }
    L.dens = off;
    off += round_up(plane * sizeof(double), 256);
  }
  L.total = off;
  return L;
}

}  // namespace

struct lbm_ctx {
  lbm_config cfg;
  Physics p;
  int storage;
  char* ws;
  Layout L;
  int cur;
  long long k, s;
  hipStream_t stream;
  // the adjoint's second stream (segment recompute, overlapped with the reverse sweep) and its
  // events; created on first use, default priority
  hipStream_t aux = nullptr;
  hipEvent_t ev_fwd = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  // particle driver: particles in the bunch, the deposit buffer the next step fills, and the bunch
  // buffer in use (with the caller's index of each stored particle; the bunch is stored by cell:
  // column of z, then radius)
  long long nbunch = 0;
  int jcur = 0;
  int bcur = 0;
  // extent of the live particles when the bunch was last set or re-sorted (lab-frame cells: lowest
  // and highest column of z, highest row of r; empty when ext[0] > ext[1]) and the number of steps
  // taken since (a state loaded in between changes k, not the distance the particles have moved):
  // it bounds where the deposits of the following steps can fall
  int ext[3] = {INT32_MAX, INT32_MIN, INT32_MIN};
  long long ext_age = 0;
  // device address of the library's fixed diagnostic scratch on the context's device
  double* scratch = nullptr;
  // set when a failed lbm_adjoint_revolve could not put the initial state back into the context's
  // buffers (which it uses as scratch); cleared by lbm_set_state / lbm_load
  bool broken = false;
  double* bunch(int b) { return (double*)(ws + L.bunch[b]); }
  double* bunch() { return bunch(bcur); }
  int32_t* pid(int b) { return (int32_t*)(ws + L.pid[b]); }
  void* sort_scratch() { return ws + L.sort; }
  int* ext_dev() { return (int*)(ws + L.ext); }
  void* jb(int b) { return ws + L.jb[b]; }
  double* dens() { return (double*)(ws + L.dens); }
  void* g(int b) { return ws + L.g[b]; }
  void* M(int b) { return ws + L.M[b]; }
  void* E(int b) { return ws + L.E[b]; }
  double* partials() { return (double*)(ws + L.partials); }
  double* red_out() { return (double*)(ws + L.out); }
  // Scratch for host transfers: the inactive population buffer (free between steps).
  void* staging() { return g(1 - cur); }
  size_t staging_bytes() const { return L.g[1] - L.g[0]; }
};

namespace {

// LBM_ESTATE for a NULL context or one whose state was lost (see lbm_ctx::broken).
int live(const lbm_ctx* c) {
  if (!c) return fail(LBM_ESTATE, "context is NULL");
  if (c->broken)
    return fail(LBM_ESTATE, "the context's state was lost by a failed lbm_adjoint_revolve; "
                            "restore a state with lbm_set_state or lbm_load");
  return LBM_OK;
}

// Driver density at the nodes (z_i, r_j) and t_{k-1} for the Gauss residual: the particle bunch
// deposited from its positions (which are at t_{k-1}) into the FP64 density plane, or nullptr for
// the rigid driver's closed form.
hipError_t driver_density_plane(lbm_ctx* c, const double** out) {
  *out = nullptr;
  if (c->p.driver != 1) return hipSuccess;
  hipError_t e = hipMemsetAsync(c->dens(), 0, (size_t)c->p.plane * sizeof(double), c->stream);
  if (e == hipSuccess)
    e = lbm::launch_bunch_density(c->p, c->s, 0.0, 0.0, c->bunch(), (int)c->nbunch, c->p.cap, c->dens(), c->stream);
  *out = c->dens();
  return e;
}

// Where J_b can be non-zero at the step about to be taken (the deposit the step reads, the
// previous one its clear removes, the next one the cleared buffer receives): the extent of the live
// particles ext_age steps ago, widened by the distance a particle can travel (|v| < c: dt per step
// in z and in r) between then and the midpoints of those deposits, by the stencils' reach and by
// one cell of rounding.  Columns in the window frame of the step.
void jb_bound(const lbm_ctx* c, lbm::StepArgs& a) {
  if (c->ext[0] > c->ext[1]) {   // no live particle: no deposit
    a.jb_c0 = 1 << 30;
    a.jb_c1 = -(1 << 30);
    a.jb_r1 = -(1 << 30);
    return;
  }
  const long long m = (long long)std::ceil(((double)c->ext_age + 2.0) * c->p.dt / c->p.h) + 3;
  const auto clampi = [](long long v) { return (int)std::min<long long>(std::max<long long>(v, -(1LL << 30)), 1LL << 30); };
  a.jb_c0 = clampi((long long)c->ext[0] - m - c->s);
  a.jb_c1 = clampi((long long)c->ext[1] + 1 + m - c->s);
  a.jb_r1 = clampi((long long)c->ext[2] + 1 + m);
}

int run_check(lbm_ctx* c) {
  const double* drv;
  HIP_CHECK(driver_density_plane(c, &drv), "bunch density launch");
  HIP_CHECK(lbm::launch_diagnostics(c->storage, c->p, c->k, c->s, c->M(c->cur), c->E(c->cur), drv,
                                    c->partials(), c->red_out(), c->stream),
            "diagnostics launch");
  double out[8];
  HIP_CHECK(hipMemcpyAsync(out, c->red_out(), sizeof out, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  if (out[4] != 0.0 || !std::isfinite(out[3]))
    return fail(LBM_EUNSTABLE, "non-finite state after step %lld", c->k);
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes) {
  Physics p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  *bytes = layout(p, cfg->storage).total;
  return LBM_OK;
}

int lbm_init(const lbm_config* cfg, const double* n_pert, const double* p_init, void* workspace,
             size_t ws_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  Physics p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
  if ((uintptr_t)workspace % 256 != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = layout(p, cfg->storage);
  if (ws_bytes < L.total)
    return fail(LBM_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  lbm_ctx* c = new (std::nothrow) lbm_ctx;
  if (!c) return fail(LBM_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->p = p;
  c->storage = cfg->storage;
  c->ws = (char*)workspace;
  c->L = L;
  c->cur = 0;
  c->k = 0;
  c->s = 0;
  c->stream = (hipStream_t)hip_stream;
  auto bail = [&](int code) { delete c; return code; };
  // the fixed scratch of lbm_diagnostics_noalloc on this device (looked up once per device)
  hipError_t e = lbm::diag_scratch(&c->scratch);
  if (e != hipSuccess) return bail(hip_fail(e, "diagnostic scratch lookup"));
  e = hipMemsetAsync(workspace, 0, L.total, c->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "workspace clear"));
  // Upload the perturbation arrays into the inactive population buffer.
  const size_t plane_u = (size_t)p.nr * p.nz;
  double* stage = (double*)c->staging();
  const double* d_pert = nullptr;
  const double* d_pinit = nullptr;
  if (3 * plane_u * sizeof(double) > c->staging_bytes()) return bail(fail(LBM_ENOMEM, "staging too small"));
  if (n_pert) {
    e = hipMemcpyAsync(stage, n_pert, plane_u * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "upload n_pert"));
    d_pert = stage;
  }
  if (p_init) {
    e = hipMemcpyAsync(stage + plane_u, p_init, 2 * plane_u * sizeof(double), hipMemcpyHostToDevice,
                       c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "upload p_init"));
    d_pinit = stage + plane_u;
  }
  e = lbm::launch_init_fluid(c->storage, p, d_pert, d_pinit, c->g(0), c->M(0), c->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "init fluid launch"));
  e = lbm::launch_init_fields(c->storage, p, c->E(0), c->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "init fields launch"));
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "init synchronise"));
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (int rc_ = live(c)) return rc_;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  // particle driver: the push of a step and the move of the next run as one launch between two
  // steps of this call (not across a diagnostic check, which reads the bunch at t_{k-1}, nor across
  // a re-sort, which sorts the positions at t_{k-1}); moved: the bunch is already at t_k with
  // J_b(t_{k-1/2}) in jb(jcur)
  const long long resort = c->cfg.resort_every > 0 ? c->cfg.resort_every : 500;
  bool moved = false;
  for (int64_t n = 0; n < nsteps; ++n) {
    lbm::StepArgs a;
    a.p = c->p;
    a.k = c->k;
    a.s = c->s;
    a.shift = (c->p.window && (c->k + 1) % c->p.m == 0) ? 1 : 0;
    a.g_in = c->g(c->cur);
    a.g_out = c->g(1 - c->cur);
    a.M_in = c->M(c->cur);
    a.M_out = c->M(1 - c->cur);
    a.E_in = c->E(c->cur);
    a.E_out = c->E(1 - c->cur);
    a.site_out = nullptr;
    a.jb_in = nullptr;
    a.jb_zero = nullptr;
    if (c->p.driver == 1) {
      // particles to t_k and their current J_b(t_{k-1/2}) into the buffer the previous step cleared
      if (!moved) {
        if (c->k > 0 && c->k % resort == 0 && c->nbunch > 0) {
          HIP_CHECK(lbm::launch_bunch_resort(c->p, c->s, c->bunch(c->bcur), c->pid(c->bcur), (int)c->nbunch,
                                             c->sort_scratch(), c->bunch(1 - c->bcur), c->pid(1 - c->bcur),
                                             c->stream),
                    "bunch sort launch");
          c->bcur ^= 1;
          // a fresh extent tightens the J_b bound (one synchronisation per re-sort)
          HIP_CHECK(lbm::launch_bunch_extent(c->p, c->bunch(), (int)c->nbunch, c->p.cap, c->ext_dev(), c->stream),
                    "bunch extent launch");
          const int nb = lbm::bunch_extent_blocks((int)c->nbunch);
          int part[3 * lbm::EXTENT_BLOCKS];
          HIP_CHECK(hipMemcpyAsync(part, c->ext_dev(), 3 * nb * sizeof(int), hipMemcpyDeviceToHost, c->stream),
                    "copy");
          HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
          c->ext[0] = INT32_MAX;
          c->ext[1] = c->ext[2] = INT32_MIN;
          for (int b = 0; b < nb; ++b) {
            c->ext[0] = std::min(c->ext[0], part[3 * b]);
            c->ext[1] = std::max(c->ext[1], part[3 * b + 1]);
            c->ext[2] = std::max(c->ext[2], part[3 * b + 2]);
          }
          c->ext_age = 0;
        }
        HIP_CHECK(lbm::launch_bunch_move(c->storage, c->p, c->s, c->bunch(), (int)c->nbunch, c->p.cap,
                                         c->jb(c->jcur), c->stream),
                  "bunch launch");
      }
      a.jb_in = c->jb(c->jcur);
      a.jb_zero = c->jb(1 - c->jcur);
      jb_bound(c, a);
    }
    HIP_CHECK(lbm::launch_step(c->storage, a, c->stream), "step launch");
    if (c->p.driver == 1) {
      const bool check_next = c->cfg.check_every > 0 && (c->k + 1) % c->cfg.check_every == 0;
      moved = n + 1 < nsteps && !check_next && (c->k + 1) % resort != 0;
      if (moved)
        HIP_CHECK(lbm::launch_bunch_push_move(c->storage, c->p, c->s, a.shift, c->E(c->cur), c->E(1 - c->cur),
                                              c->bunch(), (int)c->nbunch, c->p.cap, c->jb(1 - c->jcur), c->stream),
                  "bunch launch");
      else
        HIP_CHECK(lbm::launch_bunch_push(c->storage, c->p, c->s, a.shift, c->E(c->cur), c->E(1 - c->cur),
                                         c->bunch(), (int)c->nbunch, c->p.cap, c->stream),
                  "bunch launch");
      c->jcur ^= 1;
    }
    c->cur ^= 1;
    c->k += 1;
    c->s += a.shift;
    c->ext_age += 1;
    if (c->cfg.check_every > 0 && c->k % c->cfg.check_every == 0) {
      int rc = run_check(c);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

static int output3(lbm_ctx* c, void* dst, int32_t dtype, int32_t on_device, bool moments) {
  if (int rc_ = live(c)) return rc_;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  if (dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
  const int f64 = dtype == LBM_F64;
  const size_t nbytes = 3 * (size_t)c->p.nr * c->p.nz * (f64 ? 8 : 4);
  void* target = on_device ? dst : c->staging();
  hipError_t e = moments
      ? lbm::launch_moments_out(c->storage, c->p, c->s, c->M(c->cur), target, f64, c->stream)
      : lbm::launch_fields_out(c->storage, c->p, c->E(c->cur), target, f64, c->stream);
  HIP_CHECK(e, "output launch");
  if (!on_device) {
    HIP_CHECK(hipMemcpyAsync(dst, target, nbytes, hipMemcpyDeviceToHost, c->stream), "download");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  }
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, void* dst, int32_t dtype, int32_t dst_on_device) {
  return output3(c, dst, dtype, dst_on_device, true);
}

int lbm_fields(lbm_ctx* c, void* dst, int32_t dtype, int32_t dst_on_device) {
  return output3(c, dst, dtype, dst_on_device, false);
}

int lbm_get_state(lbm_ctx* c, double* dst, int64_t* step, int64_t* shifts) {
  if (int rc_ = live(c)) return rc_;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  const size_t pl = (size_t)c->p.nr * c->p.nz;
  double* stage = (double*)c->staging();
  for (int comp = 0; comp < 33; ++comp) {
    HIP_CHECK(lbm::launch_state_get(c->storage, c->p, c->s, c->g(c->cur), c->M(c->cur), c->E(c->cur),
                                    comp, stage, c->stream),
              "state launch");
    HIP_CHECK(hipMemcpyAsync(dst + comp * pl, stage, pl * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream),
              "download");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  }
  if (step) *step = c->k;
  if (shifts) *shifts = c->s;
  return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const double* src, int64_t step, int64_t shifts) {
  if (!c) return fail(LBM_ESTATE, "context is NULL");
  if (!src) return fail(LBM_EINVAL, "src is NULL");
  if (step < 0 || shifts < 0) return fail(LBM_EINVAL, "counters must be >= 0");
  const size_t pl = (size_t)c->p.nr * c->p.nz;
  double* stage = (double*)c->staging();
  // moments and fields first: LBM_F16N stores each population relative to its site's moments
  for (int n = 0; n < 33; ++n) {
    const int comp = (n + 27) % 33;
    HIP_CHECK(hipMemcpyAsync(stage, src + comp * pl, pl * sizeof(double), hipMemcpyHostToDevice,
                             c->stream),
              "upload");
    HIP_CHECK(lbm::launch_state_set(c->storage, c->p, shifts, c->g(c->cur), c->M(c->cur), c->E(c->cur),
                                    comp, stage, c->stream),
              "state launch");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  }
  c->k = step;
  c->s = shifts;
  c->broken = false;
  return LBM_OK;
}

namespace {
struct CkptHeader {
  char magic[8];
  int32_t storage, nz, nr, pitch;
  int64_t step, shifts, plane;
  int32_t driver, reserved;
  int64_t nbunch;   // particles in the bunch section (LBM_DRIVER_PARTICLES), else 0
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");
const char kMagic[8] = {'L', 'B', 'M', 'P', 'W', 'F', 'A', '3'};

// Head of the bunch section: the extent the J_b bound starts from and its age in steps.
struct CkptBunch {
  int32_t ext[3], reserved;
  int64_t ext_age;
};
static_assert(sizeof(CkptBunch) == 24, "bunch section head is 24 bytes");

size_t region_bytes(const lbm_ctx* c, int which) {
  const size_t plane = (size_t)c->p.plane;
  return which == 0 ? 27 * plane * pop_bytes(c->storage)
                    : (which == 1 ? 3 * plane * aux_bytes(c->storage) : field_bytes(plane, c->storage));
}

// The bunch section of a checkpoint of n particles: head, 7 coordinates per particle (FP64,
// component-major, in stored order) and each particle's index in the caller's order (int32).
size_t bunch_section_bytes(const lbm_ctx* c, long long n) {
  return c->p.driver == LBM_DRIVER_PARTICLES ? sizeof(CkptBunch) + (size_t)n * (7 * sizeof(double) + sizeof(int32_t))
                                             : 0;
}

// One piece of a checkpoint: `bytes` at `ckpt_off` in the checkpoint and at `ctx_mem` in the
// context (device memory, or host memory when `host` is set: the headers).
struct Piece {
  size_t ckpt_off;
  void* ctx_mem;
  size_t bytes;
  bool host;
};

// The pieces of the context's checkpoint after the header, in order.
void pieces(lbm_ctx* c, CkptBunch* bh, std::vector<Piece>& out) {
  size_t off = sizeof(CkptHeader);
  void* reg[3] = {c->g(c->cur), c->M(c->cur), c->E(c->cur)};
  for (int r = 0; r < 3; ++r) {
    out.push_back({off, reg[r], region_bytes(c, r), false});
    off += region_bytes(c, r);
  }
  if (c->p.driver == LBM_DRIVER_PARTICLES) {
    const size_t n = (size_t)c->nbunch;
    out.push_back({off, bh, sizeof(CkptBunch), true});
    off += sizeof(CkptBunch);
    for (int comp = 0; comp < 7; ++comp) {
      out.push_back({off, c->bunch() + comp * c->p.cap, n * sizeof(double), false});
      off += n * sizeof(double);
    }
    out.push_back({off, c->pid(c->bcur), n * sizeof(int32_t), false});
  }
}
}  // namespace

int lbm_checkpoint_bytes(lbm_ctx* c, size_t* bytes) {
  if (int rc_ = live(c)) return rc_;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  *bytes = sizeof(CkptHeader) + region_bytes(c, 0) + region_bytes(c, 1) + region_bytes(c, 2) +
           bunch_section_bytes(c, c->nbunch);
  return LBM_OK;
}

namespace {
int ckpt_save(lbm_ctx* c, void* dst, int32_t on_device) {
  if (int rc_ = live(c)) return rc_;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, 8);
  h.storage = c->storage;
  h.nz = c->p.nz;
  h.nr = c->p.nr;
  h.pitch = c->p.pitch;
  h.plane = c->p.plane;
  h.step = c->k;
  h.shifts = c->s;
  h.driver = c->p.driver;
  h.nbunch = c->p.driver == LBM_DRIVER_PARTICLES ? c->nbunch : 0;
  CkptBunch bh;
  std::memset(&bh, 0, sizeof bh);
  std::memcpy(bh.ext, c->ext, sizeof bh.ext);
  bh.ext_age = c->ext_age;
  std::vector<Piece> ps{{0, &h, sizeof h, true}};
  pieces(c, &bh, ps);
  char* d = (char*)dst;
  for (const Piece& q : ps) {
    hipError_t e = hipSuccess;
    if (!on_device && q.host)
      std::memcpy(d + q.ckpt_off, q.ctx_mem, q.bytes);
    else if (q.bytes > 0)
      e = hipMemcpyAsync(d + q.ckpt_off, q.ctx_mem, q.bytes,
                         q.host ? hipMemcpyHostToDevice : (on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost),
                         c->stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(c->stream);   // queued copies read h and bh
      return hip_fail(e, "save copy");
    }
  }
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  return LBM_OK;
}

int ckpt_load(lbm_ctx* c, const void* src, int32_t on_device) {
  if (!c) return fail(LBM_ESTATE, "context is NULL");
  if (!src) return fail(LBM_EINVAL, "src is NULL");
  const char* s = (const char*)src;
  // reads `bytes` at `off` of the checkpoint into host memory
  const auto read = [&](void* to, size_t off, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;   // `to` may be NULL (an empty bunch)
    if (!on_device) {
      std::memcpy(to, s + off, bytes);
      return hipSuccess;
    }
    const hipError_t e = hipMemcpyAsync(to, s + off, bytes, hipMemcpyDeviceToHost, c->stream);
    const hipError_t e2 = hipStreamSynchronize(c->stream);
    return e != hipSuccess ? e : e2;
  };
  CkptHeader h;
  HIP_CHECK(read(&h, 0, sizeof h), "load header");
  if (std::memcmp(h.magic, kMagic, 8) != 0) return fail(LBM_EINVAL, "not an lbmpwfa checkpoint");
  if (h.storage != c->storage || h.nz != c->p.nz || h.nr != c->p.nr || h.pitch != c->p.pitch ||
      h.plane != c->p.plane)
    return fail(LBM_EINVAL, "checkpoint is for another grid or storage precision");
  if (h.driver != c->p.driver) return fail(LBM_EINVAL, "checkpoint is for another driver");
  if (h.step < 0 || h.shifts < 0) return fail(LBM_EINVAL, "corrupt checkpoint counters");
  const bool particles = c->p.driver == LBM_DRIVER_PARTICLES;
  if (particles ? (h.nbunch < 0 || h.nbunch > c->p.cap) : h.nbunch != 0)
    return fail(LBM_EINVAL, "checkpoint holds %lld particles (max_particles %lld)", (long long)h.nbunch,
                (long long)c->p.cap);
  // the context's pieces with the checkpoint's particle count, into bunch buffer 0
  const long long n = h.nbunch;
  const int bcur_was = c->bcur;
  const long long nbunch_was = c->nbunch;
  c->bcur = 0;
  c->nbunch = particles ? n : 0;
  CkptBunch bh;
  std::vector<Piece> ps;
  pieces(c, &bh, ps);
  c->bcur = bcur_was;
  c->nbunch = nbunch_was;
  if (particles) {
    // the bunch head and the index array are checked before anything of the context changes
    HIP_CHECK(read(&bh, ps[3].ckpt_off, sizeof bh), "load bunch head");
    if (bh.ext_age < 0) return fail(LBM_EINVAL, "corrupt checkpoint bunch extent");
    std::vector<int32_t> pid((size_t)n);
    HIP_CHECK(read(pid.data(), ps.back().ckpt_off, (size_t)n * sizeof(int32_t)), "load bunch indices");
    std::vector<char> seen((size_t)n, 0);
    for (long long i = 0; i < n; ++i) {
      const int32_t o = pid[(size_t)i];
      if (o < 0 || o >= n || seen[(size_t)o]) return fail(LBM_EINVAL, "checkpoint bunch index %lld is not a permutation", i);
      seen[(size_t)o] = 1;
    }
  }
  for (const Piece& q : ps) {
    if (q.host || q.bytes == 0) continue;
    HIP_CHECK(hipMemcpyAsync(q.ctx_mem, s + q.ckpt_off, q.bytes,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
              "load copy");
  }
  if (particles) {
    // the next step deposits into a cleared buffer and clears the other only near the bunch
    for (int b = 0; b < 2; ++b)
      HIP_CHECK(hipMemsetAsync(c->jb(b), 0, 2 * (size_t)c->p.plane * aux_bytes(c->storage), c->stream), "clear");
  }
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  c->k = h.step;
  c->s = h.shifts;
  if (particles) {
    c->nbunch = n;
    c->bcur = 0;
    c->jcur = 0;
    std::memcpy(c->ext, bh.ext, sizeof c->ext);
    c->ext_age = bh.ext_age;
  }
  c->broken = false;
  return LBM_OK;
}
}  // namespace

int lbm_save(lbm_ctx* c, void* dst, int32_t on_device) {
  try {
    return ckpt_save(c, dst, on_device);
  } catch (const std::bad_alloc&) {
    return fail(LBM_ENOMEM, "host allocation failed");
  }
}

int lbm_load(lbm_ctx* c, const void* src, int32_t on_device) {
  try {
    return ckpt_load(c, src, on_device);
  } catch (const std::bad_alloc&) {
    return fail(LBM_ENOMEM, "host allocation failed");
  }
}

// The diagnostics with their partial sums in `partials` and the result in `res` (device).
static int diagnostics_into(lbm_ctx* c, lbm_diag* out, double* partials, double* res) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  const double* drv;
  HIP_CHECK(driver_density_plane(c, &drv), "bunch density launch");
  HIP_CHECK(lbm::launch_diagnostics(c->storage, c->p, c->k, c->s, c->M(c->cur), c->E(c->cur), drv,
                                    partials, res, c->stream),
            "diagnostics launch");
  double r[8];
  HIP_CHECK(hipMemcpyAsync(r, res, sizeof r, hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  out->charge = r[0];
  out->field_energy = r[1];
  out->gauss_max = r[2];
  out->umax = r[3];
  out->nonfinite = (int32_t)r[4];
  out->reserved = 0;
  out->step = c->k;
  out->shifts = c->s;
  return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* c, lbm_diag* out) {
  if (int rc_ = live(c)) return rc_;
  return diagnostics_into(c, out, c->partials(), c->red_out());
}

int lbm_diagnostics_noalloc(lbm_ctx* c, lbm_diag* out) {
  if (int rc_ = live(c)) return rc_;
  if (!c->scratch) return fail(LBM_ESTATE, "no diagnostic scratch on this context's device");
  const size_t need = ((size_t)lbm::diag_blocks(c->p) + 1) * 8;
  if (need > lbm::diag_scratch_doubles())
    return fail(LBM_EINVAL, "diagnostics need %zu scratch doubles, the library holds %zu", need,
                lbm::diag_scratch_doubles());
  return diagnostics_into(c, out, c->scratch, c->scratch + (size_t)lbm::diag_blocks(c->p) * 8);
}

// --------------------------------------------------------------------------------------------
// Adjoint
// --------------------------------------------------------------------------------------------
namespace {

size_t state_bytes(const Physics& p, int storage);

// the site record of one step for its reverse (E_z, E_r, B_theta averaged to the sites, and the
// moments of the pulled populations), auxiliary type
size_t site_bytes(const Physics& p, int storage) {
  return round_up(6 * (size_t)p.plane * aux_bytes(storage), 256);
}

// Adjoint workspace: two lambda buffers and the work planes in the adjoint precision (the
// auxiliary-plane type), the per-block partials, the gradient accumulator; the host-facing VJP
// calls add an FP64 staging area for lambda in the stored-state layout.
struct AdjLayout {
  size_t lamA, lamB, work, work2, partials, grad, core_total, stage, scratch, site, vjp_total;
};

AdjLayout adj_layout(const Physics& p, int storage) {
  AdjLayout L;
  const size_t plane_l = (size_t)p.plane * aux_bytes(storage);
  size_t off = 0;
  L.lamA = off; off += round_up(33 * plane_l, 256);
  L.lamB = off; off += round_up(33 * plane_l, 256);
  L.work = off; off += round_up(6 * plane_l, 256);
  L.work2 = off; off += round_up(6 * plane_l, 256);   // consecutive steps of the fused sweep
  L.partials = off; off += round_up((size_t)lbm::adjoint_partial_blocks(p) * 8 * sizeof(double), 256);
  L.grad = off; off += 256;
  L.core_total = off;
  L.stage = off; off += round_up(33 * (size_t)p.plane * sizeof(double), 256);
  L.scratch = off; off += state_bytes(p, storage);
  L.site = off; off += site_bytes(p, storage);
  L.vjp_total = off;
  return L;
}

// bytes of one stored state in the native layout (populations, moments, fields)
size_t state_bytes(const Physics& p, int storage) {
  const size_t plane = (size_t)p.plane;
  return round_up(27 * plane * pop_bytes(storage), 256) + round_up(3 * plane * aux_bytes(storage), 256) +
         round_up(field_bytes(plane, storage), 256);
}

struct StateView {
  void* g;
  void* M;
  void* E;
};

StateView state_at(char* base, const Physics& p, int storage) {
  const size_t plane = (size_t)p.plane;
  const size_t gb = round_up(27 * plane * pop_bytes(storage), 256);
  const size_t mb = round_up(3 * plane * aux_bytes(storage), 256);
  return StateView{base, base + gb, base + gb + mb};   // fields after the moments
}

int adj_check(lbm_ctx* c, void* ws, size_t bytes, size_t need) {
  if (int rc_ = live(c)) return rc_;
  if (!ws) return fail(LBM_EINVAL, "adjoint workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(LBM_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (bytes < need) return fail(LBM_ENOMEM, "adjoint workspace too small: %zu < %zu bytes", bytes, need);
  if ((c->p.per_z && c->p.nz < 5) || (c->p.per_r && c->p.nr < 5))
    return fail(LBM_EINVAL, "the adjoint needs at least 5 cells along periodic dimensions");
  if (c->storage != LBM_F64 && c->p.fp64_math && c->p.coll != LBM_BGK)
    return fail(LBM_EINVAL, "the adjoint takes fp64_math = 1 with the BGK collision only");
  if (c->p.driver != LBM_DRIVER_RIGID) return fail(LBM_EINVAL, "the adjoint is implemented for the rigid driver only");
  return LBM_OK;
}

// host [33][nr][nz] <-> device 33 planes of [nr][pitch] (FP64), one 2D copy per plane
hipError_t upload_lam(const Physics& p, double* dst, const double* src, hipStream_t st) {
  for (int c = 0; c < 33; ++c) {
    hipError_t e = hipMemcpy2DAsync(dst + c * (size_t)p.plane, (size_t)p.pitch * sizeof(double),
                                    src + c * (size_t)p.nr * p.nz, (size_t)p.nz * sizeof(double),
                                    (size_t)p.nz * sizeof(double), (size_t)p.nr, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t download_lam(const Physics& p, double* dst, const double* src, hipStream_t st) {
  for (int c = 0; c < 33; ++c) {
    hipError_t e = hipMemcpy2DAsync(dst + c * (size_t)p.nr * p.nz, (size_t)p.nz * sizeof(double),
                                    src + c * (size_t)p.plane, (size_t)p.pitch * sizeof(double),
                                    (size_t)p.nz * sizeof(double), (size_t)p.nr, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

lbm::AdjArgs adj_args(lbm_ctx* c, const StateView& x, const void* site, long long k, const void* lam_next,
                      void* lam, int pull_in, char* ws, const AdjLayout& L, int work_buf = 0) {
  lbm::AdjArgs a;
  a.p = c->p;
  a.k = k;
  a.s = c->p.window ? k / c->p.m : 0;
  a.shift = (c->p.window && (k + 1) % c->p.m == 0) ? 1 : 0;
  a.pull_in = pull_in;
  a.g = x.g;
  a.M = x.M;
  a.E = x.E;
  a.lam_next = lam_next;
  a.lam = lam;
  a.site = site;
  a.work = ws + (work_buf ? L.work2 : L.work);
  a.partials = (double*)(ws + L.partials);
  return a;
}

// forward step k from x into y, saving the step's site record (site may be nullptr: a plain step)
hipError_t step_with_site(lbm_ctx* c, long long k, const StateView& x, const StateView& y, void* site,
                          hipStream_t st) {
  lbm::StepArgs a;
  a.p = c->p;
  a.k = k;
  a.s = c->p.window ? k / c->p.m : 0;
  a.shift = (c->p.window && (k + 1) % c->p.m == 0) ? 1 : 0;
  a.g_in = x.g; a.g_out = y.g;
  a.M_in = x.M; a.M_out = y.M;
  a.E_in = x.E; a.E_out = y.E;
  a.site_out = site;
  a.jb_in = nullptr;
  a.jb_zero = nullptr;
  return lbm::launch_step(c->storage, a, st);
}

}  // namespace

int lbm_vjp_workspace_bytes(const lbm_config* cfg, size_t* bytes) {
  Physics p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  *bytes = adj_layout(p, cfg->storage).vjp_total;
  return LBM_OK;
}

int lbm_vjp_step(lbm_ctx* c, void* ws, size_t bytes, const double* lam_next, double* lam_out, double grad[4]) {
  if (int rc_ = live(c)) return rc_;
  const AdjLayout L = adj_layout(c->p, c->storage);
  int rc = adj_check(c, ws, bytes, L.vjp_total);
  if (rc) return rc;
  if (!lam_next || !lam_out || !grad) return fail(LBM_EINVAL, "NULL argument");
  char* w = (char*)ws;
  double* stage = (double*)(w + L.stage);
  double* gacc = (double*)(w + L.grad);
  HIP_CHECK(hipMemsetAsync(w, 0, L.vjp_total, c->stream), "clear");
  HIP_CHECK(upload_lam(c->p, stage, lam_next, c->stream), "upload");
  HIP_CHECK(lbm::launch_adjoint_cast(c->storage, c->p, stage, w + L.lamA, c->stream), "cast launch");
  const StateView x{c->g(c->cur), c->M(c->cur), c->E(c->cur)};
  const lbm::AdjArgs a = adj_args(c, x, w + L.site, c->k, w + L.lamA, w + L.lamB, 0, w, L);
  if (a.s != c->s) return fail(LBM_ESTATE, "shift count does not match the step count");
  HIP_CHECK(step_with_site(c, c->k, x, state_at(w + L.scratch, c->p, c->storage), w + L.site, c->stream),
            "step launch");
  HIP_CHECK(lbm::launch_adjoint_step(c->storage, a, c->stream), "adjoint launch");
  HIP_CHECK(lbm::launch_adjoint_state(c->storage, a, stage, c->stream), "adjoint state launch");
  HIP_CHECK(lbm::adjoint_reduce(c->p, a.partials, gacc, c->stream), "adjoint reduce");
  HIP_CHECK(download_lam(c->p, lam_out, stage, c->stream), "download");
  HIP_CHECK(hipMemcpyAsync(grad, gacc, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  return LBM_OK;
}

int lbm_vjp_init(lbm_ctx* c, void* ws, size_t bytes, const double* lam0, double grad[4]) {
  if (int rc_ = live(c)) return rc_;
  const AdjLayout L = adj_layout(c->p, c->storage);
  int rc = adj_check(c, ws, bytes, L.vjp_total);
  if (rc) return rc;
  if (!lam0 || !grad) return fail(LBM_EINVAL, "NULL argument");
  if (c->k != 0) return fail(LBM_ESTATE, "lbm_vjp_init needs the initial state (step 0)");
  char* w = (char*)ws;
  double* stage = (double*)(w + L.stage);
  double* gacc = (double*)(w + L.grad);
  HIP_CHECK(hipMemsetAsync(w, 0, L.vjp_total, c->stream), "clear");
  HIP_CHECK(upload_lam(c->p, stage, lam0, c->stream), "upload");
  HIP_CHECK(lbm::launch_adjoint_cast(c->storage, c->p, stage, w + L.lamA, c->stream), "cast launch");
  const StateView x{c->g(c->cur), c->M(c->cur), c->E(c->cur)};
  const lbm::AdjArgs a = adj_args(c, x, nullptr, 0, w + L.lamA, nullptr, 0, w, L);
  HIP_CHECK(lbm::launch_adjoint_init(c->storage, a, c->stream), "adjoint init launch");
  HIP_CHECK(lbm::adjoint_reduce(c->p, a.partials, gacc, c->stream), "adjoint reduce");
  HIP_CHECK(hipMemcpyAsync(grad, gacc, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  return LBM_OK;
}

int lbm_adjoint_workspace_bytes(const lbm_config* cfg, int64_t nsteps, int32_t ckpt_every, size_t* bytes) {
  Physics p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  if (nsteps < 1 || ckpt_every < 1) return fail(LBM_EINVAL, "nsteps and ckpt_every must be >= 1");
  const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  const size_t sb = state_bytes(p, cfg->storage);
  const int64_t seglen = ckpt_every < nsteps ? ckpt_every : nsteps;
  const int64_t nbuf = nseg > 1 ? 2 : 1;   // segment buffers (recompute overlaps the reverse sweep)
  *bytes = adj_layout(p, cfg->storage).core_total + (size_t)nseg * sb +
           (size_t)nbuf * ((size_t)(seglen + 1) * sb + (size_t)seglen * site_bytes(p, cfg->storage));
  return LBM_OK;
}

static int adjoint_run(lbm_ctx* c, const lbm_objective* obj, int64_t nsteps, int32_t ckpt_every, void* ws,
                       size_t bytes, double* J, double grad[4]) {
  if (!obj || !J || !grad) return fail(LBM_EINVAL, "NULL argument");
  if (nsteps < 1 || ckpt_every < 1) return fail(LBM_EINVAL, "nsteps and ckpt_every must be >= 1");
  if (c->k != 0) return fail(LBM_ESTATE, "lbm_adjoint needs the context at its initial state (step 0)");
  size_t need;
  int rc = lbm_adjoint_workspace_bytes(&c->cfg, nsteps, ckpt_every, &need);
  if (rc) return rc;
  rc = adj_check(c, ws, bytes, need);
  if (rc) return rc;
  const Physics& p = c->p;
  if (obj->row < 0 || obj->row >= p.nr) return fail(LBM_EINVAL, "objective row out of range");
  // witness position after nsteps: E^{N-1} at z_d(t_{N-1}) - z_behind
  const long long sN = p.window ? nsteps / p.m : 0;
  const double zstar = p.zd0 + (double)(nsteps - 1) * p.dt - obj->z_behind;
  const double xw = zstar / p.h - (double)sN - 0.5;
  const long long iw = (long long)std::floor(xw);
  if (iw < 0 || iw >= p.nz - 1) return fail(LBM_EINVAL, "witness position outside the window");
  const double ww = xw - (double)iw;

  const AdjLayout L = adj_layout(p, c->storage);
  const size_t sb = state_bytes(p, c->storage);
  const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  char* w = (char*)ws;
  char* ckpt = w + L.core_total;
  const int64_t seglen = ckpt_every < nsteps ? ckpt_every : nsteps;
  const size_t stb = site_bytes(p, c->storage);
  const size_t segbuf = (size_t)(seglen + 1) * sb + (size_t)seglen * stb;
  char* seg[2] = {ckpt + (size_t)nseg * sb, ckpt + (size_t)nseg * sb + segbuf};   // [1] unused if nseg == 1
  char* lam[2] = {w + L.lamA, w + L.lamB};
  double* gacc = (double*)(w + L.grad);
  if (!c->aux) {
    HIP_CHECK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking), "stream create");
    for (hipEvent_t* e : {&c->ev_fwd, &c->ev_rec[0], &c->ev_rec[1], &c->ev_rev[0], &c->ev_rev[1]})
      HIP_CHECK(hipEventCreateWithFlags(e, hipEventDisableTiming), "event create");
  }

  // Forward pass.  x^0 stays in the context's current buffer and is checkpoint 0; each later
  // checkpoint is written by the step that makes it (no copies).  The last segment runs with its
  // site records straight into its segment buffer, so the reverse sweep needs no recompute of it;
  // x^N goes to the context's other buffer, which becomes current when the call ends.
  const int c0 = c->cur;
  const StateView x0{c->g(c0), c->M(c0), c->E(c0)};
  const StateView xN{c->g(1 - c0), c->M(1 - c0), c->E(1 - c0)};
  auto ck_at = [&](int64_t sgi) -> StateView {
    return sgi == 0 ? x0 : state_at(ckpt + (size_t)sgi * sb, p, c->storage);
  };
  {
    // ping-pong states between checkpoints: the context's other buffer and the first slot of the
    // segment buffer that the last segment does not use
    const StateView pp[2] = {xN, state_at(seg[nseg % 2], p, c->storage)};
    StateView src = x0;
    for (int64_t sgi = 0; sgi + 1 < nseg; ++sgi)
      for (int64_t t = 0; t < ckpt_every; ++t) {
        const StateView dst = t == ckpt_every - 1 ? ck_at(sgi + 1) : pp[t % 2];
        HIP_CHECK(step_with_site(c, sgi * ckpt_every + t, src, dst, nullptr, c->stream), "step launch");
        src = dst;
      }
    const int64_t k0 = (nseg - 1) * ckpt_every, len = nsteps - k0;
    char* buf = seg[(nseg - 1) % 2];
    char* sites = buf + (size_t)(seglen + 1) * sb;
    for (int64_t t = 0; t < len; ++t) {
      const StateView dst = t == len - 1 ? xN : state_at(buf + (size_t)(t + 1) * sb, p, c->storage);
      HIP_CHECK(step_with_site(c, k0 + t, src, dst, sites + (size_t)t * stb, c->stream), "step launch");
      src = dst;
    }
  }
  // objective
  {
    const size_t ab = aux_bytes(c->storage);
    const char* ez = (const char*)xN.E + ((size_t)obj->row * p.pitch + (size_t)iw) * ab;
    double e0, e1;
    if (ab == 8) {
      double v[2];
      HIP_CHECK(hipMemcpyAsync(v, ez, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "objective");
      HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
      e0 = v[0]; e1 = v[1];
    } else {
      float v[2];
      HIP_CHECK(hipMemcpyAsync(v, ez, 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream), "objective");
      HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
      e0 = v[0]; e1 = v[1];
    }
    *J = (1.0 - ww) * e0 + ww * e1;
  }
  // seed lambda^N = dJ/dx^N
  HIP_CHECK(hipMemsetAsync(w, 0, L.core_total, c->stream), "clear");
  {
    const size_t ab = aux_bytes(c->storage);
    char* dst = lam[0] + (30 * (size_t)p.plane + (size_t)obj->row * p.pitch + (size_t)iw) * ab;
    const double seedd[2] = {1.0 - ww, ww};
    const float seedf[2] = {(float)(1.0 - ww), (float)ww};
    HIP_CHECK(hipMemcpyAsync(dst, ab == 8 ? (const void*)seedd : (const void*)seedf, 2 * ab,
                             hipMemcpyHostToDevice, c->stream),
              "seed");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  }
  int cur = 0;
  // Reverse sweep, segment by segment.  The recompute of segment sgi - 1 (states from its
  // checkpoint, and the site record of each step) runs on the second stream while the reverse
  // sweep of segment sgi runs on the caller's stream; segments alternate between two buffers.
  // Segments other than the last are full length; their first state is read from the checkpoint,
  // slots 1 .. len - 1 of the buffer hold the later states (slot len is scratch).
  auto recompute = [&](int64_t sgi, char* buf) -> hipError_t {
    const int64_t k0 = sgi * ckpt_every;
    char* sites = buf + (size_t)(seglen + 1) * sb;
    hipError_t e = hipSuccess;
    StateView src = ck_at(sgi);
    for (int64_t t = 0; e == hipSuccess && t < ckpt_every; ++t) {
      const StateView dst = state_at(buf + (size_t)(t + 1) * sb, p, c->storage);
      e = step_with_site(c, k0 + t, src, dst, sites + (size_t)t * stb, c->aux);
      src = dst;
    }
    return e;
  };
  HIP_CHECK(hipEventRecord(c->ev_fwd, c->stream), "event record");
  HIP_CHECK(hipStreamWaitEvent(c->aux, c->ev_fwd, 0), "stream wait");
  // Within the sweep, the cell part of step k and the site part of step k - 1 run as one fused
  // launch; the site part of the last step and the cell part of step 0 run alone.  At a segment
  // boundary the fused launch reads the last state (and site record) of the previous segment,
  // so the caller's stream waits for that segment's recompute first; a segment buffer is
  // released once the cell part of its first step has run.
  auto xs = [&](int64_t k) -> StateView {
    const int64_t sgi = k / ckpt_every;
    if (k == sgi * ckpt_every) return ck_at(sgi);
    return state_at(seg[sgi % 2] + (size_t)(k - sgi * ckpt_every) * sb, p, c->storage);
  };
  auto site_of = [&](int64_t k) -> const void* {
    const int64_t sgi = k / ckpt_every;
    return seg[sgi % 2] + (size_t)(seglen + 1) * sb + (size_t)(k - sgi * ckpt_every) * stb;
  };
  for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
    const int b = (int)(sgi % 2);
    if (sgi >= 1) {
      const int b2 = (int)((sgi - 1) % 2);
      if (sgi + 1 <= nseg - 1)   // buffer b2 last held segment sgi + 1: its reverse sweep must be done
        HIP_CHECK(hipStreamWaitEvent(c->aux, c->ev_rev[b2], 0), "stream wait");
      HIP_CHECK(recompute(sgi - 1, seg[b2]), "recompute launch");
      HIP_CHECK(hipEventRecord(c->ev_rec[b2], c->aux), "event record");
    }
    const int64_t k0 = sgi * ckpt_every;
    const int64_t len = std::min<int64_t>(ckpt_every, nsteps - k0);
    for (int64_t k = k0 + len - 1; k >= k0; --k) {
      if (k == nsteps - 1) {
        const lbm::AdjArgs as = adj_args(c, xs(k), site_of(k), k, lam[cur], lam[1 - cur], 1, w, L, (int)(k % 2));
        HIP_CHECK(lbm::launch_adjoint_site(c->storage, as, c->stream), "adjoint launch");
      }
      // cell part of step k: lambda^{k+1} in lam[cur], lambda^k (populations done) in lam[1 - cur]
      const lbm::AdjArgs ac = adj_args(c, xs(k), nullptr, k, lam[cur], lam[1 - cur], 1, w, L, (int)(k % 2));
      if (k >= 1) {
        if (k == k0) HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_rec[(sgi - 1) % 2], 0), "stream wait");
        const lbm::AdjArgs as = adj_args(c, xs(k - 1), site_of(k - 1), k - 1, lam[1 - cur], lam[cur], 1, w, L,
                                         (int)((k - 1) % 2));
        HIP_CHECK(lbm::launch_adjoint_fused(c->storage, ac, as, c->stream), "adjoint launch");
      } else {
        HIP_CHECK(lbm::launch_adjoint_cell(c->storage, ac, c->stream), "adjoint launch");
      }
      cur ^= 1;
    }
    HIP_CHECK(hipEventRecord(c->ev_rev[b], c->stream), "event record");
  }
  // initial state
  {
    const lbm::AdjArgs a = adj_args(c, x0, nullptr, 0, lam[cur], nullptr, 1, w, L);
    HIP_CHECK(lbm::launch_adjoint_init(c->storage, a, c->stream), "adjoint init launch");
    HIP_CHECK(lbm::adjoint_reduce(c->p, a.partials, gacc, c->stream), "adjoint reduce");
  }
  HIP_CHECK(hipMemcpyAsync(grad, gacc, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  // the context now holds x^N
  c->cur = 1 - c0;
  c->k = nsteps;
  c->s = sN;
  return LBM_OK;
}

int lbm_adjoint(lbm_ctx* c, const lbm_objective* obj, int64_t nsteps, int32_t ckpt_every, void* ws,
                size_t bytes, double* J, double grad[4]) {
  if (int rc_ = live(c)) return rc_;
  const int rc = adjoint_run(c, obj, nsteps, ckpt_every, ws, bytes, J, grad);
  if (rc != LBM_OK) {
    // work queued before the failure may still be running on either stream and writing into the
    // caller's workspace: wait for it, so the caller can free the workspace on return (the
    // context's own state, x^0, is only read by this call)
    const std::string msg = g_err;
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    (void)hipStreamSynchronize(c->stream);
    g_err = msg;
  }
  return rc;
}

// ------------------------------------------------------------------------------------------
// Adjoint with a snapshot budget: binomial (revolve-type) checkpointing.
// ------------------------------------------------------------------------------------------
namespace {

// beta(s, t) = C(s + t, s): the longest step range that s snapshots reverse with every step
// advanced at most t times (Griewank's binomial bound); saturates at 2^62.
int64_t beta(int64_t s, int64_t t) {
  double v = 1.0;
  for (int64_t i = 1; i <= t; ++i) {
    v = v * (double)(s + i) / (double)i;
    if (v > 4.6e18) return (int64_t)1 << 62;
  }
  return (int64_t)(v + 0.5);
}

struct Revolve {
  lbm_ctx* c;
  const AdjLayout* L;
  char* w;
  char* snaps;     // snapshot slots, one state each
  char* sites;     // site record of the step being reversed
  size_t sb;
  char* lam[2];
  int cur;
  int64_t nsteps;
  int32_t row;
  long long iw;
  double ww, J;
  int64_t advanced;   // forward steps taken (statistics)

  StateView slot(int i) const { return state_at(snaps + (size_t)i * sb, c->p, c->storage); }
  StateView ctxbuf(int b) const { return StateView{c->g(b), c->M(b), c->E(b)}; }

  lbm::StepArgs step_args(int64_t k, const StateView& x, const StateView& y, void* site) const {
    lbm::StepArgs a;
    a.p = c->p;
    a.k = k;
    a.s = c->p.window ? k / c->p.m : 0;
    a.shift = (c->p.window && (k + 1) % c->p.m == 0) ? 1 : 0;
    a.g_in = x.g; a.g_out = y.g;
    a.M_in = x.M; a.M_out = y.M;
    a.E_in = x.E; a.E_out = y.E;
    a.site_out = site;
    return a;
  }

  // x^{from} (in snapshot slot src) advanced to x^{to}, to > from: into snapshot slot dst if
  // dst >= 0, else into one of the context's two buffers, whose index goes to *where.
  // Intermediate states alternate between the context's buffers (never in place).
  int advance(int64_t from, int64_t to, int src, int dst, int* where = nullptr) {
    StateView x = slot(src);
    int b = 0;
    for (int64_t k = from; k < to; ++k) {
      const bool last = k + 1 == to;
      const StateView y = (last && dst >= 0) ? slot(dst) : ctxbuf(b);
      HIP_CHECK(lbm::launch_step(c->storage, step_args(k, x, y, nullptr), c->stream), "step launch");
      if (last && dst < 0 && where) *where = b;
      x = y;
      b ^= 1;
      ++advanced;
    }
    return LBM_OK;
  }

  // reverse step k from x^k (in x): the step again with its site record saved (its output, x^{k+1},
  // gives J when k = N - 1), then the reverse kernels
  int reverse_step(int64_t k, const StateView& x) {
    const StateView y = (x.g == c->g(0)) ? ctxbuf(1) : ctxbuf(0);   // not x itself
    HIP_CHECK(lbm::launch_step(c->storage, step_args(k, x, y, sites), c->stream), "step launch");
    ++advanced;
    if (k == nsteps - 1) {
      const size_t ab = aux_bytes(c->storage);
      const char* ez = (const char*)y.E + ((size_t)row * c->p.pitch + (size_t)iw) * ab;
      double e[2];
      if (ab == 8) {
        HIP_CHECK(hipMemcpyAsync(e, ez, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "objective");
      } else {
        float f[2];
        HIP_CHECK(hipMemcpyAsync(f, ez, 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream), "objective");
        HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
        e[0] = f[0];
        e[1] = f[1];
      }
      HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
      J = (1.0 - ww) * e[0] + ww * e[1];
    }
    const lbm::AdjArgs a = adj_args(c, x, sites, k, lam[cur], lam[1 - cur], 1, w, *L);
    HIP_CHECK(lbm::launch_adjoint_step(c->storage, a, c->stream), "adjoint launch");
    cur ^= 1;
    return LBM_OK;
  }

  // lambda^a from lambda^b, with x^a in snapshot slot `sa` and the slots above it free (nfree).
  // The later part of a range recurses with one snapshot fewer (depth <= nfree); the earlier
  // part continues in the loop.
  int reverse(int64_t a, int64_t b, int sa, int nfree) {
    for (;;) {
      const int64_t l = b - a;
      if (l == 1) return reverse_step(a, slot(sa));
      if (nfree == 0) {
        // no snapshot left: advance from x^a for every step of the range
        for (int64_t k = b - 1; k > a; --k) {
          int where = 0;
          int rc = advance(a, k, sa, -1, &where);
          if (rc) return rc;
          rc = reverse_step(k, ctxbuf(where));
          if (rc) return rc;
        }
        return reverse_step(a, slot(sa));
      }
      int64_t t = 1;
      while (beta(nfree, t) < l) ++t;
      const int64_t m = b - std::min<int64_t>(beta(nfree - 1, t), l - 1);
      int rc = advance(a, m, sa, sa + 1);
      if (rc) return rc;
      rc = reverse(m, b, sa + 1, nfree - 1);
      if (rc) return rc;
      b = m;
    }
  }
};

}  // namespace

int lbm_adjoint_revolve_workspace_bytes(const lbm_config* cfg, int32_t snapshots, size_t* bytes) {
  Physics p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  if (snapshots < 1) return fail(LBM_EINVAL, "snapshots must be >= 1");
  *bytes = adj_layout(p, cfg->storage).core_total + (size_t)snapshots * state_bytes(p, cfg->storage) +
           site_bytes(p, cfg->storage);
  return LBM_OK;
}

// *snap0 is set once snapshot 0 (a copy of the context's state) is queued: from then on the
// context's buffers are scratch and must be restored from it.
static int revolve_run(lbm_ctx* c, const lbm_objective* obj, int64_t nsteps, int32_t snapshots, void* ws,
                       size_t bytes, double* J, double grad[4], int64_t* steps_advanced, bool* snap0) {
  if (!obj || !J || !grad) return fail(LBM_EINVAL, "NULL argument");
  if (nsteps < 1 || snapshots < 1) return fail(LBM_EINVAL, "nsteps and snapshots must be >= 1");
  if (c->k != 0) return fail(LBM_ESTATE, "lbm_adjoint_revolve needs the context at its initial state (step 0)");
  size_t need;
  int rc = lbm_adjoint_revolve_workspace_bytes(&c->cfg, snapshots, &need);
  if (rc) return rc;
  rc = adj_check(c, ws, bytes, need);
  if (rc) return rc;
  const Physics& p = c->p;
  if (obj->row < 0 || obj->row >= p.nr) return fail(LBM_EINVAL, "objective row out of range");
  const long long sN = p.window ? nsteps / p.m : 0;
  const double zstar = p.zd0 + (double)(nsteps - 1) * p.dt - obj->z_behind;
  const double xw = zstar / p.h - (double)sN - 0.5;
  const long long iw = (long long)std::floor(xw);
  if (iw < 0 || iw >= p.nz - 1) return fail(LBM_EINVAL, "witness position outside the window");

  const AdjLayout L = adj_layout(p, c->storage);
  Revolve r;
  r.c = c;
  r.L = &L;
  r.w = (char*)ws;
  r.sb = state_bytes(p, c->storage);
  r.snaps = r.w + L.core_total;
  r.sites = r.snaps + (size_t)snapshots * r.sb;
  r.lam[0] = r.w + L.lamA;
  r.lam[1] = r.w + L.lamB;
  r.cur = 0;
  r.nsteps = nsteps;
  r.row = obj->row;
  r.iw = iw;
  r.ww = xw - (double)iw;
  r.J = 0.0;
  r.advanced = 0;
  // snapshot 0 = x^0 (the context's state); lambda^N = dJ/dx^N
  const size_t gbytes = round_up(27 * (size_t)p.plane * pop_bytes(c->storage), 256);
  const size_t mbytes = round_up(3 * (size_t)p.plane * aux_bytes(c->storage), 256);
  const size_t ebytes = round_up(field_bytes((size_t)p.plane, c->storage), 256);
  const StateView x0 = r.slot(0), ctx0{c->g(c->cur), c->M(c->cur), c->E(c->cur)};
  HIP_CHECK(hipMemcpyAsync(x0.g, ctx0.g, gbytes, hipMemcpyDeviceToDevice, c->stream), "snapshot");
  HIP_CHECK(hipMemcpyAsync(x0.M, ctx0.M, mbytes, hipMemcpyDeviceToDevice, c->stream), "snapshot");
  HIP_CHECK(hipMemcpyAsync(x0.E, ctx0.E, ebytes, hipMemcpyDeviceToDevice, c->stream), "snapshot");
  *snap0 = true;
  HIP_CHECK(hipMemsetAsync(r.w, 0, L.core_total, c->stream), "clear");
  {
    const size_t ab = aux_bytes(c->storage);
    char* dst = r.lam[0] + (30 * (size_t)p.plane + (size_t)obj->row * p.pitch + (size_t)iw) * ab;
    const double seedd[2] = {1.0 - r.ww, r.ww};
    const float seedf[2] = {(float)(1.0 - r.ww), (float)r.ww};
    HIP_CHECK(hipMemcpyAsync(dst, ab == 8 ? (const void*)seedd : (const void*)seedf, 2 * ab,
                             hipMemcpyHostToDevice, c->stream),
              "seed");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  }
  rc = r.reverse(0, nsteps, 0, snapshots - 1);
  if (rc) return rc;
  {
    const lbm::AdjArgs a = adj_args(c, x0, nullptr, 0, r.lam[r.cur], nullptr, 1, r.w, L);
    HIP_CHECK(lbm::launch_adjoint_init(c->storage, a, c->stream), "adjoint init launch");
    HIP_CHECK(lbm::adjoint_reduce(p, a.partials, (double*)(r.w + L.grad), c->stream), "adjoint reduce");
  }
  // the context's buffers served as scratch: restore the initial state
  HIP_CHECK(hipMemcpyAsync(ctx0.g, x0.g, gbytes, hipMemcpyDeviceToDevice, c->stream), "restore");
  HIP_CHECK(hipMemcpyAsync(ctx0.M, x0.M, mbytes, hipMemcpyDeviceToDevice, c->stream), "restore");
  HIP_CHECK(hipMemcpyAsync(ctx0.E, x0.E, ebytes, hipMemcpyDeviceToDevice, c->stream), "restore");
  HIP_CHECK(hipMemcpyAsync(grad, r.w + L.grad, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  *J = r.J;
  if (steps_advanced) *steps_advanced = r.advanced;
  return LBM_OK;
}

int lbm_adjoint_revolve(lbm_ctx* c, const lbm_objective* obj, int64_t nsteps, int32_t snapshots, void* ws,
                        size_t bytes, double* J, double grad[4], int64_t* steps_advanced) {
  if (int rc_ = live(c)) return rc_;
  bool snap0 = false;
  const int rc = revolve_run(c, obj, nsteps, snapshots, ws, bytes, J, grad, steps_advanced, &snap0);
  if (rc != LBM_OK) {
    // drain what was queued, then put the initial state back from snapshot 0; if that fails too,
    // the context refuses further use until a state is set or loaded
    const std::string msg = g_err;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (snap0) {
      const Physics& p = c->p;
      const size_t gbytes = round_up(27 * (size_t)p.plane * pop_bytes(c->storage), 256);
      const size_t mbytes = round_up(3 * (size_t)p.plane * aux_bytes(c->storage), 256);
      const size_t ebytes = round_up(field_bytes((size_t)p.plane, c->storage), 256);
      const StateView x0 = state_at((char*)ws + adj_layout(p, c->storage).core_total, p, c->storage);
      if (e == hipSuccess) e = hipMemcpyAsync(c->g(c->cur), x0.g, gbytes, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(c->M(c->cur), x0.M, mbytes, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(c->E(c->cur), x0.E, ebytes, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) c->broken = true;
    }
    g_err = msg;
  }
  return rc;
}

int lbm_witness(lbm_ctx* c, const lbm_objective* obj, double* J) {
  if (int rc_ = live(c)) return rc_;
  if (!obj || !J) return fail(LBM_EINVAL, "NULL argument");
  const Physics& p = c->p;
  if (c->k < 1) return fail(LBM_ESTATE, "the witness needs at least one step (E at t_{k-1})");
  if (obj->row < 0 || obj->row >= p.nr) return fail(LBM_EINVAL, "objective row out of range");
  // E^{k-1} at z_d(t_{k-1}) - z_behind, in the window's frame after s shifts
  const double zstar = p.zd0 + (double)(c->k - 1) * p.dt - obj->z_behind;
  const double xw = zstar / p.h - (double)c->s - 0.5;
  const double fl = std::floor(xw);
  if (!(fl >= 0.0 && fl < (double)(p.nz - 1))) return fail(LBM_EINVAL, "witness position outside the window");
  const long long iw = (long long)fl;
  const double ww = xw - fl;
  const size_t ab = aux_bytes(c->storage);
  const char* ez = (const char*)c->E(c->cur) + ((size_t)obj->row * p.pitch + (size_t)iw) * ab;
  double e[2];
  if (ab == 8) {
    HIP_CHECK(hipMemcpyAsync(e, ez, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "download");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  } else {
    float f[2];
    HIP_CHECK(hipMemcpyAsync(f, ez, 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream), "download");
    HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
    e[0] = f[0];
    e[1] = f[1];
  }
  *J = (1.0 - ww) * e[0] + ww * e[1];
  return LBM_OK;
}

int lbm_bubble_length(lbm_ctx* c, int32_t row, double n_star, double z_from, double z_to, int64_t* count,
                      double* length) {
  if (int rc_ = live(c)) return rc_;
  if (!count) return fail(LBM_EINVAL, "count is NULL");
  if (row < 0 || row >= c->p.nr) return fail(LBM_EINVAL, "row out of range");
  if (!(n_star > 0.0) || !std::isfinite(n_star)) return fail(LBM_EINVAL, "n_star must be positive");
  if (std::isnan(z_from) || std::isnan(z_to)) return fail(LBM_EINVAL, "z range is NaN");
  long long* d = (long long*)c->red_out();
  HIP_CHECK(lbm::launch_bubble(c->storage, c->p, c->s, c->M(c->cur), row, n_star, z_from, z_to, d, c->stream),
            "bubble launch");
  long long h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, c->stream), "download");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  *count = h;
  if (length) *length = (double)h * c->p.h;
  return LBM_OK;
}

int lbm_counters(lbm_ctx* c, int64_t* step, int64_t* shifts) {
  if (!c) return fail(LBM_ESTATE, "context is NULL");
  if (step) *step = c->k;
  if (shifts) *shifts = c->s;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return fail(LBM_ESTATE, "context is NULL");
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (hipEvent_t e : {c->ev_fwd, c->ev_rec[0], c->ev_rec[1], c->ev_rev[0], c->ev_rev[1]})
    if (e) (void)hipEventDestroy(e);
  delete c;
  return LBM_OK;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Particle driver: the bunch
// ------------------------------------------------------------------------------------------
namespace {
int set_bunch(lbm_ctx* c, int64_t n, const double* bunch, int32_t init_fields);
int get_bunch(lbm_ctx* c, double* bunch, int64_t n_max, int64_t* n);
}  // namespace

int lbm_set_bunch(lbm_ctx* c, int64_t n, const double* bunch, int32_t init_fields) {
  try {
    return set_bunch(c, n, bunch, init_fields);
  } catch (const std::bad_alloc&) {
    return fail(LBM_ENOMEM, "host allocation failed");
  }
}

int lbm_get_bunch(lbm_ctx* c, double* bunch, int64_t n_max, int64_t* n) {
  try {
    return get_bunch(c, bunch, n_max, n);
  } catch (const std::bad_alloc&) {
    return fail(LBM_ENOMEM, "host allocation failed");
  }
}

namespace {

int set_bunch(lbm_ctx* c, int64_t n, const double* bunch, int32_t init_fields) {
  if (int rc_ = live(c)) return rc_;
  if (c->p.driver != LBM_DRIVER_PARTICLES) return fail(LBM_EINVAL, "the bunch needs driver = LBM_DRIVER_PARTICLES");
  if (n < 0 || n > c->p.cap) return fail(LBM_EINVAL, "n must lie in [0, max_particles] (got %lld)", (long long)n);
  if (n > 0 && !bunch) return fail(LBM_EINVAL, "bunch is NULL");
  if (init_fields != 0 && init_fields != 1) return fail(LBM_EINVAL, "init_fields must be 0 or 1");
  if (init_fields && c->k != 0) return fail(LBM_EINVAL, "the initial field can only be set at step 0");
  for (int64_t i = 0; i < 7 * n; ++i)
    if (!std::isfinite(bunch[i])) return fail(LBM_EINVAL, "bunch value %lld is not finite", (long long)i);
  for (int64_t i = 0; i < n; ++i)
    if (bunch[6 * n + i] < 0.0) return fail(LBM_EINVAL, "particle %lld has a negative weight", (long long)i);
  // stored by grid column of z and, within a column, by radius: the 64 particles of a wavefront
  // then share a few rows and columns, so that their field gathers and current deposits touch
  // few cache lines, and a thread block's deposit fits its LDS tile
  std::vector<double> col((size_t)n), rad((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    col[(size_t)i] = std::floor(bunch[2 * n + i] / c->p.h);
    rad[(size_t)i] = bunch[i] * bunch[i] + bunch[n + i] * bunch[n + i];
  }
  std::vector<int64_t> order((size_t)n);
  std::iota(order.begin(), order.end(), (int64_t)0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return col[(size_t)a] < col[(size_t)b] || (col[(size_t)a] == col[(size_t)b] && rad[(size_t)a] < rad[(size_t)b]);
  });
  std::vector<double> sorted((size_t)(7 * n));
  for (int comp = 0; comp < 7; ++comp)
    for (int64_t i = 0; i < n; ++i) sorted[(size_t)(comp * n + i)] = bunch[comp * n + order[(size_t)i]];
  std::vector<int32_t> pid((size_t)n);
  for (int64_t i = 0; i < n; ++i) pid[(size_t)i] = (int32_t)order[(size_t)i];
  for (int comp = 0; comp < 8 && n > 0; ++comp) {
    const hipError_t e =
        comp < 7 ? hipMemcpyAsync(c->bunch() + comp * c->p.cap, sorted.data() + comp * n,
                                  (size_t)n * sizeof(double), hipMemcpyHostToDevice, c->stream)
                 : hipMemcpyAsync(c->pid(c->bcur), pid.data(), (size_t)n * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(c->stream);   // copies already queued read `sorted` and `pid`
      c->nbunch = 0;                           // the device bunch is now partly overwritten
      return hip_fail(e, "bunch upload");
    }
  }
  // the deposit buffers may hold the previous bunch's current, outside the new bunch's bound
  for (int b = 0; b < 2; ++b)
    HIP_CHECK(hipMemsetAsync(c->jb(b), 0, 2 * (size_t)c->p.plane * aux_bytes(c->storage), c->stream), "clear");
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");   // before the host buffers go
  c->nbunch = n;
  c->ext[0] = INT32_MAX;
  c->ext[1] = c->ext[2] = INT32_MIN;
  for (int64_t i = 0; i < n; ++i) {
    if (bunch[6 * n + i] == 0.0) continue;
    const double u = std::min(std::max(std::floor(bunch[2 * n + i] / c->p.h), -1e9), 1e9);
    const double v = std::min(std::floor(std::sqrt(bunch[i] * bunch[i] + bunch[n + i] * bunch[n + i]) / c->p.h), 1e9);
    c->ext[0] = std::min(c->ext[0], (int)u);
    c->ext[1] = std::max(c->ext[1], (int)u);
    c->ext[2] = std::max(c->ext[2], (int)v);
  }
  c->ext_age = 0;
  if (init_fields && c->p.fields_on) {
    // E_r^{-1} from the density at the positions (t = -dt) on the E_r columns; B^{-1/2} from the
    // density at t = -dt/2 on the B columns
    const size_t db = (size_t)c->p.plane * sizeof(double);
    for (int comp = 1; comp <= 2; ++comp) {
      HIP_CHECK(hipMemsetAsync(c->dens(), 0, db, c->stream), "clear");
      HIP_CHECK(lbm::launch_bunch_density(c->p, 0, comp == 1 ? 0.0 : 0.5, comp == 1 ? 0.0 : 0.5 * c->p.dt,
                                          c->bunch(), (int)n, c->p.cap, c->dens(), c->stream),
                "bunch density launch");
      HIP_CHECK(lbm::launch_bunch_gauss(c->storage, c->p, c->dens(), c->E(c->cur), comp, c->stream),
                "bunch field launch");
    }
  }
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  return LBM_OK;
}

int get_bunch(lbm_ctx* c, double* bunch, int64_t n_max, int64_t* n) {
  if (int rc_ = live(c)) return rc_;
  if (c->p.driver != LBM_DRIVER_PARTICLES) return fail(LBM_EINVAL, "the bunch needs driver = LBM_DRIVER_PARTICLES");
  if (!n) return fail(LBM_EINVAL, "n is NULL");
  if (n_max < c->nbunch) return fail(LBM_EINVAL, "n_max %lld < %lld particles", (long long)n_max, c->nbunch);
  if (c->nbunch > 0 && !bunch) return fail(LBM_EINVAL, "bunch is NULL");
  const long long nb = c->nbunch;
  std::vector<double> stored((size_t)(7 * nb));
  std::vector<int32_t> pid((size_t)nb);
  for (int comp = 0; comp < 8 && nb > 0; ++comp) {
    const hipError_t e =
        comp < 7 ? hipMemcpyAsync(stored.data() + comp * nb, c->bunch() + comp * c->p.cap,
                                  (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, c->stream)
                 : hipMemcpyAsync(pid.data(), c->pid(c->bcur), (size_t)nb * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(c->stream);   // copies already queued write `stored` and `pid`
      return hip_fail(e, "bunch download");
    }
  }
  HIP_CHECK(hipStreamSynchronize(c->stream), "synchronise");
  // back to the caller's order; the indices are a permutation of [0, nb) (checked, so that a
  // damaged index array is reported rather than followed)
  std::vector<char> seen((size_t)nb, 0);
  for (long long i = 0; i < nb; ++i) {
    const int32_t o = pid[(size_t)i];
    if (o < 0 || o >= nb || seen[(size_t)o]) return fail(LBM_ESTATE, "bunch index %lld is not a permutation", i);
    seen[(size_t)o] = 1;
  }
  for (int comp = 0; comp < 7; ++comp)
    for (long long i = 0; i < nb; ++i) bunch[comp * nb + pid[(size_t)i]] = stored[(size_t)(comp * nb + i)];
  *n = nb;
  return LBM_OK;
}

}  // namespace
