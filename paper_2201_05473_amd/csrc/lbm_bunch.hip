// Particle driver (gfx950): the electron bunch as macroparticles of Sec. II, Eq. (1), coupled to
// the grid through its projected current.
//
// The bunch is stored as SoA doubles [7][cap]: x, y, z (lab frame), p_x, p_y, p_z (m_e c units),
// w (electrons, n_0 / k_p^3).  After k steps the positions are at t_{k-1} and the momenta at
// t_{k-1/2}.  Step k runs:
//   bunch_move_kernel  positions to t_k, current w beta at the midpoints -> J_b(t_{k-1/2}) (z at the
//                      E_z points, r at the E_r points): the shares of neighbouring lanes that
//                      start at the same node summed within the wavefront, then per block in LDS
//                      when the block's particles span few columns (the bunch is stored by column
//                      of z, then by radius: sorted on upload, and again on the device every few
//                      hundred steps as the particles drift apart), then added to the grid with
//                      hardware float atomics;
//   (the step kernel reads J_b in Ampere's law)
//   bunch_push_kernel  Boris push of the momenta to t_{k+1/2} with E^k and
//                      B^k = (B^{k-1/2} + B^{k+1/2}) / 2 at the positions at t_k.
// Between two steps of one lbm_step call the push of step k and the move of step k + 1 run as one
// launch (bunch_move_kernel<ST, true>): each particle's push and move are independent of the
// other particles, and the deposit goes to the buffer that step k has just cleared.
// Projection and interpolation share one stencil: linear in z onto the field's own points, linear
// in r between its rows, rows r_j = (j + 1/2) dr for E_z and densities (the row below the axis folds
// onto row 0) or (j + 1) dr for E_r and B_theta (zero on the axis; the share below the first row is
// dropped).  A particle whose stencil leaves columns [1, nz - 2] or the rows is lost: weight zero,
// no longer moved.  One thread per particle; the bunch is small next to the grid.
#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

// threads per block of the particle kernels: one wavefront (measured on C2 with 200,000 particles:
// 64 -> 79.7 us per step, 128 -> 80.1, 256 -> 83.0, 512 -> 85.4, 1024 -> 88.9)
constexpr int BT = 64;
constexpr double TWO_PI = 6.283185307179586;

struct Stencil {
  int i0, j0;     // lower node column and row
  double fz, fr;  // weight of the upper node in z and in r
};

// Nodes z = (s + i + zoff) dz and rows (j + 1/2) dr (edge = false) or (j + 1) dr (edge = true);
// ih = 1 / dz, computed once per thread by the caller.
__device__ __forceinline__ Stencil stencil(double ih, double z, double r, long long s, double zoff, bool edge) {
  const double u = z * ih - (double)s - zoff;
  const double v = r * ih - (edge ? 1.0 : 0.5);
  const double fi = floor(u), fj = floor(v);
  Stencil st;
  st.i0 = (int)fi;
  st.j0 = (int)fj;
  st.fz = u - fi;
  st.fr = v - fj;
  return st;
}

__device__ __forceinline__ bool inside(const Physics& p, const Stencil& st) {
  return st.i0 >= 1 && st.i0 + 1 <= p.nz - 2 && st.j0 >= -1 && st.j0 + 1 <= p.nr - 1;
}

__device__ __forceinline__ void atomic_add(float* a, double v) { unsafeAtomicAdd(a, (float)v); }
__device__ __forceinline__ void atomic_add(double* a, double v) { unsafeAtomicAdd(a, v); }

// Adds val, spread over the stencil's nodes and divided by each node's annular volume
// 2 pi r_node dz dr, to the pitched plane F.
template <typename T>
__device__ __forceinline__ void deposit(const Physics& p, const Stencil& st, bool edge, double val, T* F) {
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    int j = st.j0 + dj;
    if (j < 0) {
      if (edge) continue;   // the axis node of E_r / J_r carries nothing
      j = 0;                // the row below the axis folds onto row 0
    }
    const double rn = ((double)j + (edge ? 1.0 : 0.5)) * p.h;
    const double vr = val * (dj ? st.fr : 1.0 - st.fr) / (TWO_PI * rn * p.h * p.h);
#pragma unroll
    for (int di = 0; di < 2; ++di)
      atomic_add(F + (long long)j * p.pitch + (st.i0 + di), vr * (di ? st.fz : 1.0 - st.fz));
  }
}

// F at the particle with the stencil's weights; col_shift maps the stencil's columns to the array's
// (1 for an array written after a window shift).  The row below the axis is row 0 for the E_z
// points and zero for the edge points (its weight is zeroed; the load reads row 0, in range).
// No branches: the four loads issue together.
// F is one plane, addressed through a buffer resource with 32-bit element offsets.
template <typename A>
__device__ __forceinline__ double gather(const Physics& p, const Stencil& st, bool edge, Rsrc F, int col_shift) {
  const uint32_t c = (uint32_t)(st.i0 - col_shift);
  const uint32_t o0 = (uint32_t)(st.j0 < 0 ? 0 : st.j0) * (uint32_t)p.pitch + c;
  const uint32_t o1 = (uint32_t)(st.j0 + 1) * (uint32_t)p.pitch + c;
  const double f00 = (double)bload<A>(F, o0), f10 = (double)bload<A>(F, o0 + 1);
  const double f01 = (double)bload<A>(F, o1), f11 = (double)bload<A>(F, o1 + 1);
  const double wr0 = (edge && st.j0 < 0) ? 0.0 : 1.0 - st.fr, wr1 = st.fr;
  const double wz0 = 1.0 - st.fz, wz1 = st.fz;
  double out = 0.0;
  out = out + wz0 * wr0 * f00;
  out = out + wz0 * wr1 * f01;
  out = out + wz1 * wr0 * f10;
  out = out + wz1 * wr1 * f11;
  return out;
}

// LDS tile of the deposit privatisation: the J_z and J_r shares of a block's particles are summed
// here first when they fall in at most TW consecutive columns and TRW consecutive rows (the bunch
// is kept ordered by column, then radius, so a block's particles share a few columns and a band
// of rows), then added to the grid once per touched cell.  The tile is packed to the block's own
// extent: row-major, nc columns wide from column c0 and row r0.
// Rows: 192 (12 KB of FP32 tiles per block, 13 blocks per CU); measured with 200,000 particles, 128
// rows sent more blocks of the paper's finer grid (preset P, the bunch over ~100 rows) to the
// direct-atomic path: 79.9 against 76.1 us per step there, C2 79.8 against 80.3.
constexpr int TW = 8, TRW = 192;
// Particles per thread of the move kernel (a block moves PPT * BT consecutive particles).  Measured
// on C2 with 200,000 particles: 1 is best (2: +1.5 %, 4: +12 %); with 10^6 particles 2 gains 2 %.
constexpr int PPT = 1;

// Lane shifts of the data-parallel primitives (DPP) for the segmented sums below; lanes whose source
// lies outside the pattern read zero.  ROW_SHR(k): lane l reads lane l - k of its row of 16;
// BCAST15: rows 1 and 3 read the last lane of the row before; BCAST31: rows 2 and 3 read lane 31.
constexpr int ROW_SHR1 = 0x111, ROW_SHR2 = 0x112, ROW_SHR4 = 0x114, ROW_SHR8 = 0x118;
constexpr int BCAST15 = 0x142, BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Inclusive sum of v over the lanes of the run of equal keys that ends at this lane (pos: this
// lane's distance from the start of its run).  Every lane of the wavefront must take part, and
// every shift runs on all of them: a lane shift reads nothing from a lane switched off, so the
// shifted value is taken unconditionally and weighted by 0 or 1 (a select would let the compiler
// move the shift under a branch).  The values are finite.
template <typename V>
__device__ __forceinline__ V run_sum(V v, int pos, int lane) {
  V y = dpp<ROW_SHR1, 0xf>(v);
  v += y * (V)(pos >= 1);
  y = dpp<ROW_SHR2, 0xf>(v);
  v += y * (V)(pos >= 2);
  y = dpp<ROW_SHR4, 0xf>(v);
  v += y * (V)(pos >= 4);
  y = dpp<ROW_SHR8, 0xf>(v);
  v += y * (V)(pos >= 8);
  y = dpp<BCAST15, 0xa>(v);
  v += y * (V)(pos > (lane & 15) && (lane & 16));
  y = dpp<BCAST31, 0xc>(v);
  v += y * (V)(pos > lane - 32 && lane >= 32);
  return v;
}

// Adds the shares of val over the stencil's nodes to the packed tile (row-major, nc columns from
// column c0 and row r0).  The E_r points' row below the axis carries nothing; the E_z points' folds
// onto row 0.  Lanes whose stencils start at the same node and are neighbours in the wavefront
// (the bunch is stored by cell, so runs are long) first sum their four node shares; the last lane
// of each run adds the sums, so one LDS atomic serves the run.  Every lane of the wavefront takes
// part (live = false: no particle).
// FP64 tiles (FP64 storage) take the shares in FP64, as the oracle (the run's sum is divided by
// the node volume once); FP32 tiles in FP32 with the hardware reciprocal (1 ulp), below the FP32
// rounding of the stored current.
template <typename T>
__device__ __forceinline__ void deposit_tile(const Physics& p, const Stencil& st, bool edge, double val, bool live,
                                             T* tile, int c0, int r0, int nc) {
  const int lane = threadIdx.x % 64;
  const int key = live ? (st.j0 - r0 + 1) * TW + (st.i0 - c0) : -1;
  const int prev = __shfl_up(key, 1, 64);
  const unsigned long long heads = __ballot(lane == 0 || prev != key);
  const int pos = lane - (63 - __clzll(heads & (~0ull >> (63 - lane))));
  const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
  const T v = live ? (T)val : T(0), fr = (T)st.fr, fz = (T)st.fz;
  const T a0 = v * (T(1) - fr), a1 = v * fr;
  const T s00 = run_sum(a0 * (T(1) - fz), pos, lane), s01 = run_sum(a0 * fz, pos, lane);
  const T s10 = run_sum(a1 * (T(1) - fz), pos, lane), s11 = run_sum(a1 * fz, pos, lane);
  if (!tail || key < 0) return;
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    const int j = st.j0 + dj;
    if (edge && j < 0) continue;
    const int jj = j < 0 ? 0 : j;
    T* row = tile + (jj - r0) * nc + (st.i0 - c0);
    const T lo = dj ? s10 : s00, hi = dj ? s11 : s01;
    if constexpr (std::is_same<T, double>::value) {
      // val / (2 pi r_node dz dr) with r_node = (jj + 1 or 1/2) dr
      const double vol = TWO_PI * (((double)jj + (edge ? 1.0 : 0.5)) * p.h) * p.h * p.h;
      atomicAdd(row, lo / vol);
      atomicAdd(row + 1, hi / vol);
    } else {
      const float k = (float)(1.0 / (TWO_PI * p.h * p.h * p.h)) *
                      __builtin_amdgcn_rcpf((float)jj + (edge ? 1.f : 0.5f));
      atomicAdd(row, lo * k);
      atomicAdd(row + 1, hi * k);
    }
  }
}

// Wavefront minimum / maximum, the same in every lane (all 64 lanes take part): a scan with the
// lane shifts above (lanes outside a shift's pattern read the identity), whose last lane holds the
// result.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dppi(int identity, int v) {
  return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, dppi<ROW_SHR1, 0xf>(INT32_MAX, v));
  v = min(v, dppi<ROW_SHR2, 0xf>(INT32_MAX, v));
  v = min(v, dppi<ROW_SHR4, 0xf>(INT32_MAX, v));
  v = min(v, dppi<ROW_SHR8, 0xf>(INT32_MAX, v));
  v = min(v, dppi<BCAST15, 0xa>(INT32_MAX, v));
  v = min(v, dppi<BCAST31, 0xc>(INT32_MAX, v));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max(int v) {
  v = max(v, dppi<ROW_SHR1, 0xf>(INT32_MIN, v));
  v = max(v, dppi<ROW_SHR2, 0xf>(INT32_MIN, v));
  v = max(v, dppi<ROW_SHR4, 0xf>(INT32_MIN, v));
  v = max(v, dppi<ROW_SHR8, 0xf>(INT32_MIN, v));
  v = max(v, dppi<BCAST15, 0xa>(INT32_MIN, v));
  v = max(v, dppi<BCAST31, 0xc>(INT32_MIN, v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Boris push for dp/dt = -(E + beta x B) of one particle at (x, y, z) (positions at t_k, frame s):
// E^k from Eout (frame s + shift), B^k the mean of B^{k-1/2} (Ein, frame s) and B^{k+1/2} (Eout);
// the momenta go from t_{k-1/2} to t_{k+1/2}.
template <typename A>
__device__ __forceinline__ void boris_push(const Physics& p, long long s, int shift, const A* Ein, const A* Eout,
                                           double x, double y, double z, double& px, double& py, double& pz) {
  const double ih = 1.0 / p.h;
  const double r = sqrt(x * x + y * y);
  const Stencil sc = stencil(ih, z, r, s, 0.5, false);   // E_z points
  const Stencil se = stencil(ih, z, r, s, 0.0, true);    // E_r points
  const Stencil sb = stencil(ih, z, r, s, 0.5, true);    // B_theta points
  const double ez = gather<A>(p, sc, false, plane_rsrc<A>(Eout, p.plane, 0), shift);
  const double er = gather<A>(p, se, true, plane_rsrc<A>(Eout, p.plane, 1), shift);
  const double bt = 0.5 * (gather<A>(p, sb, true, plane_rsrc<A>(Ein, p.plane, 2), 0) +
                           gather<A>(p, sb, true, plane_rsrc<A>(Eout, p.plane, 2), shift));
  const double ir = r > 0.0 ? 1.0 / r : 0.0;
  const double cx = x * ir, cy = y * ir;
  const double Ex = er * cx, Ey = er * cy, Ez = ez;
  const double Bx = -bt * cy, By = bt * cx, Bz = 0.0;
  // half kick, rotation, half kick
  const double dt = p.dt;
  const double mx = px - 0.5 * dt * Ex, my = py - 0.5 * dt * Ey, mz = pz - 0.5 * dt * Ez;
  const double h2g = -0.5 * dt / sqrt(1.0 + (mx * mx + my * my + mz * mz));
  const double tx = h2g * Bx, ty = h2g * By, tz = h2g * Bz;
  const double ux = mx + (my * tz - mz * ty), uy = my + (mz * tx - mx * tz), uz = mz + (mx * ty - my * tx);
  const double t2 = 1.0 + (tx * tx + ty * ty + tz * tz);
  const double i2 = 2.0 / t2;
  const double sx = tx * i2, sy = ty * i2, sz = tz * i2;
  px = mx + (uy * sz - uz * sy) - 0.5 * dt * Ex;
  py = my + (uz * sx - ux * sz) - 0.5 * dt * Ey;
  pz = mz + (ux * sy - uy * sx) - 0.5 * dt * Ez;
}

// The bunch's coordinates: non-temporal (NT) accesses keep them out of the caches' way.
template <bool NT>
__device__ __forceinline__ double bunch_ld(const double* a) {
  if constexpr (NT) return __builtin_nontemporal_load(a);
  else return *a;
}
template <bool NT>
__device__ __forceinline__ void bunch_st(double v, double* a) {
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// Move to the next time level and deposit the midpoint current; PUSH: first the Boris push of the
// step that has just run (s, shift, Ein, Eout as for bunch_push_kernel), then the move in the frame
// s + shift of the next step.  NT: non-temporal loads and stores of the coordinates.
template <int ST, bool PUSH, bool NT>
__global__ __launch_bounds__(BT) void bunch_move_kernel(Physics p, long long s, int shift, const void* Einv,
                                                        const void* Eoutv, double* b, int n, long long cap,
                                                        void* jbv) {
  using A = typename Mode<ST, false>::A;
  const double ih = 1.0 / p.h;
  __shared__ A tile[2][TRW * TW];
  __shared__ int ext[BT / 64][4];   // per wavefront: lowest column, highest column, lowest row, highest row
  bool live[PPT];
  Stencil jz[PPT], jr[PPT];
  double vz[PPT], vr[PPT];
  int lcmin = INT32_MAX, lcmax = -1, lrmin = INT32_MAX, lrmax = -1;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    // the block's particles are one contiguous run of the z-ordered bunch; every lane loads its
    // particle (a clamped one past the end) before any test, so the loads issue together
    const long long q = ((long long)blockIdx.x * PPT + u) * BT + threadIdx.x;
    const long long qc = q < n ? q : (long long)n - 1;
    const double w = bunch_ld<NT>(b + 6 * cap + qc);
    const double x = bunch_ld<NT>(b + qc), y = bunch_ld<NT>(b + cap + qc), z = bunch_ld<NT>(b + 2 * cap + qc);
    double px = bunch_ld<NT>(b + 3 * cap + qc), py = bunch_ld<NT>(b + 4 * cap + qc), pz = bunch_ld<NT>(b + 5 * cap + qc);
    live[u] = false;
    jz[u] = Stencil{};
    jr[u] = Stencil{};
    vz[u] = 0.0;
    vr[u] = 0.0;
    if (q >= n || w == 0.0) continue;
    if (PUSH) {
      boris_push(p, s, shift, (const A*)Einv, (const A*)Eoutv, x, y, z, px, py, pz);
      bunch_st<NT>(px, b + 3 * cap + q);
      bunch_st<NT>(py, b + 4 * cap + q);
      bunch_st<NT>(pz, b + 5 * cap + q);
    }
    const long long sm = PUSH ? s + shift : s;   // frame of the move
    const double ig = 1.0 / sqrt(1.0 + (px * px + py * py + pz * pz));
    const double bx = px * ig, by = py * ig, bz = pz * ig;
    const double xn = x + p.dt * bx, yn = y + p.dt * by, zn = z + p.dt * bz;
    const double xm = 0.5 * (x + xn), ym = 0.5 * (y + yn), zm = 0.5 * (z + zn);
    const double rm = sqrt(xm * xm + ym * ym), rn = sqrt(xn * xn + yn * yn);
    jz[u] = stencil(ih, zm, rm, sm, 0.5, false);
    jr[u] = stencil(ih, zm, rm, sm, 0.0, true);
    const bool ok = inside(p, jz[u]) && inside(p, jr[u]) && inside(p, stencil(ih, zn, rn, sm, 0.5, false)) &&
                    inside(p, stencil(ih, zn, rn, sm, 0.0, true)) && inside(p, stencil(ih, zn, rn, sm, 0.5, true));
    if (!ok) {
      b[6 * cap + q] = 0.0;   // lost
      continue;
    }
    bunch_st<NT>(xn, b + q);
    bunch_st<NT>(yn, b + cap + q);
    bunch_st<NT>(zn, b + 2 * cap + q);
    vz[u] = w * bz;
    vr[u] = w * (rm > 0.0 ? (xm * bx + ym * by) / rm : 0.0);
    live[u] = true;
    // deposited columns and rows (E_z points: row -1 folds onto 0; E_r points: row -1 dropped)
    lcmin = min(lcmin, min(jz[u].i0, jr[u].i0));
    lcmax = max(lcmax, max(jz[u].i0, jr[u].i0) + 1);
    lrmin = min(lrmin, max(0, min(jz[u].j0, jr[u].j0)));
    lrmax = max(lrmax, max(jz[u].j0, jr[u].j0) + 1);
  }
  // the block's extent: wavefront reductions, then (several wavefronts) one slot per wavefront
  int c0 = wave_min(lcmin), c1 = wave_max(lcmax), r0 = wave_min(lrmin), r1 = wave_max(lrmax);
  if constexpr (BT > 64) {
    const int wv = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
      ext[wv][0] = c0;
      ext[wv][1] = c1;
      ext[wv][2] = r0;
      ext[wv][3] = r1;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BT / 64; ++k) {
      c0 = min(c0, ext[k][0]);
      c1 = max(c1, ext[k][1]);
      r0 = min(r0, ext[k][2]);
      r1 = max(r1, ext[k][3]);
    }
  }
  A* J = (A*)jbv;
  if (c1 < 0) return;                            // no live particle in the block (uniform)
  const int nc = c1 - c0 + 1, nrow = r1 - r0 + 1;
  if (nc > TW || nrow > TRW) {                   // too spread for the tile: straight to the grid
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      if (!live[u]) continue;
      deposit(p, jz[u], false, vz[u], J);
      deposit(p, jr[u], true, vr[u], J + p.plane);
    }
    return;
  }
  const int cells = nrow * nc;
  for (int t = threadIdx.x; t < cells; t += BT) {
    tile[0][t] = A(0);
    tile[1][t] = A(0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PPT; ++u) {   // every lane, live or not (wavefront-wide sums)
    deposit_tile(p, jz[u], false, vz[u], live[u], tile[0], c0, r0, nc);
    deposit_tile(p, jr[u], true, vr[u], live[u], tile[1], c0, r0, nc);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < cells; t += BT) {
    const int j = r0 + t / nc, c = c0 + t % nc;
    const long long o = (long long)j * p.pitch + c;
    const A a0 = tile[0][t], a1 = tile[1][t];
    if (a0 != A(0)) atomic_add(J + o, (double)a0);
    if (a1 != A(0)) atomic_add(J + p.plane + o, (double)a1);
  }
}

template <int ST>
__global__ __launch_bounds__(BT) void bunch_push_kernel(Physics p, long long s, int shift, const void* Einv,
                                                        const void* Eoutv, double* b, int n, long long cap) {
  using A = typename Mode<ST, false>::A;
  const int q = blockIdx.x * BT + threadIdx.x;
  if (q >= n) return;
  if (b[6 * cap + q] == 0.0) return;
  double px = b[3 * cap + q], py = b[4 * cap + q], pz = b[5 * cap + q];
  boris_push(p, s, shift, (const A*)Einv, (const A*)Eoutv, b[q], b[cap + q], b[2 * cap + q], px, py, pz);
  b[3 * cap + q] = px;
  b[4 * cap + q] = py;
  b[5 * cap + q] = pz;
}

__global__ __launch_bounds__(BT) void bunch_density_kernel(Physics p, long long s, double zoff, double t_ahead,
                                                           const double* b, int n, long long cap, double* dens) {
  const int q = blockIdx.x * BT + threadIdx.x;
  if (q >= n) return;
  const double px = b[3 * cap + q], py = b[4 * cap + q], pz = b[5 * cap + q];
  const double g = sqrt(1.0 + (px * px + py * py + pz * pz));
  const double x = b[q] + t_ahead * (px / g), y = b[cap + q] + t_ahead * (py / g);
  const double z = b[2 * cap + q] + t_ahead * (pz / g);
  const double r = sqrt(x * x + y * y);
  const double ih = 1.0 / p.h;
  const Stencil st = stencil(ih, z, r, s, zoff, false);
  if (!inside(p, st)) return;
  deposit(p, st, false, b[6 * cap + q], dens);
}

// Discrete Gauss law of the density (one thread per column): E_r at r = (j + 1) dr is
// -(dr / (j + 1)) sum_{j' <= j} (j' + 1/2) n(r_j').
template <int ST>
__global__ void bunch_gauss_kernel(Physics p, const double* dens, void* Ev, int comp) {
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nz) return;
  A* E = (A*)Ev + comp * p.plane;
  double cum = 0.0;
  for (int j = 0; j < p.nr; ++j) {
    const long long oo = (long long)j * p.pitch + i;
    cum += (j + 0.5) * dens[oo];
    const double v = -p.h * cum / (j + 1.0);
    stv(E + oo, v);
    set_field_lo<ST>(Ev, p.plane, oo, comp, v);
  }
}

// Re-sort of the bunch: a counting sort by cell.  The key of a particle at its position (t_{k-1},
// frame s) is its cell, column-major: the column of z in the window, then the row of r >> rshift,
// both clamped to the grid; lost particles (w = 0) take the last key.  A pass counts the particles
// per key (an atomic increment, whose return value is the particle's rank within its key), an
// exclusive scan turns the counts into offsets, and a scatter moves each particle to offset + rank.
// The order within a key is the order of the atomics: arbitrary, which only the order of the
// float additions of the deposit can tell.
constexpr int SCAN_T = 1024;            // threads of the scan kernels
constexpr int SCAN_ITEMS = 4;           // keys per thread
constexpr int SCAN_CHUNK = SCAN_T * SCAN_ITEMS;
constexpr long long MAX_KEYS = 1 << 22; // rows are coarsened (rshift) to stay within this many keys

__global__ __launch_bounds__(256) void sort_clear_kernel(uint32_t* counts, long long nkeys) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t < nkeys) counts[t] = 0u;
}

__global__ __launch_bounds__(256) void sort_count_kernel(Physics p, long long s, int rshift, const double* b, int n,
                                                         long long cap, uint32_t* counts, uint32_t* key,
                                                         uint32_t* rank) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const uint32_t nrk = (uint32_t)((p.nr - 1) >> rshift) + 1u;
  uint32_t k = (uint32_t)p.nz * nrk;
  if (b[6 * cap + q] != 0.0) {
    const double ih = 1.0 / p.h;
    const double x = b[q], y = b[cap + q];
    const double u = floor(b[2 * cap + q] * ih) - (double)s;
    const double v = floor(sqrt(x * x + y * y) * ih);
    const int i = (int)fmin(fmax(u, 0.0), (double)(p.nz - 1));
    const int j = (int)fmin(fmax(v, 0.0), (double)(p.nr - 1));
    k = (uint32_t)i * nrk + (uint32_t)(j >> rshift);
  }
  key[q] = k;
  rank[q] = atomicAdd(counts + k, 1u);
}

// Exclusive scan of v over the SCAN_T threads of the block; *total gets the block's sum.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d *= 2) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < SCAN_T / 64; ++w) {
    const uint32_t t = wsum[w];
    before += w < wv ? t : 0u;
    all += t;
  }
  __syncthreads();   // wsum is free again for the caller's next scan
  *total = all;
  return before + x - v;
}

// Sum of each chunk of SCAN_CHUNK counts into bsum[chunk].
__global__ __launch_bounds__(SCAN_T) void sort_chunk_sum_kernel(const uint32_t* counts, long long nkeys,
                                                                 uint32_t* bsum) {
  __shared__ uint32_t wsum[SCAN_T / 64];
  const long long base = (long long)blockIdx.x * SCAN_CHUNK + (long long)threadIdx.x * SCAN_ITEMS;
  uint32_t v = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) v += base + e < nkeys ? counts[base + e] : 0u;
  uint32_t total;
  (void)block_scan(v, wsum, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the chunk sums in place (one block, chunks of SCAN_T with a carry).
__global__ __launch_bounds__(SCAN_T) void sort_top_scan_kernel(uint32_t* bsum, int nchunks) {
  __shared__ uint32_t wsum[SCAN_T / 64];
  uint32_t carry = 0;
  for (int base = 0; base < nchunks; base += SCAN_T) {
    const int t = base + threadIdx.x;
    const uint32_t v = t < nchunks ? bsum[t] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan(v, wsum, &total);
    if (t < nchunks) bsum[t] = carry + ex;
    carry += total;
  }
}

// Counts to exclusive offsets in place: the chunk's offset plus the scan within the chunk.
__global__ __launch_bounds__(SCAN_T) void sort_offsets_kernel(uint32_t* counts, long long nkeys,
                                                               const uint32_t* bsum) {
  __shared__ uint32_t wsum[SCAN_T / 64];
  const long long base = (long long)blockIdx.x * SCAN_CHUNK + (long long)threadIdx.x * SCAN_ITEMS;
  uint32_t c[SCAN_ITEMS], v = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    c[e] = base + e < nkeys ? counts[base + e] : 0u;
    v += c[e];
  }
  uint32_t total;
  uint32_t off = bsum[blockIdx.x] + block_scan(v, wsum, &total);
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    if (base + e < nkeys) counts[base + e] = off;
    off += c[e];
  }
}

// out[:, offsets[key[q]] + rank[q]] = in[:, q] for the 7 components, and the same for pid.
__global__ __launch_bounds__(256) void sort_scatter_kernel(const double* in, const int32_t* pid_in,
                                                           const uint32_t* offsets, const uint32_t* key,
                                                           const uint32_t* rank, int n, long long cap, double* out,
                                                           int32_t* pid_out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const long long d = (long long)offsets[key[q]] + rank[q];
#pragma unroll
  for (int c = 0; c < 7; ++c) out[c * cap + d] = in[c * cap + q];
  pid_out[d] = pid_in[q];
}

}  // namespace

void bunch_sort_shape(const Physics& p, int* rshift, long long* nkeys) {
  int r = 0;
  while ((long long)p.nz * (((p.nr - 1) >> r) + 1) + 1 > MAX_KEYS && ((p.nr - 1) >> r) > 0) ++r;
  *rshift = r;
  *nkeys = (long long)p.nz * (((p.nr - 1) >> r) + 1) + 1;
}

size_t bunch_sort_bytes(const Physics& p) {
  int r;
  long long nkeys;
  bunch_sort_shape(p, &r, &nkeys);
  const long long nchunks = (nkeys + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up((size_t)nkeys * 4) + up((size_t)nchunks * 4) + 2 * up((size_t)p.cap * 4);
}

hipError_t launch_bunch_resort(const Physics& p, long long s, const double* in, const int32_t* pid_in, int n,
                               void* scratch, double* out, int32_t* pid_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int rshift;
  long long nkeys;
  bunch_sort_shape(p, &rshift, &nkeys);
  const long long nchunks = (nkeys + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  char* w = (char*)scratch;
  uint32_t* counts = (uint32_t*)w;
  uint32_t* bsum = (uint32_t*)(w + up((size_t)nkeys * 4));
  uint32_t* key = (uint32_t*)(w + up((size_t)nkeys * 4) + up((size_t)nchunks * 4));
  uint32_t* rank = (uint32_t*)((char*)key + up((size_t)p.cap * 4));
  const dim3 gp((n + 255) / 256);
  sort_clear_kernel<<<dim3((unsigned)((nkeys + 255) / 256)), 256, 0, st>>>(counts, nkeys);
  sort_count_kernel<<<gp, 256, 0, st>>>(p, s, rshift, in, n, p.cap, counts, key, rank);
  sort_chunk_sum_kernel<<<dim3((unsigned)nchunks), SCAN_T, 0, st>>>(counts, nkeys, bsum);
  sort_top_scan_kernel<<<1, SCAN_T, 0, st>>>(bsum, (int)nchunks);
  sort_offsets_kernel<<<dim3((unsigned)nchunks), SCAN_T, 0, st>>>(counts, nkeys, bsum);
  sort_scatter_kernel<<<gp, 256, 0, st>>>(in, pid_in, counts, key, rank, n, p.cap, out, pid_out);
  return hipGetLastError();
}

namespace {

// Extent of the live particles, per block of EXT_T threads striding over the bunch: lowest and
// highest column floor(z / dz) and highest row floor(r / dr), in the lab frame, into
// out[3 * blockIdx.x ..].
constexpr int EXT_T = 1024;
__global__ __launch_bounds__(EXT_T) void bunch_extent_kernel(Physics p, const double* b, int n, long long cap,
                                                             int* out) {
  __shared__ int part[EXT_T / 64][3];
  const double ih = 1.0 / p.h;
  int zlo = INT32_MAX, zhi = INT32_MIN, rhi = INT32_MIN;
  for (int q = blockIdx.x * EXT_T + threadIdx.x; q < n; q += gridDim.x * EXT_T) {
    if (b[6 * cap + q] == 0.0) continue;
    const double x = b[q], y = b[cap + q];
    const double u = fmin(fmax(floor(b[2 * cap + q] * ih), -1e9), 1e9);
    const double v = fmin(floor(sqrt(x * x + y * y) * ih), 1e9);
    zlo = min(zlo, (int)u);
    zhi = max(zhi, (int)u);
    rhi = max(rhi, (int)v);
  }
  zlo = wave_min(zlo);
  zhi = wave_max(zhi);
  rhi = wave_max(rhi);
  if (threadIdx.x % 64 == 0) {
    part[threadIdx.x / 64][0] = zlo;
    part[threadIdx.x / 64][1] = zhi;
    part[threadIdx.x / 64][2] = rhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < EXT_T / 64; ++w) {
      zlo = min(zlo, part[w][0]);
      zhi = max(zhi, part[w][1]);
      rhi = max(rhi, part[w][2]);
    }
    out[3 * blockIdx.x + 0] = zlo;
    out[3 * blockIdx.x + 1] = zhi;
    out[3 * blockIdx.x + 2] = rhi;
  }
}

}  // namespace

int bunch_extent_blocks(int n) { return n <= 0 ? 1 : (n + EXT_T - 1) / EXT_T < EXTENT_BLOCKS ? (n + EXT_T - 1) / EXT_T : EXTENT_BLOCKS; }

hipError_t launch_bunch_extent(const Physics& p, const double* bunch, int n, long long cap, int* out,
                               hipStream_t st) {
  bunch_extent_kernel<<<bunch_extent_blocks(n), EXT_T, 0, st>>>(p, bunch, n, cap, out);
  return hipGetLastError();
}

#define BUNCH_DISPATCH(storage, KERNEL, GRID, STREAM, ...)                         \
  do {                                                                             \
    if ((storage) == 0) KERNEL<0><<<(GRID), BT, 0, (STREAM)>>>(__VA_ARGS__);       \
    else if ((storage) == 1) KERNEL<1><<<(GRID), BT, 0, (STREAM)>>>(__VA_ARGS__);  \
    else KERNEL<2><<<(GRID), BT, 0, (STREAM)>>>(__VA_ARGS__);                      \
  } while (0)

template <bool PUSH>
hipError_t move_dispatch(int storage, const Physics& p, long long s, int shift, const void* Ein, const void* Eout,
                         double* bunch, int n, long long cap, void* jb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + PPT * BT - 1) / (PPT * BT));
  if (p.bunch_nt) {
    if (storage == 0) bunch_move_kernel<0, PUSH, true><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
    else if (storage == 1) bunch_move_kernel<1, PUSH, true><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
    else bunch_move_kernel<2, PUSH, true><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
  } else {
    if (storage == 0) bunch_move_kernel<0, PUSH, false><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
    else if (storage == 1) bunch_move_kernel<1, PUSH, false><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
    else bunch_move_kernel<2, PUSH, false><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
  }
  return hipGetLastError();
}

hipError_t launch_bunch_move(int storage, const Physics& p, long long s, double* bunch, int n, long long cap,
                             void* jb, hipStream_t st) {
  return move_dispatch<false>(storage, p, s, 0, nullptr, nullptr, bunch, n, cap, jb, st);
}

hipError_t launch_bunch_push_move(int storage, const Physics& p, long long s, int shift, const void* Ein,
                                  const void* Eout, double* bunch, int n, long long cap, void* jb, hipStream_t st) {
  return move_dispatch<true>(storage, p, s, shift, Ein, Eout, bunch, n, cap, jb, st);
}

hipError_t launch_bunch_push(int storage, const Physics& p, long long s, int shift, const void* Ein,
                             const void* Eout, double* bunch, int n, long long cap, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  BUNCH_DISPATCH(storage, bunch_push_kernel, dim3((n + BT - 1) / BT), st, p, s, shift, Ein, Eout, bunch, n, cap);
  return hipGetLastError();
}

hipError_t launch_bunch_density(const Physics& p, long long s, double zoff, double t_ahead, const double* bunch,
                                int n, long long cap, double* dens, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  bunch_density_kernel<<<dim3((n + BT - 1) / BT), BT, 0, st>>>(p, s, zoff, t_ahead, bunch, n, cap, dens);
  return hipGetLastError();
}

hipError_t launch_bunch_gauss(int storage, const Physics& p, const double* dens, void* E, int comp, hipStream_t st) {
  const dim3 grid((p.nz + 63) / 64);
  if (storage == 0) bunch_gauss_kernel<0><<<grid, 64, 0, st>>>(p, dens, E, comp);
  else if (storage == 1) bunch_gauss_kernel<1><<<grid, 64, 0, st>>>(p, dens, E, comp);
  else bunch_gauss_kernel<2><<<grid, 64, 0, st>>>(p, dens, E, comp);
  return hipGetLastError();
}

}  // namespace lbm
