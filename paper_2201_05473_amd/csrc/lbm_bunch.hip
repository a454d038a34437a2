// Particle driver (gfx950): the electron bunch as macroparticles of Sec. II, Eq. (1), coupled to
// the grid through its projected current.
//
// The bunch is stored as SoA doubles [7][cap]: x, y, z (lab frame), p_x, p_y, p_z (m_e c units),
// w (electrons, n_0 / k_p^3).  After k steps the positions are at t_{k-1} and the momenta at
// t_{k-1/2}.  Step k runs:
//   bunch_move_kernel  positions to t_k, current w beta at the midpoints -> J_b(t_{k-1/2}) (z at the
//                      E_z points, r at the E_r points): summed per block in LDS when the block's
//                      particles span few columns (the bunch is stored by column of z, then by
//                      radius), then added to the grid with hardware float atomics;
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

constexpr int BT = 256;   // threads per block of the particle kernels
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
// (1 for an array written after a window shift).
template <typename A>
__device__ __forceinline__ double gather(const Physics& p, const Stencil& st, bool edge, const A* F, int col_shift) {
  double out = 0.0;
#pragma unroll
  for (int di = 0; di < 2; ++di) {
    const double wz = di ? st.fz : 1.0 - st.fz;
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      const double wr = dj ? st.fr : 1.0 - st.fr;
      const int j = st.j0 + dj;
      double val;
      if (j < 0) val = edge ? 0.0 : (double)F[st.i0 + di - col_shift];
      else val = (double)F[(long long)j * p.pitch + st.i0 + di - col_shift];
      out = out + wz * wr * val;
    }
  }
  return out;
}

// LDS tile of the deposit privatisation: the J_z and J_r shares of a block's particles are summed
// here first when they fall in TW consecutive columns and the first TRW rows (the bunch is kept
// ordered by column, so a block's particles share a few columns), then added to the grid once per
// cell.
constexpr int TW = 8, TRW = 192;
// Particles per thread of the move kernel (a block moves PPT * BT consecutive particles).  Measured
// on C2 with 200,000 particles: 1 is best (2: +1.5 %, 4: +12 %); with 10^6 particles 2 gains 2 %.
constexpr int PPT = 1;

template <typename T>
__device__ __forceinline__ void lds_add(T* a, double v) { atomicAdd(a, (T)v); }

// Adds the shares of val over the stencil's nodes to the tile (columns from c0).
template <typename T>
__device__ __forceinline__ void deposit_tile(const Physics& p, const Stencil& st, bool edge, double val, T* tile,
                                             int c0) {
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    int j = st.j0 + dj;
    if (j < 0) {
      if (edge) continue;
      j = 0;
    }
    const double rn = ((double)j + (edge ? 1.0 : 0.5)) * p.h;
    const double vr = val * (dj ? st.fr : 1.0 - st.fr) / (TWO_PI * rn * p.h * p.h);
#pragma unroll
    for (int di = 0; di < 2; ++di) lds_add(tile + j * TW + (st.i0 + di - c0), vr * (di ? st.fz : 1.0 - st.fz));
  }
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
  const double ez = gather(p, sc, false, Eout, shift);
  const double er = gather(p, se, true, Eout + p.plane, shift);
  const double bt = 0.5 * (gather(p, sb, true, Ein + 2 * p.plane, 0) + gather(p, sb, true, Eout + 2 * p.plane, shift));
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

// Move to the next time level and deposit the midpoint current; PUSH: first the Boris push of the
// step that has just run (s, shift, Ein, Eout as for bunch_push_kernel), then the move in the frame
// s + shift of the next step.
template <int ST, bool PUSH>
__global__ __launch_bounds__(BT) void bunch_move_kernel(Physics p, long long s, int shift, const void* Einv,
                                                        const void* Eoutv, double* b, int n, long long cap,
                                                        void* jbv) {
  using A = typename Mode<ST, false>::A;
  const double ih = 1.0 / p.h;
  __shared__ A tile[2][TRW * TW];
  __shared__ int cmin, cmax, rmax;
  if (threadIdx.x == 0) {
    cmin = INT32_MAX;
    cmax = -1;
    rmax = -1;
  }
  __syncthreads();
  bool live[PPT];
  Stencil jz[PPT], jr[PPT];
  double vz[PPT], vr[PPT];
  int lcmin = INT32_MAX, lcmax = -1, lrmax = -1;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    // the block's particles are one contiguous run of the z-ordered bunch
    const long long q = ((long long)blockIdx.x * PPT + u) * BT + threadIdx.x;
    live[u] = false;
    jz[u] = Stencil{};
    jr[u] = Stencil{};
    vz[u] = 0.0;
    vr[u] = 0.0;
    if (q >= n || b[6 * cap + q] == 0.0) continue;
    const double w = b[6 * cap + q];
    const double x = b[q], y = b[cap + q], z = b[2 * cap + q];
    double px = b[3 * cap + q], py = b[4 * cap + q], pz = b[5 * cap + q];
    if (PUSH) {
      boris_push(p, s, shift, (const A*)Einv, (const A*)Eoutv, x, y, z, px, py, pz);
      b[3 * cap + q] = px;
      b[4 * cap + q] = py;
      b[5 * cap + q] = pz;
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
    b[q] = xn;
    b[cap + q] = yn;
    b[2 * cap + q] = zn;
    vz[u] = w * bz;
    vr[u] = w * (rm > 0.0 ? (xm * bx + ym * by) / rm : 0.0);
    live[u] = true;
    lcmin = min(lcmin, min(jz[u].i0, jr[u].i0));
    lcmax = max(lcmax, max(jz[u].i0, jr[u].i0) + 1);
    lrmax = max(lrmax, max(jz[u].j0, jr[u].j0) + 1);
  }
  if (lcmax >= 0) {
    atomicMin(&cmin, lcmin);
    atomicMax(&cmax, lcmax);
    atomicMax(&rmax, lrmax);
  }
  __syncthreads();
  A* J = (A*)jbv;
  const int c0 = cmin, nc = cmax - cmin + 1, nrow = rmax + 1;
  if (cmax < 0) return;                          // no live particle in the block (uniform)
  if (nc > TW || nrow > TRW) {                   // too spread for the tile: straight to the grid
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      if (!live[u]) continue;
      deposit(p, jz[u], false, vz[u], J);
      deposit(p, jr[u], true, vr[u], J + p.plane);
    }
    return;
  }
  for (int t = threadIdx.x; t < nrow * TW; t += BT) {
    tile[0][t] = A(0);
    tile[1][t] = A(0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    if (!live[u]) continue;
    deposit_tile(p, jz[u], false, vz[u], tile[0], c0);
    deposit_tile(p, jr[u], true, vr[u], tile[1], c0);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nrow * TW; t += BT) {
    const int j = t / TW, c = t % TW;
    if (c >= nc) continue;
    const long long o = (long long)j * p.pitch + c0 + c;
    if (tile[0][t] != A(0)) atomic_add(J + o, (double)tile[0][t]);
    if (tile[1][t] != A(0)) atomic_add(J + p.plane + o, (double)tile[1][t]);
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

}  // namespace

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
  if (storage == 0) bunch_move_kernel<0, PUSH><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
  else if (storage == 1) bunch_move_kernel<1, PUSH><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
  else bunch_move_kernel<2, PUSH><<<grid, BT, 0, st>>>(p, s, shift, Ein, Eout, bunch, n, cap, jb);
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
