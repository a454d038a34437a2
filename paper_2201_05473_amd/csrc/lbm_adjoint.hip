// Hand-written discrete adjoint of the lattice-Boltzmann plasma-wakefield step (gfx950).
//
// For the state x^k = (g^{k-1}, A*^{k-1}, E^{k-1}, B^{k-1/2}) and the step x^{k+1} = Phi(x^k; theta)
// of the forward kernel, these kernels compute lambda^k = (dPhi/dx^k)^T lambda^{k+1} and the
// parameter partials (dPhi/dtheta)^T lambda^{k+1}, theta = (ramp length, n0, sigma_r, n_b).
// The adjoint variables are stored in the precision of the auxiliary planes (FP64 for FP64
// storage, FP32 otherwise).  Arithmetic: the site part (the collision's VJP) computes in the
// forward step's precision (FP64 for FP64 storage, FP32 otherwise); the cell part (transposes of
// the Yee curls and site averages, which difference neighbouring adjoints) and every theta
// partial stay in FP64, where FP32 would lose the cancelling digits.  All variables are the raw
// populations, moments and fields (the deviation encoding of the stored density lattice is an
// identity map for the adjoint).
//
// Population adjoints are carried in "pulled" form: f_bar^k(y, q) is the adjoint of the population
// that site y pulls in step k (the collision input).  Every collision operator is linear in the
// pulled populations apart from the equilibrium, g' = P f + (I - P) f_eq + w dt F, so its VJP is
// f_bar^k(y, .) = P^T g_bar^{k+1}(y, .) + A_bar_kk(y) (kk = lattice of q; BGK: P = (1 - 1/tau) I,
// which gives rank-3 structure), and the adjoint of the stored population is its transposed
// pull, g_bar^k(x, q) = f_bar^k(x + xi_q, q).  So each
// reverse step reads and writes the 27 population planes once, exactly like the forward step.
// Gather form throughout: every output has a single writer, no atomics, fixed summation order.
//
//   adj_site_kernel   per fluid site: gather g_bar^{k+1} (pull of f_bar^{k+1}); the site fields and
//                     the moments A of the pulled populations come from the site record that the
//                     forward step wrote (the populations of x^k are not read); then the VJP of the
//                     collision: f_bar^k (27), and the site adjoints F_bar (3, source terms),
//                     E_bar_z, E_bar_r, B_bar; theta partials of the window-front ghost and of
//                     the new front column.
//   adj_cell_kernel   per cell: transposes of the site averages, Faraday and Ampere (every ghost
//                     rule), staged through LDS: lambda_E, lambda_B; lambda of the moments (face
//                     currents, the lagged radial gradient of the axisymmetric source, equilibrium
//                     ghosts); theta partials of the driver current.
//   adj_state_kernel  lambda^k in the stored-state layout (FP64): the transposed pull of f_bar^k.
//   adj_cast_kernel   an FP64 stored-state lambda into the adjoint precision (population planes as
//                     g_bar, read directly by the site kernel in its "state" input mode).
//   adj_init_*        theta partials of the initial state.
#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

// work planes written by adj_site_kernel, read by adj_cell_kernel
constexpr int W_F = 0, W_EZ = 3, W_ER = 4, W_B = 5;

// periodic wrap of an index at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// d n_bg / d(ramp_len), d n_bg / d(n0) at z (clamp derivative taken inclusive at the kinks)
__device__ __forceinline__ void dnbg(const Physics& p, double z, double& dlen, double& dn0) {
  if (p.ramp_kind == 0) { dlen = 0.0; dn0 = 1.0; return; }
  const double x = (z - p.ramp_start) / p.ramp_len;
  if (p.ramp_kind == 1) {
    dn0 = fmin(fmax(x, 0.0), 1.0);
    dlen = (x >= 0.0 && x <= 1.0) ? p.n0 * (-x / p.ramp_len) : 0.0;
    return;
  }
  const double t = tanh(2.0 * x - 1.0);
  dn0 = 0.5 * (1.0 + t);
  dlen = p.n0 * (1.0 - t * t) * (-x / p.ramp_len);
}

// driver density and its partials d/d(sigma_r), d/d(n_b)
__device__ __forceinline__ void ddriver(const Physics& p, double z, double r, double t, double& dsr,
                                        double& dnb) {
  const double dz = z - (p.zd0 + t);
  const double zr = exp(-(dz * dz) / (2.0 * p.sigma_z * p.sigma_z) - (r * r) / (2.0 * p.sigma_r * p.sigma_r));
  dnb = zr;
  dsr = p.nb * zr * r * r / (p.sigma_r * p.sigma_r * p.sigma_r);
}

// Block sum of 4 values; thread 0 adds it to acc[0..3] (each block owns its accumulator, and
// launches on one stream are ordered, so the running sums are deterministic).
__device__ __forceinline__ void block_sum4(double v[4], double* acc) {
  __shared__ double red[NTHREADS / 64][4];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] += __shfl_down(v[c], off, 64);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wid][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < NTHREADS / 64; ++w)
#pragma unroll
      for (int c = 0; c < 4; ++c) r[c] += red[w][c];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += r[c];
  }
}

// VJP of J = n beta(M) (the face current of Ampere's law) with respect to M.
template <typename T>
__device__ __forceinline__ void current_vjp(const Physics& p, const T M[3], T jzb, T jrb, T Mbar[3]) {
  T bz, br;
  if (!velocity<T>(M[0], M[1], M[2], (T)p.n_floor, bz, br)) return;
  const T n = M[0], in = T(1) / n, pz = M[1] * in, pr = M[2] * in;
  const T g2 = T(1) + pz * pz + pr * pr, ig = T(1) / sqrt(g2), ig3 = ig * ig * ig;
  // J_a = n p_a / gamma: dJ_a/dp_b = n (delta_ab / gamma - p_a p_b / gamma^3), dJ_a/dn|_p = beta_a
  const T jdot = jzb * pz + jrb * pr;
  const T pbz = n * (jzb * ig - pz * jdot * ig3), pbr = n * (jrb * ig - pr * jdot * ig3);
  const T nbar = jzb * bz + jrb * br;
  Mbar[1] += pbz * in;
  Mbar[2] += pbr * in;
  Mbar[0] += nbar - (pbz * pz + pbr * pr) * in;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// adj_site_kernel: one thread per logical fluid site (i, j) of x^k.  The site record of step k
// (E_z, E_r, B_theta averaged to the site as the fluid used them, and the moments of the pulled
// populations) comes from a.site, written by the forward step's recompute at the output index.
// ------------------------------------------------------------------------------------------
// The site part's loads (see site_body), issued by the caller ahead of other work.
template <int ST> struct SiteIn {
  typename Mode<ST, false>::A gbar[27], mbar[3], sfield[3], amom[3];
  bool gok[9];
};

// Loads of the site part for the tile whose first site is (i0, j0): g_bar^{k+1} at the site's
// output position (the transposed pull of f_bar^{k+1}, or read directly), M_bar^{k+1} unless the
// caller has it in registers (with_mbar false), and the site record the forward step wrote at the
// output index: the site fields and the moments A of the pulled populations (ghosts included).
// The collision's Jacobian depends on the pulled populations only through A, so the populations
// of x^k are not read.  Every read is of data written before the launch.
template <int ST>
__device__ __forceinline__ void site_load(const AdjArgs& a, int i0, int j0, bool with_mbar, SiteIn<ST>& in) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int tid = threadIdx.x, tx = tid % TZ, ty = tid / TZ;
  const A* __restrict__ L = (const A*)a.lam_next;
  const A* __restrict__ Sf = (const A*)a.site;
  const int i = i0 + tx, j = j0 + ty;
  const int ic = i < nz ? i : nz - 1, jc = j < nr ? j : nr - 1;
  const int ib = (ic - a.shift) < 0 ? 0 : ic - a.shift;   // output index in x^{k+1}
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int yi = ib, yj = jc;
    bool ok = true;
    if (a.pull_in) {
      yi += XZ(q);
      yj += XR(q);
      if (p.per_z) yi = wrap1(yi, nz);
      else if (yi < 0 || yi >= nz) { ok = false; yi = yi < 0 ? 0 : nz - 1; }
      if (p.per_r) yj = wrap1(yj, nr);
      else if (yj < 0 || yj >= nr) { ok = false; yj = yj < 0 ? 0 : nr - 1; }
    }
    in.gok[q] = ok;
    const int yo = yj * pitch + yi;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) in.gbar[9 * kk + q] = (L + (9 * kk + q) * plane)[yo];
  }
  const int so = jc * pitch + ib;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) in.mbar[kk] = with_mbar ? (L + (27 + kk) * plane)[so] : A(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) in.sfield[c] = p.fields_on ? (Sf + c * plane)[so] : A(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) in.amom[c] = (Sf + (3 + c) * plane)[so];
}

// Site part of a reverse step for the tile whose first site is (i0, j0) (logical columns of x^k),
// from its loads (site_load).  mreg: M_bar^{k+1} of the thread's site output, when the caller has
// it in registers (else in.mbar).  theta partials are added to part.
template <int ST, int COLL>
__device__ __forceinline__ void site_body(const AdjArgs& a, int i0, int j0, const typename Mode<ST, false>::C* mreg,
                                          double part[4], const SiteIn<ST>& in) {
  using A = typename Mode<ST, false>::A;   // auxiliary planes and adjoint variables
  using T = typename Mode<ST, false>::C;   // arithmetic (FP64 for FP64 storage, else FP32)
  const Physics& p = a.p;

  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int tid = threadIdx.x, tx = tid % TZ, ty = tid / TZ;
  const double h = p.h;
  const T dt = (T)p.dt, lam = (T)p.lam, floor_ = (T)p.n_floor;
  const A* __restrict__ L = (const A*)a.lam_next;

  const int i = i0 + tx, j = j0 + ty;
  const bool mine = i < nz && j < nr;
  const bool dropped = a.shift && i == 0;   // this column leaves the window in step k
  const A (&gbar)[27] = in.gbar;
  const A (&mbar)[3] = in.mbar;
  const A (&sfield)[3] = in.sfield;
  const A (&amom)[3] = in.amom;
  const bool (&gok)[9] = in.gok;

  if (a.shift && i == nz && j < nr) {
    // the column dropped in this step (column 0) has no site: zero adjoint sources.  Written
    // here too because a caller may start its tile at column 1 (tiles of the output frame)
    A* __restrict__ Lo = (A*)a.lam;
    A* __restrict__ W = (A*)a.work;
#pragma unroll
    for (int c = 0; c < 27; ++c) (Lo + c * plane)[j * pitch] = A(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) (W + c * plane)[j * pitch] = A(0);
  }
  if (mine) {
    const int cell = j * pitch + i;
    A* __restrict__ Lo = (A*)a.lam;
    A* __restrict__ W = (A*)a.work;
    if (dropped) {
      // the first column leaves the window in this step: no site, no adjoint source
#pragma unroll
      for (int c = 0; c < 27; ++c) (Lo + c * plane)[cell] = A(0);
#pragma unroll
      for (int c = 0; c < 6; ++c) (W + c * plane)[cell] = A(0);
    } else {
      const T Am[3] = {(T)amom[0], (T)amom[1], (T)amom[2]};
      const T n = Am[0];
      T bz, br;
      const bool live = velocity<T>(Am[0], Am[1], Am[2], floor_, bz, br);
      const T uz = lam * bz, ur = lam * br;
      T pz = T(0.0), pr = T(0.0), ig = T(1.0), in = T(0.0);
      if (live) {
        in = T(1.0) / n;
        pz = Am[1] * in;
        pr = Am[2] * in;
        ig = T(1.0) / sqrt(T(1.0) + pz * pz + pr * pr);
      }
      const T Ebz = (T)sfield[0], Ebr = (T)sfield[1], Bb = (T)sfield[2];
      const T ir = (T)(1.0 / ((j + 0.5) * h));

      // g' = P f + (I - P) e + w dt F,  M' = A + dt F,  e = w A (1 + Q(u)), with P the collision's
      // action on the pulled populations (BGK: P = (1 - 1/tau) I).  So the pulled populations get
      // P^T g_bar, and the equilibrium gets e_bar = g_bar - P^T g_bar (BGK: g_bar / tau).
      T Fb[3], Ab[3];
      T ubz = T(0.0), ubr = T(0.0);
      T sw[3] = {T(0.0), T(0.0), T(0.0)}, s0[3] = {T(0.0), T(0.0), T(0.0)};
      const T itau = T(1.0) / (T)p.tau, usq = uz * uz + ur * ur;
      // P^T g_bar for lattice kk (operators other than BGK)
      auto ptrans = [&](int kk, T (&pt)[9]) {
        T g[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = gok[q] ? (T)gbar[9 * kk + q] : T(0.0);
        if (COLL == 1) {
          // two relaxation times: P = I - (even part / tau_plus + odd part / tau), symmetric
          const T itp = T(1.0) / (T)p.tau_plus;
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            const T gq = g[q], gb = g[OPPQ(q)];
            pt[q] = gq - T(0.5) * (gq + gb) * itp - T(0.5) * (gq - gb) * itau;
          }
        } else if (COLL == 3) {
          // multiple relaxation times: P = I - sum_m s_m b_m b_m^T / |b_m|^2, symmetric
          const T rate[9] = {T(0.0), (T)p.mrt_se, (T)p.mrt_seps, itau, (T)p.mrt_sq, itau, (T)p.mrt_sq,
                             (T)p.mrt_spi, (T)p.mrt_spi};
          T c[9];
#pragma unroll
          for (int m = 1; m < 9; ++m) {
            T nm = T(0.0);
#pragma unroll
            for (int q = 0; q < 9; ++q)
              if (MB(m, q) != 0) nm += (T)MB(m, q) * g[q];
            c[m] = rate[m] * nm / (T)MB_NORM2(m);
          }
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            T v = g[q];
#pragma unroll
            for (int m = 1; m < 9; ++m)
              if (MB(m, q) != 0) v -= (T)MB(m, q) * c[m];
            pt[q] = v;
          }
        } else {
          // regularised: P = (1 - 1/tau) H with H_qp = 3 w_q xi_q . xi_p
          T jz = T(0.0), jr = T(0.0);
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            jz += WQ<T>(q) * XZ(q) * g[q];
            jr += WQ<T>(q) * XR(q) * g[q];
          }
          const T k3 = T(3.0) * (T(1.0) - itau);
#pragma unroll
          for (int q = 0; q < 9; ++q) pt[q] = k3 * (XZ(q) * jz + XR(q) * jr);
        }
      };
      if (COLL == 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const T w = WQ<T>(q);
          const T cu = XZ(q) * uz + XR(q) * ur;
          const T e1 = w * (T(1.0) + T(3.0) * cu + T(4.5) * cu * cu - T(1.5) * usq);   // e_q / A
          const T fz = w * (T(3.0) * XZ(q) + T(9.0) * cu * XZ(q) - T(3.0) * uz);    // w dQ/du_z
          const T fr = w * (T(3.0) * XR(q) + T(9.0) * cu * XR(q) - T(3.0) * ur);
          T az = T(0.0);
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            const T gbq = gok[q] ? (T)gbar[9 * kk + q] : T(0.0);
            sw[kk] += w * gbq;
            s0[kk] += gbq * e1;
            az += gbq * Am[kk];
          }
          ubz += az * fz;
          ubr += az * fr;
        }
        ubz *= itau;
        ubr *= itau;
      } else {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          T pt[9];
          ptrans(kk, pt);
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            const T w = WQ<T>(q);
            const T cu = XZ(q) * uz + XR(q) * ur;
            const T e1 = w * (T(1.0) + T(3.0) * cu + T(4.5) * cu * cu - T(1.5) * usq);
            const T fz = w * (T(3.0) * XZ(q) + T(9.0) * cu * XZ(q) - T(3.0) * uz);
            const T fr = w * (T(3.0) * XR(q) + T(9.0) * cu * XR(q) - T(3.0) * ur);
            const T gbq = gok[q] ? (T)gbar[9 * kk + q] : T(0.0);
            const T eb = gbq - pt[q];
            sw[kk] += w * gbq;
            s0[kk] += eb * e1;
            ubz += eb * Am[kk] * fz;
            ubr += eb * Am[kk] * fr;
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const T Mb = mreg ? mreg[kk] : (T)mbar[kk];
        Fb[kk] = dt * (sw[kk] + Mb);
        Ab[kk] = COLL == 0 ? Mb + s0[kk] * itau : Mb + s0[kk];
      }
      T bbz = lam * ubz, bbr = lam * ubr;
      T Ebz_b = T(0.0), Ebr_b = T(0.0), Bb_b = T(0.0);
      if (live) {
        // F1 = -n (E_z + beta_r B), F2 = -n (E_r - beta_z B)
        bbr += Fb[1] * (-n * Bb);
        bbz += Fb[2] * (n * Bb);
        Ebz_b = -n * Fb[1];
        Ebr_b = -n * Fb[2];
        Bb_b = (-n * br) * Fb[1] + (n * bz) * Fb[2];
        Ab[0] += Fb[1] * (-(Ebz + br * Bb)) + Fb[2] * (-(Ebr - bz * Bb));
      }
      if (p.cyl_on) {
        // F_k += (-A_k beta_r + D dA_k/dr) / r
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          bbr += Fb[kk] * (-Am[kk] * ir);
          Ab[kk] += Fb[kk] * (-br * ir);
        }
      }
      if (live) {
        const T ig3 = ig * ig * ig;
        const T pdot = pz * bbz + pr * bbr;
        const T pbz = bbz * ig - pz * pdot * ig3, pbr = bbr * ig - pr * pdot * ig3;
        Ab[1] += pbz * in;
        Ab[2] += pbr * in;
        Ab[0] -= (pbz * pz + pbr * pr) * in;
      }
      // adjoint of the pulled populations: P^T g_bar' + A_bar (BGK: (1 - 1/tau) g_bar' + A_bar)
      const T c1 = T(1.0) - itau;
      T fb0[9];   // the adjoint of lattice 0's pulled populations, kept for the window-front term
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        T pt[9];
        if (COLL != 0) ptrans(kk, pt);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const T v = COLL == 0 ? c1 * (gok[q] ? (T)gbar[9 * kk + q] : T(0.0)) + Ab[kk] : pt[q] + Ab[kk];
          stv(&(Lo + (9 * kk + q) * plane)[cell], v);
          if (kk == 0) fb0[q] = v;
        }
      }
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) stv(&(W + (W_F + kk) * plane)[cell], Fb[kk]);
      stv(&(W + W_EZ * plane)[cell], Ebz_b);
      stv(&(W + W_ER * plane)[cell], Ebr_b);
      stv(&(W + W_B * plane)[cell], Bb_b);

      if (p.window && i == nz - 1) {
        // window front ghost: the populations pulled from column nz (xi_z = -1) are w_q n_bg(z_nz)
        double dl, dn;
        dnbg(p, (double)(a.s + nz) * h, dl, dn);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q)
          if (XZ(q) == -1) sum += WQ<double>(q) * (double)fb0[q];
        part[0] += sum * dl;
        part[1] += sum * dn;
        if (a.shift) {
          // the new front column of x^{k+1} (output index nz - 1): w_q n_bg and n_bg.  Its moment
          // adjoint M_bar^{k+1} is read here only in the split form; in the fused form it is made
          // in the same launch, possibly by another block, so the thread that makes it adds its
          // term (adj_fused_kernel)
          double s2 = mreg ? 0.0 : (double)(L + 27 * plane)[j * pitch + (nz - 1)];
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            int yi = nz - 1, yj = j;
            if (a.pull_in) {
              yi += XZ(q);
              yj += XR(q);
              if (yi >= nz || ((yj < 0 || yj >= nr) && !p.per_r)) continue;
              if (p.per_r) yj = wrap1(yj, nr);
            }
            s2 += WQ<double>(q) * (double)(L + q * plane)[yj * pitch + yi];
          }
          part[0] += s2 * dl;
          part[1] += s2 * dn;
        }
      }
    }
  }
}

template <int ST, int COLL>
__global__ __launch_bounds__(NTHREADS) void adj_site_kernel(AdjArgs a) {
  const int gx = (a.p.nz + TZ - 1) / TZ, gy = (a.p.nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  double part[4] = {0.0, 0.0, 0.0, 0.0};   // d/d(ramp_len, n0, sigma_r, n_b)
  const int i0 = (tile % gx) * TZ, j0 = (tile / gx) * TR;
  SiteIn<ST> in;
  site_load<ST>(a, i0, j0, true, in);
  site_body<ST, COLL>(a, i0, j0, nullptr, part, in);
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// ------------------------------------------------------------------------------------------
// adj_cell_kernel: one thread per cell (i, j) of x^k.  Field part staged through LDS:
// L_B' = adjoint of B^{k+1/2}, L_Ez', L_Er' = adjoints of E^k (as used by step k).
// ------------------------------------------------------------------------------------------
// Cell part of a reverse step for the tile whose first cell is (i0, j0) of x^k.  The moment
// adjoint of the thread's cell (zero for a thread outside the grid) is returned in mb_out as well
// as stored.  theta partials are added to part.  Every thread of the block must call it.  pre()
// runs once the cell part's own loads are issued: a fused caller issues the site part's loads
// there, so that they are in flight during the cell part (the compiler's waits count them out).
template <int ST, typename Pre>
__device__ __forceinline__ void cell_body(const AdjArgs& a, int i0, int j0, double part[4],
                                          typename Mode<ST, false>::C mb_out[3], Pre&& pre) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int tid = threadIdx.x, tx = tid % TZ, ty = tid / TZ;
  const double h = p.h, dt = p.dt, dth = dt / h;
  const A* __restrict__ W = (const A*)a.work;
  const A* __restrict__ L = (const A*)a.lam_next;
  A* Lo = (A*)a.lam;   // planes 0..26 (f_bar^k) read, planes 27..32 written

  // LDS regions (origin = lowest logical column / row)
  constexpr int BBZ = TZ + 3, BBR = TR + 3;   // site B_bar:  cols i0-1..i0+TZ+1, rows j0-1..j0+TR+1
  constexpr int EBZ = TZ + 2, EBR = TR + 1;   // site Ez_bar: cols i0-1..i0+TZ,   rows j0..j0+TR
  constexpr int RBZ = TZ + 1, RBR = TR + 2;   // site Er_bar: cols i0..i0+TZ,     rows j0-1..j0+TR
  constexpr int LBZ = TZ + 2, LBR = TR + 2;   // L_B':        cols i0-1..i0+TZ,   rows j0-1..j0+TR
  constexpr int LZZ = TZ + 1, LZR = TR + 1;   // L_Ez':       cols i0-1..i0+TZ-1, rows j0..j0+TR
  constexpr int LRZ = TZ + 1, LRR = TR + 1;   // L_Er':       cols i0..i0+TZ,     rows j0-1..j0+TR-1
  __shared__ double sBb[BBR][BBZ];
  __shared__ double sEb[EBR][EBZ];
  __shared__ double sRb[RBR][RBZ];
  __shared__ double sLB[LBR][LBZ];
  __shared__ double sLZ[LZR][LZZ];
  __shared__ double sLR[LRR][LRZ];

  // cell (ci, cj) in the domain after the periodic wrap of z (r is never periodic with fields
  // on); ci becomes the wrapped column
  auto cellz = [&](int& ci, int cj) -> bool {
    if (cj < 0 || cj >= nr) return false;
    if (p.per_z) { ci = wrapi(ci, nz); return true; }
    return ci >= 0 && ci < nz;
  };
  // clamped in-plane offset of a site value (ok: in the domain)
  auto woff = [&](int ci, int cj, bool& ok) -> int {
    ok = cellz(ci, cj);
    ci = ci < 0 ? 0 : (ci >= nz ? nz - 1 : ci);
    cj = cj < 0 ? 0 : (cj >= nr ? nr - 1 : cj);
    return cj * pitch + ci;
  };
  // clamped offset in x^{k+1} of the state value at logical cell (ci, cj) of x^k (ok: it exists,
  // i.e. in the domain and not the column dropped by the shift)
  auto noff = [&](int ci, int cj, bool& ok) -> int {
    ok = cellz(ci, cj);
    int o = ci - a.shift;
    ok = ok && o >= 0;
    o = o < 0 ? 0 : (o >= nz ? nz - 1 : o);
    cj = cj < 0 ? 0 : (cj >= nr ? nr - 1 : cj);
    return cj * pitch + o;
  };

  const int i = i0 + tx, j = j0 + ty;
  double jz = 0.0, jr = 0.0;
  const int ic = i < nz ? i : nz - 1, jc = j < nr ? j : nr - 1;
  const int cell = j * pitch + i, cellc = jc * pitch + ic;
  const bool mine = i < nz && j < nr;

  // per-cell loads first: moments of x^k, and F_bar at rows j-1, j, j+1 (axisymmetric source)
  const A* __restrict__ Min = (const A*)a.M;
  A mraw[3], fb[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) mraw[k] = (Min + k * plane)[cellc];
  if (p.cyl_on) {
    const int cm = jc >= 1 ? cellc - pitch : cellc, cp = jc + 1 < nr ? cellc + pitch : cellc;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fb[k][0] = (W + (W_F + k) * plane)[cm];
      fb[k][1] = (W + (W_F + k) * plane)[cellc];
      fb[k][2] = (W + (W_F + k) * plane)[cp];
    }
  }

  if (p.fields_on) {
    constexpr int NBB = BBR * BBZ, NEB = EBR * EBZ, NRB = RBR * RBZ;
    constexpr int NLB = LBR * LBZ, NLZ = LZR * LZZ, NLR = LRR * LRZ;
    static_assert(NBB <= 2 * NTHREADS && NEB <= 2 * NTHREADS && NRB <= 2 * NTHREADS &&
                      NLB <= 2 * NTHREADS && NLZ <= 2 * NTHREADS && NLR <= 2 * NTHREADS,
                  "two slots per thread cover every LDS region");
    // all halo loads in flight at once (clamped addresses, selected by the flags)
    A rBb[2], rEb[2], rRb[2], rLB[2], rLZ[2], rLR[2];
    bool oBb[2], oEb[2], oRb[2], oLB[2], oLZ[2], oLR[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      int t = min(tid + sl * NTHREADS, NBB - 1);
      rBb[sl] = (W + W_B * plane)[woff(i0 - 1 + t % BBZ, j0 - 1 + t / BBZ, oBb[sl])];
      t = min(tid + sl * NTHREADS, NEB - 1);
      rEb[sl] = (W + W_EZ * plane)[woff(i0 - 1 + t % EBZ, j0 + t / EBZ, oEb[sl])];
      t = min(tid + sl * NTHREADS, NRB - 1);
      rRb[sl] = (W + W_ER * plane)[woff(i0 + t % RBZ, j0 - 1 + t / RBZ, oRb[sl])];
      t = min(tid + sl * NTHREADS, NLB - 1);
      rLB[sl] = (L + 32 * plane)[noff(i0 - 1 + t % LBZ, j0 - 1 + t / LBZ, oLB[sl])];
      t = min(tid + sl * NTHREADS, NLZ - 1);
      rLZ[sl] = (L + 30 * plane)[noff(i0 - 1 + t % LZZ, j0 + t / LZZ, oLZ[sl])];
      t = min(tid + sl * NTHREADS, NLR - 1);
      rLR[sl] = (L + 31 * plane)[noff(i0 + t % LRZ, j0 - 1 + t / LRZ, oLR[sl])];
    }
    pre();
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      int t = tid + sl * NTHREADS;
      if (t < NBB) sBb[t / BBZ][t % BBZ] = oBb[sl] ? (double)rBb[sl] : 0.0;
      if (t < NEB) sEb[t / EBZ][t % EBZ] = oEb[sl] ? (double)rEb[sl] : 0.0;
      if (t < NRB) sRb[t / RBZ][t % RBZ] = oRb[sl] ? (double)rRb[sl] : 0.0;
    }
    __syncthreads();
    // 1/8 of the B_bar of the sites that average the corner (ci, cj) (rear copy rule included)
    auto bsum = [&](int ci, int cj) -> double {
      const int a0 = ci - (i0 - 1), b0 = cj - (j0 - 1);
      double v = sBb[b0][a0] + sBb[b0][a0 + 1] + sBb[b0 + 1][a0] + sBb[b0 + 1][a0 + 1];
      if (!p.per_z && ci == 0) v += sBb[b0][a0] + sBb[b0 + 1][a0];
      return v * 0.125;
    };
    // L_B' = lambda'_B + its use in the fluid's B average
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int t = tid + sl * NTHREADS;
      if (t < NLB) {
        const int ci = i0 - 1 + t % LBZ, cj = j0 - 1 + t / LBZ;
        int cw = ci;
        sLB[t / LBZ][t % LBZ] =
            cellz(cw, cj) ? (oLB[sl] ? (double)rLB[sl] : 0.0) + bsum(ci, cj) : 0.0;
      }
    }
    __syncthreads();
    auto LB = [&](int ci, int cj) -> double { return sLB[cj - (j0 - 1)][ci - (i0 - 1)]; };
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int t = tid + sl * NTHREADS;
      if (t < NLZ) {
        const int ci = i0 - 1 + t % LZZ, cj = j0 + t / LZZ;
        int cw = ci;
        double v = 0.0;
        if (cellz(cw, cj)) {
          const int ea = ci - (i0 - 1), eb = cj - j0;
          v = (oLZ[sl] ? (double)rLZ[sl] : 0.0) + 0.5 * (sEb[eb][ea] + sEb[eb][ea + 1]);
          if (!p.per_z && cw == 0) v += 0.5 * sEb[eb][ea];     // rear copy E_z(-1) = E_z(0)
          if (cj <= nr - 2) v -= dth * LB(ci, cj);
          if (cj >= 1) v += dth * LB(ci, cj - 1);
        }
        sLZ[t / LZZ][t % LZZ] = v;
      }
      if (t < NLR) {
        const int ci = i0 + t % LRZ, cj = j0 - 1 + t / LRZ;
        int cw = ci;
        double v = 0.0;
        if (cellz(cw, cj)) {
          const int ra = ci - i0, rb = cj - (j0 - 1);
          v = (oLR[sl] ? (double)rLR[sl] : 0.0) + 0.5 * (sRb[rb][ra] + sRb[rb + 1][ra]);
          if (p.per_z || cw <= nz - 2) v += dth * LB(ci, cj);
          if (p.per_z || cw >= 1) v -= dth * LB(ci - 1, cj);
        }
        sLR[t / LRZ][t % LRZ] = v;
      }
    }
    __syncthreads();
    if (mine) {
      auto LZ = [&](int ci, int cj) -> double { return sLZ[cj - j0][ci - (i0 - 1)]; };
      auto LR = [&](int ci, int cj) -> double { return sLR[cj - (j0 - 1)][ci - i0]; };
      const double lez = LZ(i, j), ler = LR(i, j);
      double lb = LB(i, j) + bsum(i, j);
      const double rj = (j + 0.5) * h;
      lb += dt * (j + 1.0) / rj * lez;
      if (j + 1 < nr) lb -= dt * (j + 1.0) / ((j + 1.5) * h) * LZ(i, j + 1);
      if (p.per_z || i >= 1) lb -= dth * ler;
      if (p.per_z || i + 1 < nz) lb += dth * LR(i + 1, j);
      stv(&(Lo + 30 * plane)[cell], lez);
      stv(&(Lo + 31 * plane)[cell], ler);
      stv(&(Lo + 32 * plane)[cell], lb);
      jz = 0.5 * dt * (lez + ((p.per_z || i >= 1) ? LZ(i - 1, j) : 0.0));
      if (!p.per_z && !p.window && i == nz - 1) jz += 0.5 * dt * lez;   // front copy of J_z
      jr = 0.5 * dt * (ler + (j >= 1 ? LR(i, j - 1) : 0.0));
      if (j == nr - 1) jr += 0.5 * dt * ler;                             // outer copy of J_r
      // driver current J_b(z_i + dz/2, r_j, t_{k-1/2})
      double dsr, dnb;
      ddriver(p, ((double)(a.s + i) + 0.5) * h, rj, ((double)a.k - 0.5) * dt, dsr, dnb);
      part[2] += dt * lez * dsr;
      part[3] += dt * lez * dnb;
    }
  } else {
    pre();
    if (mine) {
      // fields are carried unchanged and unused
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bool ok;
        const int o = noff(i, j, ok);
        stv(&(Lo + (30 + c) * plane)[cell], ok ? (double)(L + (30 + c) * plane)[o] : 0.0);
      }
    }
  }
  mb_out[0] = mb_out[1] = mb_out[2] = 0;
  if (!mine) return;   // no barrier below this point

  // ---- lambda of the moments ----
  const double M[3] = {(double)mraw[0] + nbg(p, (double)(a.s + i) * h), (double)mraw[1], (double)mraw[2]};
  double Mb[3] = {0.0, 0.0, 0.0};
  // (a) face currents of Ampere's law
  if (p.fields_on) current_vjp(p, M, jz, jr, Mb);
  // (b) lagged radial gradient of the axisymmetric source, D (M(j+1) - M(j-1)) / (2 dr r_j)
  if (p.cyl_on) {
    const double c = p.D / (2.0 * h);
    const double par[3] = {1.0, 1.0, -1.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double v = 0.0;
      if (j >= 1) v += c / ((j - 0.5) * h) * (double)fb[k][0];
      if (j + 1 < nr) v -= c / ((j + 1.5) * h) * (double)fb[k][2];
      if (j == 0) v -= par[k] * c / (0.5 * h) * (double)fb[k][1];
      if (j == nr - 1) v += c / ((j + 0.5) * h) * (double)fb[k][1];
      Mb[k] += v;
    }
  }
  // (c) equilibrium ghosts whose moments are copies (or the axis mirror) of this cell: the ghost
  // positions outside a non-periodic edge whose source is this cell, each pulled by the computed
  // site ghost + xi_q.  A side ghost is pulled in the three directions that point back into the
  // domain, a corner ghost in one.  The front ghost of the moving window is plasma at rest and
  // depends on theta only.
  const bool zlo = !p.per_z && i == 0, zhi = !p.per_z && !p.window && i == nz - 1;
  const bool rlo = !p.per_r && j == 0, rhi = !p.per_r && j == nr - 1;
  if (zlo || zhi || rlo || rhi) {
    const int gz = zlo ? -1 : nz, gr = rlo ? -1 : nr;
    // slots 0..2: the r-side ghost (i, gr); 3..5: the z-side ghost (gz, j); 6: the corner (gz, gr)
    int gsi[7], gsj[7], gq[7], yo[7];
    bool gv[7];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gsi[c] = i;
      gsj[c] = gr;
      gq[c] = rlo ? (c == 0 ? 2 : (c == 1 ? 5 : 6)) : (c == 0 ? 4 : (c == 1 ? 7 : 8));
      gv[c] = rlo || rhi;
      gsi[3 + c] = gz;
      gsj[3 + c] = j;
      gq[3 + c] = zlo ? (c == 0 ? 1 : (c == 1 ? 5 : 8)) : (c == 0 ? 3 : (c == 1 ? 6 : 7));
      gv[3 + c] = zlo || zhi;
    }
    gsi[6] = gz;
    gsj[6] = gr;
    gq[6] = zlo ? (rlo ? 5 : 8) : (rlo ? 6 : 7);
    gv[6] = (zlo || zhi) && (rlo || rhi);
    A af[7][3];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      int yi = gsi[c] + XZ(gq[c]), yj = gsj[c] + XR(gq[c]);
      if (p.per_z) yi = wrap1(yi, nz);
      else gv[c] = gv[c] && yi >= 0 && yi < nz;
      if (p.per_r) yj = wrap1(yj, nr);
      else gv[c] = gv[c] && yj >= 0 && yj < nr;
      gv[c] = gv[c] && !(a.shift && yi == 0);   // a computed site
      yi = yi < 0 ? 0 : (yi >= nz ? nz - 1 : yi);
      yj = yj < 0 ? 0 : (yj >= nr ? nr - 1 : yj);
      yo[c] = yj * pitch + yi;
#pragma unroll
      for (int k = 0; k < 3; ++k) af[c][k] = (Lo + (9 * k + gq[c]) * plane)[yo[c]];
    }
    // VJP of f_eq_{k,q}(Mg) = w_q Mg_k (1 + Q_q(u)), u = lam beta(Mg), Mg = (M0, M1, +-M2); the
    // velocity of the mirrored moments is (beta_z, -beta_r)
    double bz, br;
    const bool live = velocity<double>(M[0], M[1], M[2], p.n_floor, bz, br);
    const double n = M[0];
    const double in = live ? 1.0 / n : 0.0;
    const double pz = M[1] * in, pr0 = M[2] * in;
    const double g2 = 1.0 + pz * pz + pr0 * pr0, ig = live ? 1.0 / sqrt(g2) : 0.0, ig3 = ig * ig * ig;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      if (!gv[c]) continue;
      const int q = gq[c];
      const double sgn = gsj[c] < 0 ? -1.0 : 1.0;
      const double w = WQ<double>(q);
      const double uz = p.lam * bz, ur = p.lam * sgn * br, pr = sgn * pr0;
      const double Mg[3] = {M[0], M[1], sgn * M[2]};
      const double cu = XZ(q) * uz + XR(q) * ur;
      const double Q = 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur);
      double Mgb[3], ubz = 0.0, ubr = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double ak = (double)af[c][k];
        Mgb[k] = ak * w * (1.0 + Q);
        const double sk = ak * w * Mg[k];
        ubz += sk * (3.0 * XZ(q) + 9.0 * cu * XZ(q) - 3.0 * uz);
        ubr += sk * (3.0 * XR(q) + 9.0 * cu * XR(q) - 3.0 * ur);
      }
      if (live) {
        const double bbz = p.lam * ubz, bbr = p.lam * ubr;
        const double pdot = pz * bbz + pr * bbr;
        const double pbz = bbz * ig - pz * pdot * ig3, pbr = bbr * ig - pr * pdot * ig3;
        Mgb[1] += pbz * in;
        Mgb[2] += pbr * in;
        Mgb[0] -= (pbz * pz + pbr * pr) * in;
      }
      Mb[0] += Mgb[0];
      Mb[1] += Mgb[1];
      Mb[2] += sgn * Mgb[2];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    stv(&(Lo + (27 + k) * plane)[cell], Mb[k]);
    mb_out[k] = (A)Mb[k];   // as stored, so the fused step reads what a split one would
  }
}

template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_cell_kernel(AdjArgs a) {
  const int gx = (a.p.nz + TZ - 1) / TZ, gy = (a.p.nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  typename Mode<ST, false>::C mb[3];
  cell_body<ST>(a, (tile % gx) * TZ, (tile / gx) * TR, part, mb, [] {});
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// Fused reverse work of two consecutive steps: the cell part of step k (ac, cells of x^k) and the
// site part of step k - 1 (as, sites of x^{k-1}).  Thread (tx, ty) takes cell o = o0 + tx of x^k
// and the site o + shift_{k-1} of x^{k-1}, whose output is that cell, so the site part takes
// M_bar^k from the cell part's registers.  ac.lam and as.lam_next are the same buffer (lambda^k):
// the cell part writes its planes 27..32, the site part reads planes 0..26 (written by the
// previous launch) and writes f_bar^{k-1} into as.lam, whose planes 30..32 (lambda^{k+1}) the cell
// part reads; the two steps use different work buffers.
// The site step's arguments arrive without their physics (the same as ac.p), which keeps the
// kernel's uniform values to one copy of the physics.
template <int ST, int COLL>
__device__ __forceinline__ void fused_body(const AdjArgs& ac, const AdjStep& ss) {
  AdjArgs as;
  as.p = ac.p;
  as.k = ss.k;
  as.s = ss.s;
  as.shift = ss.shift;
  as.pull_in = ss.pull_in;
  as.g = ss.g;
  as.M = ss.M;
  as.E = ss.E;
  as.lam_next = ss.lam_next;
  as.lam = ss.lam;
  as.work = ss.work;
  as.site = ss.site;
  as.partials = ss.partials;
  const int gx = (ac.p.nz + TZ - 1) / TZ, gy = (ac.p.nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int o0 = (tile % gx) * TZ, j0 = (tile / gx) * TR;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  typename Mode<ST, false>::C mb[3];
  // The site part's loads go in flight during the cell part (FP32 and FP16 storage: 121 VGPRs, the
  // four wavefronts per SIMD that a C4-sized grid holds anyway; C4 adjoint/forward 3.49 -> 3.28).
  // FP64 would need 54 more registers for them, so it loads after the cell part.
  SiteIn<ST> in;
  if constexpr (ST == 0) {
    cell_body<ST>(ac, o0, j0, part, mb, [] {});
    site_load<ST>(as, o0 + as.shift, j0, false, in);
  } else {
    cell_body<ST>(ac, o0, j0, part, mb, [&] { site_load<ST>(as, o0 + as.shift, j0, false, in); });
  }
  const Physics& p = ac.p;
  if (p.window && as.shift && o0 + (int)threadIdx.x % TZ == p.nz - 1 && j0 + (int)threadIdx.x / TZ < p.nr) {
    // this cell is the front column that step k - 1's window shift created (density n_bg):
    // the moment-adjoint part of its theta partial (the population part is in site_body)
    double dl, dn;
    dnbg(p, (double)(as.s + p.nz) * p.h, dl, dn);
    part[0] += mb[0] * dl;
    part[1] += mb[0] * dn;
  }
  site_body<ST, COLL>(as, o0 + as.shift, j0, mb, part, in);
  block_sum4(part, as.partials + (long long)blockIdx.x * 4);
}

template <int ST, int COLL>
__global__ __launch_bounds__(NTHREADS) void adj_fused_kernel(AdjArgs ac, AdjStep ss) {
  fused_body<ST, COLL>(ac, ss);
}

// FP32 and FP16 storage: held to 128 VGPRs (4 waves per SIMD), where the kernel fits without
// spills; one register more would drop it to 3 waves per SIMD.
template <int ST, int COLL>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(4))) void adj_fused4_kernel(AdjArgs ac,
                                                                                                     AdjStep ss) {
  fused_body<ST, COLL>(ac, ss);
}

// ------------------------------------------------------------------------------------------
// adj_state_kernel: lambda^k in the stored-state layout, FP64, one thread per cell:
// g_bar^k(x, q) = f_bar^k(x + xi_q, q) over the sites computed in step k, moments and fields copied.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_state_kernel(AdjArgs a, double* out) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int i = blockIdx.x * TZ + threadIdx.x % TZ, j = blockIdx.y * TR + threadIdx.x / TZ;
  if (i >= nz || j >= nr) return;
  const A* __restrict__ L = (const A*)a.lam;
  const int cell = j * pitch + i;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int yi = i + XZ(q), yj = j + XR(q);
    bool ok = true;
    if (p.per_z) yi = wrap1(yi, nz);
    else ok = ok && yi >= 0 && yi < nz;
    if (p.per_r) yj = wrap1(yj, nr);
    else ok = ok && yj >= 0 && yj < nr;
    ok = ok && !(a.shift && yi == 0);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
      out[(9 * kk + q) * plane + cell] = ok ? (double)L[(9 * kk + q) * plane + yj * pitch + yi] : 0.0;
  }
  for (int c = 27; c < 33; ++c) out[c * plane + cell] = (double)L[c * plane + cell];
}

// adj_cast_kernel: an FP64 stored-state lambda into the adjoint precision (33 planes)
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_cast_kernel(Physics p, const double* in, void* out) {
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * TZ + threadIdx.x % TZ, j = blockIdx.y * TR + threadIdx.x / TZ;
  if (i >= p.nz || j >= p.nr) return;
  const int cell = j * p.pitch + i;
#pragma unroll
  for (int c = 0; c < 33; ++c) stv(&((A*)out)[c * p.plane + cell], in[c * p.plane + cell]);
}

// ------------------------------------------------------------------------------------------
// adj_init_cell_kernel: theta partials of the initial populations and moments, one thread per cell
// (n_init = n_bg (1 + delta) at the initial momentum, populations at equilibrium).
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_init_cell_kernel(AdjArgs a) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int gx = (nz + TZ - 1) / TZ, gy = (nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int i = (tile % gx) * TZ + threadIdx.x % TZ, j = (tile / gx) * TR + threadIdx.x / TZ;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < nz && j < nr) {
    const A* __restrict__ L = (const A*)a.lam_next;   // lambda^0
    const A* __restrict__ Min = (const A*)a.M;
    const int cell = j * pitch + i;
    const double z = (double)i * p.h;
    const double nb0 = nbg(p, z);
    double dl, dn;
    dnbg(p, z, dl, dn);
    const double n = (double)Min[cell] + nb0;
    const double m1 = Min[plane + cell], m2 = Min[2 * plane + cell];
    double bz, br;
    const bool live = velocity<double>(n, m1, m2, p.n_floor, bz, br);
    const double pz = live ? m1 / n : 0.0, pr = live ? m2 / n : 0.0;
    const double uz = p.lam * bz, ur = p.lam * br;
    double nbar = (double)L[27 * plane + cell] + pz * (double)L[28 * plane + cell] +
                  pr * (double)L[29 * plane + cell];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      // adjoint of the stored population g^0(x, q): direct, or the transposed pull of f_bar^0
      int yi = i, yj = j;
      bool ok = true;
      if (a.pull_in) {
        yi += XZ(q);
        yj += XR(q);
        if (p.per_z) yi = wrap1(yi, nz);
        else ok = ok && yi >= 0 && yi < nz;
        if (p.per_r) yj = wrap1(yj, nr);
        else ok = ok && yj >= 0 && yj < nr;
        ok = ok && !(a.shift && yi == 0);
      }
      if (!ok) continue;
      const int ys = yj * pitch + yi;
      const double cu = XZ(q) * uz + XR(q) * ur;
      const double e = WQ<double>(q) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur));
      nbar += e * ((double)L[q * plane + ys] + pz * (double)L[(9 + q) * plane + ys] +
                   pr * (double)L[(18 + q) * plane + ys]);
    }
    if (nb0 > 0.0) {
      const double ratio = n / nb0;   // 1 + delta
      part[0] += nbar * ratio * dl;
      part[1] += nbar * ratio * dn;
    }
  }
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// adj_init_field_kernel: theta partials of the initial driver fields, one thread per column.
// E_r^{-1}(j) = -h / (j+1) sum_{j' <= j} (j' + 1/2) n_b(z_i, r_j', -dt); B^{-1/2} likewise at
// z_i + dz/2, -dt/2.  The driver is separable: n_b = nb e_z(z, t) e_r(r).
template <int ST>
__global__ __launch_bounds__(64) void adj_init_field_kernel(AdjArgs a) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int i = blockIdx.x * 64 + threadIdx.x;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < p.nz && p.fields_on) {
    const A* __restrict__ L = (const A*)a.lam_next;
    const long long plane = p.plane;
    const double h = p.h, dt = p.dt;
    const double z = (double)i * h;
    const double d1 = z - (p.zd0 - dt), d2 = z + 0.5 * h - (p.zd0 - 0.5 * dt);
    const double ez1 = exp(-(d1 * d1) / (2.0 * p.sigma_z * p.sigma_z));
    const double ez2 = exp(-(d2 * d2) / (2.0 * p.sigma_z * p.sigma_z));
    const double s3 = p.sigma_r * p.sigma_r * p.sigma_r;
    double c0 = 0.0, c1 = 0.0;   // sum_{j' <= j} (j' + 1/2) e_r r^2 / sigma_r^3, (j' + 1/2) e_r
    for (int j = 0; j < p.nr; ++j) {
      const double r = (j + 0.5) * h;
      const double er = exp(-(r * r) / (2.0 * p.sigma_r * p.sigma_r));
      c0 += (j + 0.5) * er * r * r / s3;
      c1 += (j + 0.5) * er;
      const int cell = j * p.pitch + i;
      const double f = -h / (j + 1.0);
      const double l31 = (double)L[31 * plane + cell], l32 = (double)L[32 * plane + cell];
      // d/d(sigma_r): nb e_z e_r r^2 / sigma_r^3 ; d/d(n_b): e_z e_r
      part[2] += f * p.nb * c0 * (l31 * ez1 + l32 * ez2);
      part[3] += f * c1 * (l31 * ez1 + l32 * ez2);
    }
  }
  // block of 64 threads = one wavefront
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < 4; ++c) part[c] += __shfl_down(part[c], off, 64);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) a.partials[(long long)blockIdx.x * 4 + c] += part[c];
}

// sum of per-block partials (fixed order) added into acc[4]
__global__ __launch_bounds__(NTHREADS) void partials_sum_kernel(const double* partials, int nblocks,
                                                                double* acc) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += NTHREADS)
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] += partials[(long long)b * 4 + c];
  // block_sum4 adds into acc from thread 0 only, after its own barrier
  block_sum4(v, acc);
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static int step_blocks(const Physics& p) {
  return ((p.nz + TZ - 1) / TZ) * ((p.nr + TR - 1) / TR);
}

int adjoint_partial_blocks(const Physics& p) { return step_blocks(p); }

#define ADJ_DISPATCH(storage, KERNEL, GRID, BLOCK, STREAM, ...)                      \
  do {                                                                               \
    if ((storage) == 0) KERNEL<0><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);    \
    else if ((storage) == 1) KERNEL<1><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__); \
    else KERNEL<2><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);                   \
  } while (0)

// a.partials holds 2 * adjoint_partial_blocks(p) accumulators of 4 doubles (site kernel, then
// cell kernel); they must be zero before the first step and are summed by adjoint_reduce.
// The site part with the run's collision operator.
template <int COLL>
static void site_launch_c(int storage, dim3 grid, hipStream_t st, const AdjArgs& a) {
  if (storage == 0) adj_site_kernel<0, COLL><<<grid, NTHREADS, 0, st>>>(a);
  else if (storage == 1) adj_site_kernel<1, COLL><<<grid, NTHREADS, 0, st>>>(a);
  else adj_site_kernel<2, COLL><<<grid, NTHREADS, 0, st>>>(a);
}
static void site_launch(int storage, dim3 grid, hipStream_t st, const AdjArgs& a) {
  if (a.p.coll == 1) site_launch_c<1>(storage, grid, st, a);
  else if (a.p.coll == 2) site_launch_c<2>(storage, grid, st, a);
  else if (a.p.coll == 3) site_launch_c<3>(storage, grid, st, a);
  else site_launch_c<0>(storage, grid, st, a);
}
template <int COLL>
static void fused_launch_c(int storage, dim3 grid, hipStream_t st, const AdjArgs& cell, const AdjStep& ss) {
  if (storage == 0) adj_fused_kernel<0, COLL><<<grid, NTHREADS, 0, st>>>(cell, ss);
  else if (storage == 1) adj_fused4_kernel<1, COLL><<<grid, NTHREADS, 0, st>>>(cell, ss);
  else adj_fused4_kernel<2, COLL><<<grid, NTHREADS, 0, st>>>(cell, ss);
}

hipError_t launch_adjoint_step(int storage, const AdjArgs& a, hipStream_t st) {
  const int nb = step_blocks(a.p);
  site_launch(storage, dim3(nb), st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  AdjArgs b = a;
  b.partials = a.partials + (long long)adjoint_partial_blocks(a.p) * 4;
  ADJ_DISPATCH(storage, adj_cell_kernel, dim3(nb), NTHREADS, st, b);
  return hipGetLastError();
}

hipError_t launch_adjoint_site(int storage, const AdjArgs& a, hipStream_t st) {
  site_launch(storage, dim3(step_blocks(a.p)), st, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_cell(int storage, const AdjArgs& a, hipStream_t st) {
  AdjArgs b = a;
  b.partials = a.partials + (long long)adjoint_partial_blocks(a.p) * 4;
  ADJ_DISPATCH(storage, adj_cell_kernel, dim3(step_blocks(a.p)), NTHREADS, st, b);
  return hipGetLastError();
}

hipError_t launch_adjoint_fused(int storage, const AdjArgs& cell, const AdjArgs& site, hipStream_t st) {
  const AdjStep ss{site.k, site.s, site.shift, site.pull_in, site.g, site.M, site.E,
                   site.lam_next, site.lam, site.work, site.site, site.partials};
  const dim3 grid(step_blocks(cell.p));
  if (cell.p.coll == 1) fused_launch_c<1>(storage, grid, st, cell, ss);
  else if (cell.p.coll == 2) fused_launch_c<2>(storage, grid, st, cell, ss);
  else if (cell.p.coll == 3) fused_launch_c<3>(storage, grid, st, cell, ss);
  else fused_launch_c<0>(storage, grid, st, cell, ss);
  return hipGetLastError();
}

hipError_t launch_adjoint_init(int storage, const AdjArgs& a, hipStream_t st) {
  ADJ_DISPATCH(storage, adj_init_cell_kernel, dim3(step_blocks(a.p)), NTHREADS, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  AdjArgs b = a;
  b.partials = a.partials + (long long)adjoint_partial_blocks(a.p) * 4;
  ADJ_DISPATCH(storage, adj_init_field_kernel, dim3((a.p.nz + 63) / 64), 64, st, b);
  return hipGetLastError();
}

hipError_t launch_adjoint_state(int storage, const AdjArgs& a, double* out, hipStream_t st) {
  const dim3 grid((a.p.nz + TZ - 1) / TZ, (a.p.nr + TR - 1) / TR);
  ADJ_DISPATCH(storage, adj_state_kernel, grid, NTHREADS, st, a, out);
  return hipGetLastError();
}

hipError_t launch_adjoint_cast(int storage, const Physics& p, const double* in, void* out, hipStream_t st) {
  const dim3 grid((p.nz + TZ - 1) / TZ, (p.nr + TR - 1) / TR);
  ADJ_DISPATCH(storage, adj_cast_kernel, grid, NTHREADS, st, p, in, out);
  return hipGetLastError();
}

hipError_t adjoint_reduce(const Physics& p, const double* partials, double* grad_acc, hipStream_t st) {
  partials_sum_kernel<<<1, NTHREADS, 0, st>>>(partials, 2 * adjoint_partial_blocks(p), grad_acc);
  return hipGetLastError();
}

}  // namespace lbm
