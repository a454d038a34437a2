// Hand-written discrete adjoint of the lattice-Boltzmann plasma-wakefield step (gfx950).
//
// For the state x^k = (g^{k-1}, A*^{k-1}, E^{k-1}, B^{k-1/2}) and the step x^{k+1} = Phi(x^k; theta)
// of the forward kernel, these kernels compute lambda^k = (dPhi/dx^k)^T lambda^{k+1} and the
// parameter partials (dPhi/dtheta)^T lambda^{k+1}, theta = (ramp length, n0, sigma_r, n_b), in FP64.
// All variables are the raw populations, moments and fields (the deviation encoding of the stored
// density lattice is an identity map for the adjoint).  Gather form throughout: every output has
// a single writer, no atomics, fixed summation order (bit-reproducible).
//
//   adj_site_kernel   per fluid site: recompute the field tile (Ampere, Faraday) and the site's
//                     forward collision, then the VJP of the collision: A_bar (3, through the
//                     zeroth moments), F_bar (3, source terms), and the adjoints of the site fields
//                     E_bar_z, E_bar_r, B_bar; theta partials of the window-front ghost and of the
//                     new front column.
//   adj_field_kernel  transposes of the site averages, Faraday and Ampere (with every ghost rule):
//                     lambda_E, lambda_B and the adjoint of the face currents; theta partials of
//                     the driver current.
//   adj_pop_kernel    transpose of the pull (a gather of (1 - 1/tau) g'_bar + A_bar from the site
//                     each population streams to), and lambda of the moments: current, the lagged
//                     radial gradient of the axisymmetric source, and the equilibrium ghosts.
//   adj_init_kernel   theta partials of the initial state.
#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

// work planes written by adj_site_kernel / adj_field_kernel
constexpr int W_A = 0, W_F = 3, W_EZ = 6, W_ER = 7, W_B = 8, W_JZ = 9, W_JR = 10;

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
  const double zr = exp(-(dz * dz) / (2.0 * p.sigma_z * p.sigma_z)) *
                    exp(-(r * r) / (2.0 * p.sigma_r * p.sigma_r));
  dnb = zr;
  dsr = p.nb * zr * r * r / (p.sigma_r * p.sigma_r * p.sigma_r);
}

__device__ __forceinline__ void block_sum4(double v[4], double* out) {
  __shared__ double red[NTHREADS / 64][4];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  for (int off = 32; off > 0; off >>= 1)
    for (int c = 0; c < 4; ++c) v[c] += __shfl_down(v[c], off, 64);
  if (lane == 0)
    for (int c = 0; c < 4; ++c) red[wid][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < NTHREADS / 64; ++w)
      for (int c = 0; c < 4; ++c) r[c] += red[w][c];
    for (int c = 0; c < 4; ++c) out[c] = r[c];
  }
}

// VJP of f_eq_q(M) (all three lattices at once) with respect to the moments M:
// f_eq_{k,q} = w_q M_k (1 + Q_q(u)), u = lam beta(M).  a[k] is the adjoint of f_eq_{k,q}.
__device__ __forceinline__ void feq_vjp(const Physics& p, int q, const double M[3], const double a[3],
                                        double Mbar[3]) {
  const double w = WQ<double>(q);
  double bz, br;
  const bool live = velocity<double>(M[0], M[1], M[2], p.n_floor, bz, br);
  const double uz = p.lam * bz, ur = p.lam * br;
  const double cu = XZ(q) * uz + XR(q) * ur;
  const double Q = 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur);
  double ubz = 0.0, ubr = 0.0;
  for (int k = 0; k < 3; ++k) {
    Mbar[k] += a[k] * w * (1.0 + Q);
    const double s = a[k] * w * M[k];
    ubz += s * (3.0 * XZ(q) + 9.0 * cu * XZ(q) - 3.0 * uz);
    ubr += s * (3.0 * XR(q) + 9.0 * cu * XR(q) - 3.0 * ur);
  }
  if (live) {
    const double n = M[0], pz = M[1] / n, pr = M[2] / n;
    const double g2 = 1.0 + pz * pz + pr * pr, ig = 1.0 / sqrt(g2), ig3 = ig / g2;
    const double bbz = p.lam * ubz, bbr = p.lam * ubr;
    const double pdot = pz * bbz + pr * bbr;
    const double pbz = bbz * ig - pz * pdot * ig3, pbr = bbr * ig - pr * pdot * ig3;
    Mbar[1] += pbz / n;
    Mbar[2] += pbr / n;
    Mbar[0] -= (pbz * pz + pbr * pr) / n;
  }
}

// VJP of J = n beta(M) (the face current of Ampere's law) with respect to M.
__device__ __forceinline__ void current_vjp(const Physics& p, const double M[3], double jzb, double jrb,
                                            double Mbar[3]) {
  double bz, br;
  if (!velocity<double>(M[0], M[1], M[2], p.n_floor, bz, br)) return;
  const double n = M[0], pz = M[1] / n, pr = M[2] / n;
  const double g2 = 1.0 + pz * pz + pr * pr, ig = 1.0 / sqrt(g2), ig3 = ig / g2;
  // J_a = n p_a / gamma: dJ_a/dp_b = n (delta_ab / gamma - p_a p_b / gamma^3), dJ_a/dn|_p = beta_a
  const double jdot = jzb * pz + jrb * pr;
  const double pbz = n * (jzb * ig - pz * jdot * ig3), pbr = n * (jrb * ig - pr * jdot * ig3);
  const double nbar = jzb * bz + jrb * br;
  Mbar[1] += pbz / n;
  Mbar[2] += pbr / n;
  Mbar[0] += nbar - (pbz * pz + pbr * pr) / n;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// adj_site_kernel: one thread per logical fluid site (i, j) of x^k.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_site_kernel(AdjArgs a) {
  using S = typename Mode<ST, false>::S;
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  constexpr int MZ = TZ + 2, MR = TR + 2;
  constexpr int BZ = TZ + 3, BR = TR + 3;
  constexpr int EZZ = TZ + 1, EZR = TR + 2;
  constexpr int ERZ = TZ + 2, ERR = TR + 1;
  constexpr int BNZ = TZ + 1, BNR = TR + 1;
  __shared__ double sM[3][MR][MZ];   // raw moments with the ghost ring
  __shared__ double sJ[2][MR][MZ];
  __shared__ double sBo[BR][BZ];
  __shared__ double sEz[EZR][EZZ];
  __shared__ double sEr[ERR][ERZ];
  __shared__ double sBn[BNR][BNZ];
  __shared__ double sN[MZ];

  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int gx = (nz + TZ - 1) / TZ, gy = (nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int i0 = (tile % gx) * TZ;   // logical columns of x^k
  const int j0 = (tile / gx) * TR;
  const int tid = threadIdx.x, tx = tid % TZ, ty = tid / TZ;
  const double h = p.h, dt = p.dt;
  const A* Min = (const A*)a.M;
  const A* Ein = (const A*)a.E;
  const S* gin = (const S*)a.g;
  auto zcol = [&](int i) { return p.per_z ? wrapi(i, nz) : (i < 0 ? 0 : (i < nz ? i : nz - 1)); };
  auto rrow = [&](int j) { return p.per_r ? wrapi(j, nr) : (j < 0 ? 0 : (j < nr ? j : nr - 1)); };

  for (int t = tid; t < MZ; t += NTHREADS) {
    const int ii = i0 - 1 + t;
    sN[t] = nbg(p, (double)(a.s + (p.per_z ? wrapi(ii, nz) : ii)) * h);
  }
  __syncthreads();
  for (int t = tid; t < MR * MZ; t += NTHREADS) {
    const int bb = t / MZ, aa = t % MZ;
    const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
    const int ci = zcol(ii), rj = rrow(jj);
    const int off = rj * pitch + ci;
    double m0 = (double)Min[off] + nbg(p, (double)(a.s + ci) * h);
    double m1 = (double)Min[plane + off], m2 = (double)Min[2 * plane + off];
    if (!p.per_z && p.window && ii == nz) { m0 = sN[aa]; m1 = 0.0; m2 = 0.0; }
    if (!p.per_r && jj < 0) m2 = -m2;
    sM[0][bb][aa] = m0;
    sM[1][bb][aa] = m1;
    sM[2][bb][aa] = m2;
    double bz, br;
    velocity<double>(m0, m1, m2, p.n_floor, bz, br);
    sJ[0][bb][aa] = m0 * bz;
    sJ[1][bb][aa] = m0 * br;
  }
  if (p.fields_on) {
    for (int t = tid; t < BR * BZ; t += NTHREADS) {
      const int bb = t / BZ, aa = t % BZ;
      const int jj = j0 - 2 + bb;
      sBo[bb][aa] = jj < 0 ? 0.0 : (double)Ein[2 * plane + rrow(jj) * pitch + zcol(i0 - 2 + aa)];
    }
    for (int t = tid; t < EZR * EZZ; t += NTHREADS) {
      const int bb = t / EZZ, aa = t % EZZ;
      sEz[bb][aa] = (double)Ein[rrow(j0 - 1 + bb) * pitch + zcol(i0 - 1 + aa)];
    }
    for (int t = tid; t < ERR * ERZ; t += NTHREADS) {
      const int bb = t / ERZ, aa = t % ERZ;
      sEr[bb][aa] = (double)Ein[plane + rrow(j0 - 1 + bb) * pitch + zcol(i0 - 1 + aa)];
    }
    __syncthreads();
    const double tb = ((double)a.k - 0.5) * dt;
    for (int t = tid; t < EZR * EZZ; t += NTHREADS) {
      const int bb = t / EZZ, aa = t % EZZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr) {
        const double rj = (jj + 0.5) * h;
        const double curl = ((jj + 1.0) * sBo[bb + 1][aa + 1] - jj * sBo[bb][aa + 1]) / rj;
        const double jf = 0.5 * (sJ[0][bb][aa] + sJ[0][bb][aa + 1]);
        const int ci = p.per_z ? wrapi(ii, nz) : ii;
        const double jb = driver<double>(p, ((double)(a.s + ci) + 0.5) * h, rj, tb);
        sEz[bb][aa] = sEz[bb][aa] + dt * (curl + jf + jb);
      }
    }
    for (int t = tid; t < ERR * ERZ; t += NTHREADS) {
      const int bb = t / ERZ, aa = t % ERZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr) {
        const double curl = -(sBo[bb + 1][aa + 1] - sBo[bb + 1][aa]) / h;
        const double jf = 0.5 * (sJ[1][bb][aa] + sJ[1][bb + 1][aa]);
        sEr[bb][aa] = sEr[bb][aa] + dt * (curl + jf);
      }
    }
    __syncthreads();
    if (!p.per_z) {
      if (i0 == 0)
        for (int bb = tid; bb < EZR; bb += NTHREADS) sEz[bb][0] = sEz[bb][1];
      const int af = nz - (i0 - 1);
      if (af >= 1 && af < ERZ)
        for (int bb = tid; bb < ERR; bb += NTHREADS) sEr[bb][af] = sEr[bb][af - 1];
    }
    __syncthreads();
    {
      const int bo = nr - (j0 - 1);
      if (bo >= 1 && bo < EZR)
        for (int aa = tid; aa < EZZ; aa += NTHREADS) sEz[bo][aa] = sEz[bo - 1][aa];
    }
    if (j0 == 0)
      for (int aa = tid; aa < ERZ; aa += NTHREADS) sEr[0][aa] = 0.0;
    __syncthreads();
    for (int t = tid; t < BNR * BNZ; t += NTHREADS) {
      const int bb = t / BNZ, aa = t % BNZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      double v = 0.0;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr)
        v = sBo[bb + 1][aa + 1] + dt * ((sEz[bb + 1][aa] - sEz[bb][aa]) / h - (sEr[bb][aa + 1] - sEr[bb][aa]) / h);
      sBn[bb][aa] = v;
    }
    __syncthreads();
    if (!p.per_z && i0 == 0)
      for (int bb = tid; bb < BNR; bb += NTHREADS) sBn[bb][0] = sBn[bb][1];
  }
  __syncthreads();

  const int i = i0 + tx, j = j0 + ty;
  double part[4] = {0.0, 0.0, 0.0, 0.0};   // d/d(ramp_len, n0, sigma_r, n_b)
  if (i < nz && j < nr) {
    const int cell = j * pitch + i;
    double* W = a.work;
    if (a.shift && i == 0) {
      // the first column leaves the window in this step: no site, no adjoint source
      for (int c = 0; c < 9; ++c) W[c * plane + cell] = 0.0;
    } else {
      const int oo = j * pitch + (i - a.shift);   // index of the site's output in x^{k+1}
      const double* L = a.lam_next;
      // forward recompute of the site (raw values)
      double f[3][9];
      for (int q = 0; q < 9; ++q) {
        const int si = i - XZ(q), sj = j - XR(q);
        const bool oz = si < 0 || si >= nz, orr = sj < 0 || sj >= nr;
        if ((oz && !p.per_z) || (orr && !p.per_r)) {
          const int ga = tx + 1 - XZ(q), gb = ty + 1 - XR(q);
          const double Mg[3] = {sM[0][gb][ga], sM[1][gb][ga], sM[2][gb][ga]};
          double bz, br;
          velocity<double>(Mg[0], Mg[1], Mg[2], p.n_floor, bz, br);
          const double uz = p.lam * bz, ur = p.lam * br;
          const double cu = XZ(q) * uz + XR(q) * ur;
          const double Q = 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur);
          for (int k = 0; k < 3; ++k) f[k][q] = WQ<double>(q) * Mg[k] * (1.0 + Q);
        } else {
          const int pi = oz ? wrapi(si, nz) : si, pj = orr ? wrapi(sj, nr) : sj;
          const int off = pj * pitch + pi;
          f[0][q] = (double)ldv(gin[q * plane + off]) + WQ<double>(q) * sN[tx + 1 - XZ(q)];
          f[1][q] = (double)ldv(gin[(9 + q) * plane + off]);
          f[2][q] = (double)ldv(gin[(18 + q) * plane + off]);
        }
      }
      double Am[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < 3; ++k)
        for (int q = 0; q < 9; ++q) Am[k] += f[k][q];
      const double n = Am[0];
      double bz, br;
      const bool live = velocity<double>(Am[0], Am[1], Am[2], p.n_floor, bz, br);
      const double uz = p.lam * bz, ur = p.lam * br;
      double pz = 0.0, pr = 0.0, ig = 1.0;
      if (live) {
        pz = Am[1] / n;
        pr = Am[2] / n;
        ig = 1.0 / sqrt(1.0 + pz * pz + pr * pr);
      }
      double Ebz = 0.0, Ebr = 0.0, Bb = 0.0;
      if (p.fields_on) {
        Ebz = 0.5 * (sEz[ty + 1][tx] + sEz[ty + 1][tx + 1]);
        Ebr = 0.5 * (sEr[ty][tx + 1] + sEr[ty + 1][tx + 1]);
        Bb = ((sBo[ty + 2][tx + 2] + sBn[ty + 1][tx + 1]) + (sBo[ty + 2][tx + 1] + sBn[ty + 1][tx]) +
              (sBo[ty + 1][tx + 2] + sBn[ty][tx + 1]) + (sBo[ty + 1][tx + 1] + sBn[ty][tx])) / 8.0;
      }
      const double ir = 1.0 / ((j + 0.5) * h);

      // adjoint inputs
      double gb[3][9], Mb[3], Fb[3], Ab[3];
      for (int k = 0; k < 3; ++k) {
        for (int q = 0; q < 9; ++q) gb[k][q] = L[(9 * k + q) * plane + oo];
        Mb[k] = L[(27 + k) * plane + oo];
      }
      // g' = (1 - 1/tau) f + e/tau + w dt F,  M' = A + dt F,  e = w A (1 + Q(u))
      double ubz = 0.0, ubr = 0.0;
      for (int k = 0; k < 3; ++k) {
        double sw = 0.0, s0 = 0.0;
        for (int q = 0; q < 9; ++q) {
          const double w = WQ<double>(q);
          const double cu = XZ(q) * uz + XR(q) * ur;
          const double Q = 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur);
          const double eb = gb[k][q] / p.tau;
          sw += w * gb[k][q];
          s0 += eb * w * (1.0 + Q);
          const double s = eb * w * Am[k];
          ubz += s * (3.0 * XZ(q) + 9.0 * cu * XZ(q) - 3.0 * uz);
          ubr += s * (3.0 * XR(q) + 9.0 * cu * XR(q) - 3.0 * ur);
        }
        Fb[k] = dt * (sw + Mb[k]);
        Ab[k] = Mb[k] + s0;
      }
      double bbz = p.lam * ubz, bbr = p.lam * ubr;
      double Ebz_b = 0.0, Ebr_b = 0.0, Bb_b = 0.0;
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
        for (int k = 0; k < 3; ++k) {
          bbr += Fb[k] * (-Am[k] * ir);
          Ab[k] += Fb[k] * (-br * ir);
        }
      }
      if (live) {
        const double g2 = 1.0 + pz * pz + pr * pr, ig3 = ig / g2;
        const double pdot = pz * bbz + pr * bbr;
        const double pbz = bbz * ig - pz * pdot * ig3, pbr = bbr * ig - pr * pdot * ig3;
        Ab[1] += pbz / n;
        Ab[2] += pbr / n;
        Ab[0] -= (pbz * pz + pbr * pr) / n;
      }
      for (int k = 0; k < 3; ++k) {
        W[(W_A + k) * plane + cell] = Ab[k];
        W[(W_F + k) * plane + cell] = Fb[k];
      }
      W[W_EZ * plane + cell] = Ebz_b;
      W[W_ER * plane + cell] = Ebr_b;
      W[W_B * plane + cell] = Bb_b;

      if (p.window && i == nz - 1) {
        // window front ghost: the populations pulled from column nz (xi_z = -1) are w_q n_bg(z_nz)
        double dl, dn;
        dnbg(p, (double)(a.s + nz) * h, dl, dn);
        double sum = 0.0;
        for (int q = 0; q < 9; ++q)
          if (XZ(q) == -1) sum += WQ<double>(q) * ((1.0 - 1.0 / p.tau) * gb[0][q] + Ab[0]);
        part[0] += sum * dl;
        part[1] += sum * dn;
        if (a.shift) {
          // the new front column of x^{k+1} (output index nz - 1): w_q n_bg and n_bg
          const int of = j * pitch + (nz - 1);
          double s2 = L[27 * plane + of];
          for (int q = 0; q < 9; ++q) s2 += WQ<double>(q) * L[q * plane + of];
          part[0] += s2 * dl;
          part[1] += s2 * dn;
        }
      }
    }
  }
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// ------------------------------------------------------------------------------------------
// adj_field_kernel: one thread per cell (i, j) of x^k.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_field_kernel(AdjArgs a) {
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int gx = (nz + TZ - 1) / TZ, gy = (nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int i0 = (tile % gx) * TZ, j0 = (tile / gx) * TR;
  const int tid = threadIdx.x, tx = tid % TZ, ty = tid / TZ;
  const double h = p.h, dt = p.dt;
  const double* W = a.work;
  const double* L = a.lam_next;
  // site adjoints (zero outside the domain; the dropped column already holds zeros)
  auto site = [&](int plane_id, int i, int j) -> double {
    if (j < 0 || j >= nr) return 0.0;
    if (p.per_z) i = wrapi(i, nz);
    else if (i < 0 || i >= nz) return 0.0;
    return W[plane_id * plane + j * pitch + i];
  };
  // adjoint of E^k / B^{k+1/2} as state of x^{k+1} (zero for the column dropped by the shift)
  auto next = [&](int c, int i, int j) -> double {
    if (p.per_z) i = wrapi(i, nz);
    const int o = i - a.shift;
    if (o < 0 || i >= nz || j < 0 || j >= nr) return 0.0;
    return L[c * plane + j * pitch + o];
  };
  // 1/8 of the B_bar of the sites that average the corner (i, j) (with the rear copy rule)
  auto bsum = [&](int i, int j) -> double {
    double s = site(W_B, i, j) + site(W_B, i + 1, j) + site(W_B, i, j + 1) + site(W_B, i + 1, j + 1);
    if (!p.per_z && i == 0) s += site(W_B, 0, j) + site(W_B, 0, j + 1);
    return s / 8.0;
  };
  auto LBp = [&](int i, int j) -> double {   // adjoint of B^{k+1/2}(i, j)
    if (j < 0 || j >= nr) return 0.0;
    if (p.per_z) i = wrapi(i, nz);
    else if (i < 0 || i >= nz) return 0.0;
    return next(32, i, j) + bsum(i, j);
  };
  auto LEz = [&](int i, int j) -> double {   // adjoint of E_z^k(i, j)
    if (j < 0 || j >= nr) return 0.0;
    if (p.per_z) i = wrapi(i, nz);
    else if (i < 0 || i >= nz) return 0.0;
    double v = next(30, i, j) + 0.5 * (site(W_EZ, i, j) + site(W_EZ, i + 1, j));
    if (!p.per_z && i == 0) v += 0.5 * site(W_EZ, 0, j);   // rear copy E_z(-1) = E_z(0)
    if (p.fields_on) {
      if (j <= nr - 2) v -= dt / h * LBp(i, j);
      if (j >= 1) v += dt / h * LBp(i, j - 1);
    }
    return v;
  };
  auto LEr = [&](int i, int j) -> double {   // adjoint of E_r^k(i, j)
    if (j < 0 || j >= nr) return 0.0;
    if (p.per_z) i = wrapi(i, nz);
    else if (i < 0 || i >= nz) return 0.0;
    double v = next(31, i, j) + 0.5 * (site(W_ER, i, j) + (j + 1 < nr ? site(W_ER, i, j + 1) : 0.0));
    if (p.fields_on) {
      if (p.per_z || i <= nz - 2) v += dt / h * LBp(i, j);
      if (p.per_z || i >= 1) v -= dt / h * LBp(i - 1, j);
    }
    return v;
  };

  const int i = i0 + tx, j = j0 + ty;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < nz && j < nr) {
    const int cell = j * pitch + i;
    double* Lo = a.lam;
    double* Wo = a.work;
    if (p.fields_on) {
      const double lez = LEz(i, j), ler = LEr(i, j);
      double lb = LBp(i, j) + bsum(i, j);
      const double rj = (j + 0.5) * h;
      lb += dt * (j + 1.0) / rj * lez;
      if (j + 1 < nr) lb -= dt * (j + 1.0) / ((j + 1.5) * h) * LEz(i, j + 1);
      if (p.per_z || i >= 1) lb -= dt / h * ler;
      if (p.per_z || i + 1 < nz) lb += dt / h * LEr(i + 1, j);
      Lo[30 * plane + cell] = lez;
      Lo[31 * plane + cell] = ler;
      Lo[32 * plane + cell] = lb;
      double jz = 0.5 * dt * (lez + ((p.per_z || i >= 1) ? LEz(i - 1, j) : 0.0));
      if (!p.per_z && !p.window && i == nz - 1) jz += 0.5 * dt * lez;   // front copy of J_z
      double jr = 0.5 * dt * (ler + (j >= 1 ? LEr(i, j - 1) : 0.0));
      if (j == nr - 1) jr += 0.5 * dt * ler;                             // outer copy of J_r
      Wo[W_JZ * plane + cell] = jz;
      Wo[W_JR * plane + cell] = jr;
      // driver current J_b(z_i + dz/2, r_j, t_{k-1/2})
      const int ci = p.per_z ? wrapi(i, nz) : i;
      double dsr, dnb;
      ddriver(p, ((double)(a.s + ci) + 0.5) * h, rj, ((double)a.k - 0.5) * dt, dsr, dnb);
      part[2] += dt * lez * dsr;
      part[3] += dt * lez * dnb;
    } else {
      // fields are carried unchanged and unused
      Lo[30 * plane + cell] = next(30, i, j);
      Lo[31 * plane + cell] = next(31, i, j);
      Lo[32 * plane + cell] = next(32, i, j);
      Wo[W_JZ * plane + cell] = 0.0;
      Wo[W_JR * plane + cell] = 0.0;
    }
  }
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// ------------------------------------------------------------------------------------------
// adj_pop_kernel: one thread per cell (i, j) of x^k.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_pop_kernel(AdjArgs a) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int gx = (nz + TZ - 1) / TZ, gy = (nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int i0 = (tile % gx) * TZ, j0 = (tile / gx) * TR;
  const int i = i0 + threadIdx.x % TZ, j = j0 + threadIdx.x / TZ;
  if (i >= nz || j >= nr) return;
  const double h = p.h;
  const double* W = a.work;
  const double* L = a.lam_next;
  const A* Min = (const A*)a.M;
  const int cell = j * pitch + i;
  const double c1 = 1.0 - 1.0 / p.tau;
  // a computed site y of step k (inside the domain after periodic wrap, not the dropped column)
  auto computed = [&](int& yi, int& yj) -> bool {
    if (p.per_z) yi = wrapi(yi, nz);
    if (p.per_r) yj = wrapi(yj, nr);
    if (yi < 0 || yi >= nz || yj < 0 || yj >= nr) return false;
    return !(a.shift && yi == 0);
  };
  // adjoint of the pulled population f_{k,q} at site y: (1 - 1/tau) g'_bar + A_bar
  auto lamf = [&](int k, int q, int yi, int yj) -> double {
    const int ys = yj * pitch + yi;
    return c1 * L[(9 * k + q) * plane + yj * pitch + (yi - a.shift)] + W[(W_A + k) * plane + ys];
  };

  // transpose of the pull: g_q(x) streams to y = x + xi_q
  double* Lo = a.lam;
  for (int k = 0; k < 3; ++k)
    for (int q = 0; q < 9; ++q) {
      int yi = i + XZ(q), yj = j + XR(q);
      Lo[(9 * k + q) * plane + cell] = computed(yi, yj) ? lamf(k, q, yi, yj) : 0.0;
    }

  // moments: raw values of x^k at this cell
  const double M[3] = {(double)Min[cell] + nbg(p, (double)(a.s + i) * h), (double)Min[plane + cell],
                       (double)Min[2 * plane + cell]};
  double Mb[3] = {0.0, 0.0, 0.0};
  // (a) face currents of Ampere's law
  if (p.fields_on) current_vjp(p, M, W[W_JZ * plane + cell], W[W_JR * plane + cell], Mb);
  // (b) lagged radial gradient of the axisymmetric source, D (M(j+1) - M(j-1)) / (2 dr r_j)
  if (p.cyl_on) {
    const double c = p.D / (2.0 * h);
    const double par[3] = {1.0, 1.0, -1.0};
    for (int k = 0; k < 3; ++k) {
      double v = 0.0;
      if (j >= 1) v += c / ((j - 0.5) * h) * W[(W_F + k) * plane + cell - pitch];
      if (j + 1 < nr) v -= c / ((j + 1.5) * h) * W[(W_F + k) * plane + cell + pitch];
      if (j == 0) v -= par[k] * c / (0.5 * h) * W[(W_F + k) * plane + cell];
      if (j == nr - 1) v += c / ((j + 0.5) * h) * W[(W_F + k) * plane + cell];
      Mb[k] += v;
    }
  }
  // (c) equilibrium ghosts whose moments are copies (or the axis mirror) of this cell: replay the
  // forward's ghost test for every site within two cells that may pull such a ghost (periodic
  // dimensions hold at least 5 cells, so the wrapped sites are distinct)
  const bool edge = (!p.per_z && (i <= 1 || i >= nz - 2)) || (!p.per_r && (j <= 1 || j >= nr - 2));
  if (edge) {
    const double Mx[3] = {M[0], M[1], M[2]};
    for (int dyi = -2; dyi <= 2; ++dyi)
      for (int dyj = -2; dyj <= 2; ++dyj) {
        int yi = i + dyi, yj = j + dyj;
        if (p.per_z) yi = wrapi(yi, nz);
        else if (yi < 0 || yi >= nz) continue;
        if (p.per_r) yj = wrapi(yj, nr);
        else if (yj < 0 || yj >= nr) continue;
        if (a.shift && yi == 0) continue;   // not a computed site
        for (int q = 0; q < 9; ++q) {
          const int si = yi - XZ(q), sj = yj - XR(q);
          const bool oz = si < 0 || si >= nz, orr = sj < 0 || sj >= nr;
          if (!((oz && !p.per_z) || (orr && !p.per_r))) continue;   // a regular pull
          int ci, rj;
          double sgn = 1.0;
          if (p.per_z) ci = wrapi(si, nz);
          else if (si < 0) ci = 0;
          else if (si >= nz) {
            if (p.window) continue;   // plasma at rest: depends on theta only
            ci = nz - 1;
          } else ci = si;
          if (p.per_r) rj = wrapi(sj, nr);
          else if (sj < 0) { rj = 0; sgn = -1.0; }
          else if (sj >= nr) rj = nr - 1;
          else rj = sj;
          if (ci != i || rj != j) continue;
          const double Mg[3] = {Mx[0], Mx[1], sgn * Mx[2]};
          double Mgb[3] = {0.0, 0.0, 0.0};
          const double af[3] = {lamf(0, q, yi, yj), lamf(1, q, yi, yj), lamf(2, q, yi, yj)};
          feq_vjp(p, q, Mg, af, Mgb);
          Mb[0] += Mgb[0];
          Mb[1] += Mgb[1];
          Mb[2] += sgn * Mgb[2];
        }
      }
  }
  Lo[27 * plane + cell] = Mb[0];
  Lo[28 * plane + cell] = Mb[1];
  Lo[29 * plane + cell] = Mb[2];
}

// ------------------------------------------------------------------------------------------
// adj_init_kernel: theta partials of the initial state, one thread per column.
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(NTHREADS) void adj_init_kernel(AdjArgs a) {
  using A = typename Mode<ST, false>::A;
  const Physics& p = a.p;
  const int i = blockIdx.x * NTHREADS + threadIdx.x;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < p.nz) {
    const long long plane = p.plane;
    const double h = p.h, dt = p.dt;
    const double* L = a.lam_next;   // lambda^0
    const A* Min = (const A*)a.M;
    const double z = (double)i * h;
    const double nb0 = nbg(p, z);
    double dl, dn;
    dnbg(p, z, dl, dn);
    double cer[2] = {0.0, 0.0}, cb[2] = {0.0, 0.0};   // cumulative d/d(sigma_r), d/d(n_b)
    for (int j = 0; j < p.nr; ++j) {
      const int cell = j * p.pitch + i;
      // populations and moments: f_eq of n_init = n_bg (1 + delta) at the initial momentum
      const double n = (double)Min[cell] + nb0;
      const double m1 = Min[plane + cell], m2 = Min[2 * plane + cell];
      double bz, br;
      const bool live = velocity<double>(n, m1, m2, p.n_floor, bz, br);
      const double pz = live ? m1 / n : 0.0, pr = live ? m2 / n : 0.0;
      const double uz = p.lam * bz, ur = p.lam * br;
      double nbar = L[27 * plane + cell] + pz * L[28 * plane + cell] + pr * L[29 * plane + cell];
      for (int q = 0; q < 9; ++q) {
        const double cu = XZ(q) * uz + XR(q) * ur;
        const double e = WQ<double>(q) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur));
        nbar += e * (L[q * plane + cell] + pz * L[(9 + q) * plane + cell] + pr * L[(18 + q) * plane + cell]);
      }
      if (nb0 > 0.0) {
        const double ratio = n / nb0;   // 1 + delta
        part[0] += nbar * ratio * dl;
        part[1] += nbar * ratio * dn;
      }
      if (p.fields_on) {
        // E_r^{-1}(j) = -h / (j+1) sum_{j' <= j} (j' + 1/2) n_b(z_i, r_j', -dt); B^{-1/2} likewise
        const double r = (j + 0.5) * h;
        double dsr, dnb;
        ddriver(p, z, r, -dt, dsr, dnb);
        cer[0] += (j + 0.5) * dsr;
        cer[1] += (j + 0.5) * dnb;
        ddriver(p, z + 0.5 * h, r, -0.5 * dt, dsr, dnb);
        cb[0] += (j + 0.5) * dsr;
        cb[1] += (j + 0.5) * dnb;
        const double f = -h / (j + 1.0);
        part[2] += f * (L[31 * plane + cell] * cer[0] + L[32 * plane + cell] * cb[0]);
        part[3] += f * (L[31 * plane + cell] * cer[1] + L[32 * plane + cell] * cb[1]);
      }
    }
  }
  block_sum4(part, a.partials + (long long)blockIdx.x * 4);
}

// sum of per-block partials (fixed order) added into acc[4]
__global__ __launch_bounds__(NTHREADS) void partials_sum_kernel(const double* partials, int nblocks,
                                                                double* acc) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += NTHREADS)
    for (int c = 0; c < 4; ++c) v[c] += partials[(long long)b * 4 + c];
  __shared__ double res[4];
  block_sum4(v, res);
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < 4; ++c) acc[c] += res[c];
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static int step_blocks(const Physics& p) {
  return ((p.nz + TZ - 1) / TZ) * ((p.nr + TR - 1) / TR);
}

int adjoint_partial_blocks(const Physics& p) {
  const int a = step_blocks(p), b = (p.nz + NTHREADS - 1) / NTHREADS;
  return a > b ? a : b;
}

#define ADJ_DISPATCH(storage, KERNEL, GRID, STREAM, ARGS)                            \
  do {                                                                               \
    if ((storage) == 0) KERNEL<0><<<(GRID), NTHREADS, 0, (STREAM)>>>(ARGS);          \
    else if ((storage) == 1) KERNEL<1><<<(GRID), NTHREADS, 0, (STREAM)>>>(ARGS);     \
    else KERNEL<2><<<(GRID), NTHREADS, 0, (STREAM)>>>(ARGS);                         \
  } while (0)

hipError_t launch_adjoint_step(int storage, const AdjArgs& a, double* grad_acc, hipStream_t st) {
  const int nb = step_blocks(a.p);
  ADJ_DISPATCH(storage, adj_site_kernel, dim3(nb), st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  partials_sum_kernel<<<1, NTHREADS, 0, st>>>(a.partials, nb, grad_acc);
  ADJ_DISPATCH(storage, adj_field_kernel, dim3(nb), st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  partials_sum_kernel<<<1, NTHREADS, 0, st>>>(a.partials, nb, grad_acc);
  ADJ_DISPATCH(storage, adj_pop_kernel, dim3(nb), st, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_init(int storage, const AdjArgs& a, double* grad_acc, hipStream_t st) {
  const int nb = (a.p.nz + NTHREADS - 1) / NTHREADS;
  ADJ_DISPATCH(storage, adj_init_kernel, dim3(nb), st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  partials_sum_kernel<<<1, NTHREADS, 0, st>>>(a.partials, nb, grad_acc);
  return hipGetLastError();
}

}  // namespace lbm
