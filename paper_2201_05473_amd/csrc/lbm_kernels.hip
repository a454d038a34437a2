// HIP kernels (gfx950) of the lattice-Boltzmann plasma-wakefield step.
//
// One launch per time step: the fused kernel first advances the Yee fields of its tile (plus a
// one-cell halo, recomputed from LDS) and then performs the pull-stream / collision (BGK, TRT,
// regularised or MRT) of the three D2Q9 lattices of its sites.  Notation and step order follow the paper (Parise et al.,
// arXiv:2201.05473): Eq. (5) for the fields, Eqs. (6)-(10), (13), (14) for the lattices; the
// readings where the paper is silent are stated at each use.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------------------------------------
// The fused step kernel.
//
// Memory schedule: every thread first issues its share of the halo loads (moments, B^{k-1/2},
// E^{k-1}) and then its 27 population loads, all from clamped in-range addresses so that every
// thread issues the same number of loads.  Vector-memory counters retire in order, so the field
// phase can wait for the halo loads alone while the population loads stay in flight across the
// LDS barriers (which only wait for LDS traffic).
// ------------------------------------------------------------------------------------------
// PER = false: the grid is known not to be periodic, and the wrap code is compiled out.
// DRV = 1: the driver current J_b comes from the particle bunch's deposit (a.jb_in, z and r
// components) in place of the rigid driver's closed form.
// SITE = true: the adjoint's forward recompute; the step also writes its site record (the
// site-averaged fields and the moments of the pulled populations, a.site_out).
// FP32 storage keeps E_r and B_theta compensated: an FP32 value plus a bfloat16 residual in a
// fourth field plane, updated with a two-sum (lbm_device.h, "Compensated fields").
// Occupancy.  With FP32 arithmetic the halo goes straight to LDS, so a thread holds little more
// than its 27 populations: FP32 storage fits 64 VGPRs without spills (8 waves per SIMD), except
// MRT, whose moment transform needs more (6 blocks).  FP16 storage keeps its bound of 7 blocks
// (FP16N with MRT spills a few registers under it and still runs faster than at 6).  FP64
// arithmetic needs about twice the registers and takes the compiler's choice.
template <int ST, bool FIELDS, bool M64, bool SITE, int COLL, bool PER, int DRV>
__global__ __launch_bounds__(NTHREADS, (ST == 0 || M64) ? 1 : (ST >= 2 ? 7 : (COLL == 3 ? 6 : 8))) void step_kernel(StepArgs a) {
  using S = typename Mode<ST, M64>::S;
  using C = typename Mode<ST, M64>::C;
  using A = typename Mode<ST, M64>::A;
  using CF = typename Mode<ST, M64>::CF;
  // sums of the eight moving equilibria: compensated for FP32 storage with FP32 arithmetic; plain
  // in FP64, and for FP16 storage, whose error is set by its storage and whose step is
  // instruction-bound
  using SE = EqSum<C, ST == 1 && !M64>;
  constexpr bool NEQ = neq_storage(ST);   // populations stored off their site's equilibrium
  const Physics& p = a.p;
  constexpr int MZ = TZ + 2, MR = TR + 2;    // moments:  cols i0-1..i0+TZ,   rows j0-1..j0+TR
  constexpr int BZ = TZ + 3, BR = TR + 3;    // B^{k-1/2}: cols i0-2..i0+TZ,  rows j0-2..j0+TR
  constexpr int EZZ = TZ + 1, EZR = TR + 2;  // E_z:      cols i0-1..i0+TZ-1, rows j0-1..j0+TR
  constexpr int ERZ = TZ + 2, ERR = TR + 1;  // E_r:      cols i0-1..i0+TZ,   rows j0-1..j0+TR-1
  constexpr int BNZ = TZ + 1, BNR = TR + 1;  // B^{k+1/2}: cols i0-1..i0+TZ-1, rows j0-1..j0+TR-1
  constexpr int NM = MR * MZ, NB = BR * BZ, NEZ = EZR * EZZ, NER = ERR * ERZ;
  constexpr int SM = (NM + NTHREADS - 1) / NTHREADS, SB = (NB + NTHREADS - 1) / NTHREADS;
  constexpr int SEZ = (NEZ + NTHREADS - 1) / NTHREADS, SER = (NER + NTHREADS - 1) / NTHREADS;
  // Halo tiles in LDS, row-major, each padded to a whole number of block-wide passes: element t of
  // a tile is the t-th load of the tile's flattened halo, so the 64 loads of a wavefront fill 64
  // consecutive words.  With FP32 auxiliary planes and FP32 field arithmetic the halo loads go
  // straight from memory to LDS (no registers held while the population loads are in flight);
  // otherwise they pass through registers (conversion to FP64).
  constexpr bool HDMA = std::is_same<A, float>::value && std::is_same<CF, float>::value;
  // FP32 storage: compensated E_r and B_theta (their bfloat16 residuals in a fourth field plane).
  // With FP32 field arithmetic the residual words are a fifth LDS tile over B's halo (E_r's
  // residual of the cell whose B is at a slot shares its word) and the updates accumulate with
  // acc_comp; with FP64 field arithmetic the residuals are folded into the FP64 tiles at load and
  // split off again at the store.
  constexpr bool XLO = fields_lo(ST) && FIELDS;
  constexpr bool COMP = XLO && HDMA;
  __shared__ CF sMst[3][SM * NTHREADS];
  __shared__ CF sBost[SB * NTHREADS];
  __shared__ CF sEzst[SEZ * NTHREADS];
  __shared__ CF sErst[SER * NTHREADS];
  __shared__ uint32_t sXst[COMP ? SB * NTHREADS : 1];
  CF(*const sM[3])[MZ] = {reinterpret_cast<CF(*)[MZ]>(sMst[0]), reinterpret_cast<CF(*)[MZ]>(sMst[1]),
                          reinterpret_cast<CF(*)[MZ]>(sMst[2])};
  CF(*const sBo)[BZ] = reinterpret_cast<CF(*)[BZ]>(sBost);
  CF(*const sEz)[EZZ] = reinterpret_cast<CF(*)[EZZ]>(sEzst);
  CF(*const sEr)[ERZ] = reinterpret_cast<CF(*)[ERZ]>(sErst);
  // residual words: slot (b, a) of the B tile; E_r slot (b, a) is word (b + 1, a + 1).  Halves are
  // written with 16-bit stores (little endian: E_r's residual at the even halfword)
  uint32_t(*const sX)[BZ] = reinterpret_cast<uint32_t(*)[BZ]>(sXst);
  uint16_t* const sX16 = reinterpret_cast<uint16_t*>(sXst);
  auto xer16 = [&](int b, int a) -> uint16_t& { return sX16[2 * (b * BZ + a)]; };
  auto xb16 = [&](int b, int a) -> uint16_t& { return sX16[2 * (b * BZ + a) + 1]; };
  __shared__ CF sJ[2][MR][MZ];
  __shared__ CF sBn[BNR][BNZ];
  __shared__ double sN[MZ];
  __shared__ CF sDz[EZZ];   // exp(-(z - z_d)^2 / 2 sigma_z^2) at the E_z columns
  __shared__ CF sDr[EZR];   // n_b exp(-r^2 / 2 sigma_r^2) at the fluid / E_z rows
  __shared__ CF sIr[EZR];   // 1 / r_j at the fluid / E_z rows
  __shared__ CF sJbzst[DRV ? SEZ * NTHREADS : 1];   // particle driver: J_bz at the E_z points
  __shared__ CF sJbrst[DRV ? SER * NTHREADS : 1];   // and J_br at the E_r points
  CF(*const sJbz)[EZZ] = reinterpret_cast<CF(*)[EZZ]>(sJbzst);
  CF(*const sJbr)[ERZ] = reinterpret_cast<CF(*)[ERZ]>(sJbrst);
  __shared__ CF sU[NEQ ? 2 : 1][NEQ ? MR : 1][NEQ ? MZ : 1];   // NEQ: lattice velocity u* of the moments

  const int nz = p.nz, nr = p.nr, pitch = p.pitch;
  const long long plane = p.plane;
  const int gx = (nz + TZ - 1) / TZ, gy = (nr + TR - 1) / TR;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int o0 = (tile % gx) * TZ;
  const int i0 = o0 + a.shift;  // logical (pre-shift) column of the first site
  const int j0 = (tile / gx) * TR;
  const int tid = threadIdx.x;
  const int tx = tid % TZ, ty = tid / TZ;
  // particle driver: J_b is zero outside the bunch's bound, so a tile (halo included) that misses it
  // neither reads J_b nor clears the next step's buffer (uniform)
  const bool jb_on = DRV && i0 + TZ + 1 >= a.jb_c0 && i0 - 2 <= a.jb_c1 && j0 - 2 <= a.jb_r1;
  const double h = p.h, dt = p.dt;
  const C hc = (C)h, dtc = (C)dt;
  const CF hf = (CF)h, dtf = (CF)dt;
  const A* Min = (const A*)a.M_in;
  const A* Ein = (const A*)a.E_in;
  const S* gin = (const S*)a.g_in;

  // Column of a logical position after the z rule for copies (rear copy, front copy, wrap) and
  // row after the r rule (axis mirror row 0, outer copy, wrap); always in range.
  auto zcol = [&](int i) { return PER && p.per_z ? wrapi(i, nz) : (i < 0 ? 0 : (i < nz ? i : nz - 1)); };
  auto rrow = [&](int j) { return PER && p.per_r ? wrapi(j, nr) : (j < 0 ? 0 : (j < nr ? j : nr - 1)); };
  // one buffer resource per plane (uniform) + 32-bit in-plane offsets (a plane holds fewer than
  // 2^31 elements and fewer than 2^32 bytes)
  const Rsrc M0p = plane_rsrc<A>(Min, plane, 0);
  const Rsrc M1p = plane_rsrc<A>(Min, plane, 1);
  const Rsrc M2p = plane_rsrc<A>(Min, plane, 2);
  const Rsrc Ezp = plane_rsrc<A>(Ein, plane, 0);
  const Rsrc Erp = plane_rsrc<A>(Ein, plane, 1);
  const Rsrc Bp = plane_rsrc<A>(Ein, plane, 2);
  const Rsrc Xp = plane_rsrc<uint32_t>(Ein, plane, 3);   // residual words (fields_lo storage)

  // --- 1. halo loads: into LDS (HDMA), or into registers ------------------------------------
  // Every lane loads from a clamped, in-range address; with HDMA a wave's 64 words land at its
  // 64 consecutive slots of the padded tile (slots past the tile are padding).
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);   // wavefront of the block (uniform)
  auto hload = [&](Rsrc r, uint32_t off, CF* tile, int s, A& reg) {
    if constexpr (HDMA)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)(tile + s * NTHREADS + wv * 64),
                                               4, (int)(off * 4u), 0, 0, 0);
    else
      reg = bload<A>(r, off);
  };
  A hm[HDMA ? 1 : SM][3];
  A hb[HDMA ? 1 : SB], hez[HDMA ? 1 : SEZ], her[HDMA ? 1 : SER];
  uint32_t hxb[XLO && !HDMA ? SB : 1], hxr[XLO && !HDMA ? SER : 1];
  A hjz[DRV && !HDMA ? SEZ : 1], hjr[DRV && !HDMA ? SER : 1];
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int t = min(tid + s * NTHREADS, NM - 1);
    const uint32_t off = rrow(j0 - 1 + t / MZ) * pitch + zcol(i0 - 1 + t % MZ);
    hload(M0p, off, sMst[0], s, hm[HDMA ? 0 : s][0]);
    hload(M1p, off, sMst[1], s, hm[HDMA ? 0 : s][1]);
    hload(M2p, off, sMst[2], s, hm[HDMA ? 0 : s][2]);
  }
  if (FIELDS) {
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int t = min(tid + s * NTHREADS, NB - 1);
      const uint32_t off = rrow(j0 - 2 + t / BZ) * pitch + zcol(i0 - 2 + t % BZ);
      hload(Bp, off, sBost, s, hb[HDMA ? 0 : s]);
      if constexpr (COMP)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            Xp, (__attribute__((address_space(3))) void*)(sXst + s * NTHREADS + wv * 64), 4, (int)(off * 4u), 0, 0, 0);
      else if constexpr (XLO)
        hxb[s] = bload<uint32_t>(Xp, off);
    }
#pragma unroll
    for (int s = 0; s < SEZ; ++s) {
      const int t = min(tid + s * NTHREADS, NEZ - 1);
      const uint32_t off = rrow(j0 - 1 + t / EZZ) * pitch + zcol(i0 - 1 + t % EZZ);
      hload(Ezp, off, sEzst, s, hez[HDMA ? 0 : s]);
      if (jb_on) hload(plane_rsrc<A>(a.jb_in, plane, 0), off, sJbzst, s, hjz[HDMA ? 0 : s]);
    }
#pragma unroll
    for (int s = 0; s < SER; ++s) {
      const int t = min(tid + s * NTHREADS, NER - 1);
      const uint32_t off = rrow(j0 - 1 + t / ERZ) * pitch + zcol(i0 - 1 + t % ERZ);
      hload(Erp, off, sErst, s, her[HDMA ? 0 : s]);
      if constexpr (XLO && !HDMA) hxr[s] = bload<uint32_t>(Xp, off);
      if (jb_on) hload(plane_rsrc<A>(a.jb_in, plane, 1), off, sJbrst, s, hjr[HDMA ? 0 : s]);
    }
  }
  // the population loads below must be issued after every halo load (the wait before the first
  // barrier counts on it)
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");

  // --- 2. per-column and per-row factors of the tile.  With the halo in LDS they are computed
  // before the population loads are issued (the FP64 ramp profile needs many registers for a
  // moment, which the in-flight populations would otherwise have to give up); with the halo in
  // registers, after them. -------------------------------------------------------------------
  const double tb = ((double)a.k - 0.5) * dt;
  auto factors = [&]() {
    // background density at the lab position of the physical column
    for (int t = tid; t < MZ; t += NTHREADS) {
      const int ii = i0 - 1 + t;
      sN[t] = nbg(p, (double)(a.s + (PER && p.per_z ? wrapi(ii, nz) : ii)) * h);
    }
    // the driver density factorises into a column and a row factor
    if (FIELDS && !DRV) {
      for (int t = tid; t < EZZ; t += NTHREADS) {
        const int ii = i0 - 1 + t;
        const int ci = PER && p.per_z ? wrapi(ii, nz) : ii;
        const CF dz = (CF)(((double)(a.s + ci) + 0.5) * h - (p.zd0 + tb));
        sDz[t] = mexp(-(dz * dz) / (CF)(2.0 * p.sigma_z * p.sigma_z));
      }
    }
    for (int t = tid; t < EZR; t += NTHREADS) {
      const double r = (j0 - 1 + t + 0.5) * h;
      const CF rr = (CF)r;
      if (!DRV) sDr[t] = (CF)p.nb * mexp(-(rr * rr) / (CF)(2.0 * p.sigma_r * p.sigma_r));
      sIr[t] = CF(1) / rr;
    }
  };
  if constexpr (HDMA) factors();
  __builtin_amdgcn_sched_barrier(0);

  // --- 3. population loads (Eq. (6), pull form f_q(x) = g_q(x - xi_q)) ----------------------
  const int o = o0 + tx;       // output column (post-shift)
  const int i = i0 + tx;       // logical column (pre-shift)
  const int j = j0 + ty;
  const bool site_ok = o < nz && j < nr;
  const bool fresh_site = site_ok && a.shift && i == nz;
  const bool active = site_ok && !fresh_site;
  S r0[9], r1[9], r2[9];
  // FP32 and FP16: one resource per lattice (nine planes, under 4 GiB at the largest grid), the
  // plane selected by the instruction's scalar offset; FP64: one resource per plane
  constexpr bool GRP = sizeof(S) <= 4;
  const uint32_t pbytes = (uint32_t)(plane * (long long)sizeof(S));
  const Rsrc lat_in[3] = {brsrc((const S*)gin, GRP ? 9u * pbytes : 0u),
                          brsrc((const S*)gin + 9 * plane, GRP ? 9u * pbytes : 0u),
                          brsrc((const S*)gin + 18 * plane, GRP ? 9u * pbytes : 0u)};
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    // ghost sources are replaced below; their (in-range) load is discarded.  FP64 populations are
    // read non-temporally (measured: FP64 step 110 -> 96.5 us on 2048 x 512; FP32 loses 25 %)
    constexpr int POL = ST == 0 ? 2 : 0;
    const uint32_t off = rrow(j - XR(q)) * pitch + zcol(i - XZ(q));
    if constexpr (GRP) {
      r0[q] = bload_g<S, POL>(lat_in[0], off, (uint32_t)q * pbytes);
      r1[q] = bload_g<S, POL>(lat_in[1], off, (uint32_t)q * pbytes);
      r2[q] = bload_g<S, POL>(lat_in[2], off, (uint32_t)q * pbytes);
    } else {
      r0[q] = bload<S, POL>(plane_rsrc<S>(gin, plane, q), off);
      r1[q] = bload<S, POL>(plane_rsrc<S>(gin, plane, 9 + q), off);
      r2[q] = bload<S, POL>(plane_rsrc<S>(gin, plane, 18 + q), off);
    }
  }
  if constexpr (!HDMA) factors();

  if constexpr (HDMA) {
    // the halo's loads to LDS were issued before the 27 population loads, and vector-memory
    // counters retire in order: waiting until at most 27 are outstanding leaves the populations in
    // flight (gfx9 encoding: vmcnt 27, expcnt and lgkmcnt not waited for)
    static_assert(27 < 64, "vmcnt holds 6 bits");
    __builtin_amdgcn_s_waitcnt((1 << 14) | (0xF << 8) | (0x7 << 4) | (27 & 0xF));
  }
  __syncthreads();

  // --- 4. moments with the ghost ring (z rule, then r rule) and their current J = n beta ----
  // sM[0] holds the density moment as the deviation from n_bg of this LDS column; a ghost
  // copied from another column carries the difference of the two columns' n_bg.
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int t = tid + s * NTHREADS;
    if (t < NM) {
      const int bb = t / MZ, aa = t % MZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      const bool fresh = !p.per_z && p.window && ii == nz;   // window front: plasma at rest
      CF d0, m1, m2;
      if constexpr (HDMA) {
        d0 = sM[0][bb][aa];
        m1 = sM[1][bb][aa];
        m2 = sM[2][bb][aa];
      } else {
        d0 = (CF)hm[s][0];
        m1 = (CF)hm[s][1];
        m2 = (CF)hm[s][2];
      }
      if (fresh) {
        d0 = CF(0);
        m1 = CF(0);
        m2 = CF(0);
      } else if (!p.per_z && (ii < 0 || ii >= nz)) {
        // the copied column lies inside this LDS tile (the ghost borders it)
        d0 += (CF)(sN[zcol(ii) - (i0 - 1)] - sN[aa]);
      }
      if (!p.per_r && jj < 0) m2 = -m2;                     // axis mirror: n p_r is odd
      sM[0][bb][aa] = d0;
      sM[1][bb][aa] = m1;
      sM[2][bb][aa] = m2;
      if (FIELDS || NEQ) {
        const CF m0 = (CF)sN[aa] + d0;
        CF bz, br;
        velocity<CF>(m0, m1, m2, (CF)p.n_floor, bz, br);
        if (FIELDS) {
          sJ[0][bb][aa] = m0 * bz;
          sJ[1][bb][aa] = m0 * br;
        }
        if (NEQ) {
          sU[0][bb][aa] = (CF)p.lam * bz;
          sU[1][bb][aa] = (CF)p.lam * br;
        }
      }
    }
  }

  if (FIELDS) {
    // --- 5. B^{k-1/2}, E^{k-1} into LDS (ghosts: B = 0 on the axis, zero-gradient elsewhere) --
    if constexpr (HDMA) {
      // the tiles are in LDS already; only B's rows below the axis are replaced (by zero)
      if (j0 == 0) {
#pragma unroll
        for (int s = 0; s < SB; ++s) {
          const int t = tid + s * NTHREADS;
          if (t < 2 * BZ) {
            sBo[t / BZ][t % BZ] = CF(0);
            if constexpr (COMP) sX[t / BZ][t % BZ] = 0u;   // B's residual, and E_r's of row -1
          }
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int t = tid + s * NTHREADS;
        if (t < NB) {
          CF v = (CF)hb[s];
          if constexpr (XLO) v += (CF)lo_b(hxb[s]);
          sBo[t / BZ][t % BZ] = (j0 - 2 + t / BZ) < 0 ? CF(0) : v;
        }
      }
#pragma unroll
      for (int s = 0; s < SEZ; ++s) {
        const int t = tid + s * NTHREADS;
        if (t < NEZ) sEz[t / EZZ][t % EZZ] = (CF)hez[s];
        if (jb_on && t < NEZ) sJbz[t / EZZ][t % EZZ] = (CF)hjz[s];
      }
#pragma unroll
      for (int s = 0; s < SER; ++s) {
        const int t = tid + s * NTHREADS;
        if (t < NER) {
          CF v = (CF)her[s];
          if constexpr (XLO) v += (CF)lo_er(hxr[s]);
          sEr[t / ERZ][t % ERZ] = v;
        }
        if (jb_on && t < NER) sJbr[t / ERZ][t % ERZ] = (CF)hjr[s];
      }
    }
    __syncthreads();

    // --- 6. Ampere, Eq. (5): E^k = E^{k-1} + dt (curl B^{k-1/2} + J*_face + J_b(t_{k-1/2})) ----
    const CF ih = CF(1) / hf;
    for (int t = tid; t < NEZ; t += NTHREADS) {
      const int bb = t / EZZ, aa = t % EZZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr) {
        // (1/r) d(r B)/dr = ((j+1) B_j - j B_{j-1}) / r_j with r_j = (j + 1/2) dr, written as
        // (B_j + j (B_j - B_{j-1})) / r_j: same value, no large cancellation at large j in
        // reduced precision; the axis flux (j = 0) vanishes
        const CF bj = sBo[bb + 1][aa + 1];
        CF curl;
        if constexpr (COMP) {
          // B_theta's residuals enter the difference and the axis term
          const CF lj = lo_b(sX[bb + 1][aa + 1]), lm = lo_b(sX[bb][aa + 1]);
          const CF d = (bj - sBo[bb][aa + 1]) + (lj - lm);
          curl = (bj + (lj + (CF)jj * d)) * sIr[bb];
        } else {
          curl = (bj + (CF)jj * (bj - sBo[bb][aa + 1])) * sIr[bb];
        }
        const CF jf = CF(0.5) * (sJ[0][bb][aa] + sJ[0][bb][aa + 1]);
        const CF jb = DRV ? (jb_on ? sJbz[DRV ? bb : 0][DRV ? aa : 0] : CF(0)) : sDz[aa] * sDr[bb];
        sEz[bb][aa] = sEz[bb][aa] + dtf * (curl + jf + jb);
      }
    }
    for (int t = tid; t < NER; t += NTHREADS) {
      const int bb = t / ERZ, aa = t % ERZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr) {
        CF dB = sBo[bb + 1][aa + 1] - sBo[bb + 1][aa];
        if constexpr (COMP) dB += lo_b(sX[bb + 1][aa + 1]) - lo_b(sX[bb + 1][aa]);
        const CF curl = -dB * ih;   // -dB/dz
        const CF jf = CF(0.5) * (sJ[1][bb][aa] + sJ[1][bb + 1][aa]);
        const CF jbr = jb_on ? sJbr[DRV ? bb : 0][DRV ? aa : 0] : CF(0);
        if constexpr (COMP) {
          float hi = sEr[bb][aa], lo = lo_er(sX[bb + 1][aa + 1]);
          acc_comp(hi, lo, dtf * (curl + jf + jbr));
          sEr[bb][aa] = hi;
          xer16(bb + 1, aa + 1) = (uint16_t)bf16_rne(lo);
        } else {
          sEr[bb][aa] = sEr[bb][aa] + dtf * (curl + jf + jbr);
        }
      }
    }
    __syncthreads();
    // ghosts of E^k (zero-gradient fields, E_r = 0 on the axis), z rule first: rear E_z copy,
    // front E_r copy ...
    if (!p.per_z) {
      if (i0 == 0)
        for (int bb = tid; bb < EZR; bb += NTHREADS) sEz[bb][0] = sEz[bb][1];
      const int af = nz - (i0 - 1);   // LDS column of i = nz
      if (af >= 1 && af < ERZ)
        for (int bb = tid; bb < ERR; bb += NTHREADS) {
          sEr[bb][af] = sEr[bb][af - 1];
          if constexpr (COMP) xer16(bb + 1, af + 1) = xer16(bb + 1, af);
        }
    }
    __syncthreads();
    // ... then the r rule: outer E_z copy, E_r = 0 on the axis
    {
      const int bo = nr - (j0 - 1);   // LDS row of j = nr
      if (bo >= 1 && bo < EZR)
        for (int aa = tid; aa < EZZ; aa += NTHREADS) sEz[bo][aa] = sEz[bo - 1][aa];
    }
    if (j0 == 0)
      for (int aa = tid; aa < ERZ; aa += NTHREADS) sEr[0][aa] = CF(0);
    __syncthreads();

    // --- 7. Faraday, Eq. (5) with the standard sign: B^{k+1/2} = B^{k-1/2} + dt (dE_z/dr - dE_r/dz)
    for (int t = tid; t < BNR * BNZ; t += NTHREADS) {
      const int bb = t / BNZ, aa = t % BNZ;
      const int ii = i0 - 1 + aa, jj = j0 - 1 + bb;
      CF v = CF(0);
      float vlo = 0.f;
      if ((p.per_z || (ii >= 0 && ii < nz)) && jj >= 0 && jj < nr) {
        const CF dez = (sEz[bb + 1][aa] - sEz[bb][aa]) * ih;
        CF dEr = sEr[bb][aa + 1] - sEr[bb][aa];
        if constexpr (COMP) dEr += lo_er(sX[bb + 1][aa + 2]) - lo_er(sX[bb + 1][aa + 1]);
        const CF der = dEr * ih;
        if constexpr (COMP) {
          float hi = sBo[bb + 1][aa + 1];
          vlo = lo_b(sX[bb + 1][aa + 1]);
          acc_comp(hi, vlo, dtf * (dez - der));
          v = hi;
        } else {
          v = sBo[bb + 1][aa + 1] + dtf * (dez - der);
        }
      }
      sBn[bb][aa] = v;
      // B^{k+1/2}'s residual replaces B^{k-1/2}'s in the same word (read above by this thread only)
      if constexpr (COMP) xb16(bb + 1, aa + 1) = (uint16_t)bf16_rne(vlo);
    }
    __syncthreads();
    if (!p.per_z && i0 == 0)
      for (int bb = tid; bb < BNR; bb += NTHREADS) {   // rear copy
        sBn[bb][0] = sBn[bb][1];
        if constexpr (COMP) xb16(bb + 1, 1) = xb16(bb + 1, 2);
      }
    __syncthreads();
  } else {
    __syncthreads();
  }

  // --- 8. fluid phase: one site per thread ------------------------------------------------
  if (!site_ok) return;   // no barrier below this point
  const uint32_t oo = j * pitch + o;
  if (jb_on) {
    // the next step's deposit buffer, cleared at this output cell
    bstore<A>(plane_rsrc<A>(a.jb_zero, plane, 0), oo, C(0));
    bstore<A>(plane_rsrc<A>(a.jb_zero, plane, 1), oo, C(0));
  }
  const void* gout = a.g_out;
  const void* Mout = a.M_out;
  const void* Eout = a.E_out;

  if (fresh_site) {
    // new front column of the moved window: plasma at rest at n_bg, no fields
    for (int c = 0; c < 27; ++c) bstore<S>(plane_rsrc<S>(gout, plane, c), oo, C(0));
    for (int c = 0; c < 3; ++c) {
      bstore<A>(plane_rsrc<A>(Mout, plane, c), oo, C(0));
      bstore<A>(plane_rsrc<A>(Eout, plane, c), oo, C(0));
    }
    if constexpr (fields_lo(ST)) bstore<uint32_t>(plane_rsrc<uint32_t>(Eout, plane, 3), oo, 0u);
    return;
  }

  const double nref_d = sN[tx + 1];
  const C nref = (C)nref_d;

  // Ghost sources take f_eq of the ghost moments (Eq. (14): boundary populations at the
  // equilibrium of the boundary values).  Lattice 0 is carried as the deviation from
  // w_q n_bg(z_i).
  C f0[9], f1[9], f2[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int si = i - XZ(q), sj = j - XR(q);
    const bool oz = si < 0 || si >= nz, orr = sj < 0 || sj >= nr;
    const C w = WQ<C>(q);
    if ((oz && !p.per_z) || (orr && !p.per_r)) {
      const int ga = tx + 1 - XZ(q), gb = ty + 1 - XR(q);
      const C dg = (C)sM[0][gb][ga] + (C)(sN[ga] - nref_d);   // ghost density minus n_bg(z_i)
      const C m0 = nref + dg, m1 = (C)sM[1][gb][ga], m2 = (C)sM[2][gb][ga];
      C bz, br;
      velocity<C>(m0, m1, m2, (C)p.n_floor, bz, br);
      const C uz = (C)p.lam * bz, ur = (C)p.lam * br;
      const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
      const C Q = C(3) * cu + C(4.5) * cu * cu - C(1.5) * (uz * uz + ur * ur);
      f0[q] = w * (dg + m0 * Q);
      f1[q] = w * m1 * (C(1) + Q);
      f2[q] = w * m2 * (C(1) + Q);
    } else {
      const C dn = (C)(sN[tx + 1 - XZ(q)] - nref_d);
      f0[q] = ldv(r0[q]) + w * dn;
      f1[q] = ldv(r1[q]);
      f2[q] = ldv(r2[q]);
      if (NEQ) {
        // add back the equilibrium of the source site's stored moments (from the LDS halo)
        const int ga = tx + 1 - XZ(q), gb = ty + 1 - XR(q);
        const C d0s = (C)sM[0][gb][ga];
        C e0, e1, e2;
        eq_dir<C>(q, d0s, (C)sN[ga] + d0s, (C)sM[1][gb][ga], (C)sM[2][gb][ga], (C)sU[0][gb][ga],
                  (C)sU[1][gb][ga], e0, e1, e2);
        f0[q] += e0;
        f1[q] += e1;
        f2[q] += e2;
      }
    }
  }

  // Eq. (8): zeroth moments; the advecting velocity is beta_e from the n and n p lattices
  C dA0 = C(0), A1 = C(0), A2 = C(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    dA0 += f0[q];
    A1 += f1[q];
    A2 += f2[q];
  }
  const C A0 = nref + dA0;
  if (SITE) {
    // the pulled moments for the reverse sweep, which then needs none of the populations
    bstore<A>(plane_rsrc<A>(a.site_out, plane, 3), oo, A0);
    bstore<A>(plane_rsrc<A>(a.site_out, plane, 4), oo, A1);
    bstore<A>(plane_rsrc<A>(a.site_out, plane, 5), oo, A2);
  }
  C bz, br;
  const bool live = velocity<C>(A0, A1, A2, (C)p.n_floor, bz, br);
  const C uz = (C)p.lam * bz, ur = (C)p.lam * br;   // lattice velocity u* = beta c dt/dz
  const C usq = uz * uz + ur * ur;

  // fields at the site: E^k averaged, B^k = (B^{k-1/2} + B^{k+1/2}) / 2 averaged
  C Ebz = C(0), Ebr = C(0), Bb = C(0);
  if (FIELDS) {
    Ebz = (C)(CF(0.5) * (sEz[ty + 1][tx] + sEz[ty + 1][tx + 1]));
    Ebr = (C)(CF(0.5) * (sEr[ty][tx + 1] + sEr[ty + 1][tx + 1]));
    Bb = (C)((sBo[ty + 2][tx + 2] + sBo[ty + 2][tx + 1] + sBo[ty + 1][tx + 2] + sBo[ty + 1][tx + 1] +
              sBn[ty + 1][tx + 1] + sBn[ty + 1][tx] + sBn[ty][tx + 1] + sBn[ty][tx]) * CF(0.125));
    if (SITE) {
      bstore<A>(plane_rsrc<A>(a.site_out, plane, 0), oo, Ebz);
      bstore<A>(plane_rsrc<A>(a.site_out, plane, 1), oo, Ebr);
      bstore<A>(plane_rsrc<A>(a.site_out, plane, 2), oo, Bb);
    }
  }

  // Eq. (4): F = -n (E + beta x B), (beta x B)_z = beta_r B, (beta x B)_r = -beta_z B
  C F0 = C(0), F1 = C(0), F2 = C(0);
  if (live) {
    F1 = A0 * (-(Ebz + br * Bb));
    F2 = A0 * (-(Ebr - bz * Bb));
  }
  if (p.cyl_on) {
    // Eq. (13): -A u_r / r + D (dA/dr) / r, gradient of the previous step's moments
    const C ir = (C)sIr[ty + 1];
    const C Dc = (C)p.D * C(0.5) / hc;
    F0 += (-A0 * br + Dc * (C)(sM[0][ty + 2][tx + 1] - sM[0][ty][tx + 1])) * ir;
    F1 += (-A1 * br + Dc * (C)(sM[1][ty + 2][tx + 1] - sM[1][ty][tx + 1])) * ir;
    F2 += (-A2 * br + Dc * (C)(sM[2][ty + 2][tx + 1] - sM[2][ty][tx + 1])) * ir;
  }

  // Moments stored for the next step, A* = A + dt F (the zeroth moments of the populations
  // written below).  NEQ: as rounded to the auxiliary type, with their lattice velocity, so that
  // the equilibrium subtracted here is the one the next step adds back from the stored values.
  C mo0 = dA0 + dtc * F0, mo1 = A1 + dtc * F1, mo2 = A2 + dtc * F2;
  C uoz = C(0), uor = C(0);
  if (NEQ) {
    mo0 = (C)(A)mo0;
    mo1 = (C)(A)mo1;
    mo2 = (C)(A)mo2;
    C boz, bor;
    velocity<C>(nref + mo0, mo1, mo2, (C)p.n_floor, boz, bor);
    uoz = (C)p.lam * boz;
    uor = (C)p.lam * bor;
  }
  // population 9 k + q of the output site (NEQ: less the equilibrium of the stored moments)
  auto put = [&](int kq, C v) {
    if (NEQ) {
      C e0, e1, e2;
      eq_dir<C>(kq % 9, mo0, nref + mo0, mo1, mo2, uoz, uor, e0, e1, e2);
      v -= kq < 9 ? e0 : (kq < 18 ? e1 : e2);
    }
    if constexpr (sizeof(S) <= 4) {
      const uint32_t pb = (uint32_t)(plane * (long long)sizeof(S));
      bstore_g<S>(brsrc((const S*)gout + (kq / 9) * 9 * plane, 9u * pb), oo, (uint32_t)(kq % 9) * pb, v);
    } else {
      bstore<S>(plane_rsrc<S>(gout, plane, kq), oo, v);
    }
  };

  // Eqs. (7), (9), (10): relaxation toward the equilibrium (standard D2Q9 coefficients) plus
  // w_q dt F.  The equilibrium of direction q splits into a part even under xi -> -xi,
  // w (A (1 + 4.5 cu^2 - 1.5 u^2)), and an odd part, w A 3 cu (lattice 0 as the deviation).
  const C itau = (C)(1.0 / p.tau);
  if (COLL == 0) {
    // BGK, Eq. (7).  The rest population's equilibrium is taken as the moment minus the other
    // eight (equal to Eq. (9) in exact arithmetic; EqSum), so that the equilibrium's zeroth
    // moments are the moments themselves to about an ulp.  Otherwise the rounding of the
    // equilibria (and of the weights 1/9, 1/36 in FP32) would drift the density and momentum
    // moments over many steps.
    // g' = f (1 - 1/tau) + (f_eq / tau + w dt F): two FMAs per population
    SE se0, se1, se2;
    const C omt = C(1) - itau;
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const C w = WQ<C>(q);
      const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
      const C Q = C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
      const C e0 = w * (dA0 + A0 * Q);
      const C e1 = w * A1 * (C(1) + Q);
      const C e2 = w * A2 * (C(1) + Q);
      se0.add(e0);
      se1.add(e1);
      se2.add(e2);
      const C wdt = w * dtc;
      put(q, f0[q] * omt + (e0 * itau + wdt * F0));
      put(9 + q, f1[q] * omt + (e1 * itau + wdt * F1));
      put(18 + q, f2[q] * omt + (e2 * itau + wdt * F2));
    }
    const C wdt = WQ<C>(0) * dtc;
    put(0, f0[0] * omt + (se0.rest(dA0) * itau + wdt * F0));
    put(9, f1[0] * omt + (se1.rest(A1) * itau + wdt * F1));
    put(18, f2[0] * omt + (se2.rest(A2) * itau + wdt * F2));
  } else if (COLL == 1) {
    // two relaxation times: the even part of f - f_eq relaxes with 1/tau_plus, the odd part
    // (which carries the flux and so sets D) with 1/tau.  The rest population is even.
    const C itp = (C)(1.0 / p.tau_plus);
    SE se0, se1, se2;   // equilibria of the eight moving directions
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = t < 2 ? 1 + t : 5 + (t - 2);   // 1, 2, 5, 6
      const int b = t < 2 ? 3 + t : 7 + (t - 2);   // their opposites 3, 4, 7, 8
      const C w = WQ<C>(q), wdt = w * dtc;
      const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
      const C ev = C(4.5) * cu * cu - C(1.5) * usq;
      const C od = C(3) * cu;
      se0.add(C(2) * w * (dA0 + A0 * ev));
      se1.add(C(2) * w * A1 * (C(1) + ev));
      se2.add(C(2) * w * A2 * (C(1) + ev));
      {
        const C re = (C(0.5) * (f0[q] + f0[b]) - w * (dA0 + A0 * ev)) * itp;
        const C ro = (C(0.5) * (f0[q] - f0[b]) - w * A0 * od) * itau;
        put(q, f0[q] - re - ro + wdt * F0);
        put(b, f0[b] - re + ro + wdt * F0);
      }
      {
        const C re = (C(0.5) * (f1[q] + f1[b]) - w * A1 * (C(1) + ev)) * itp;
        const C ro = (C(0.5) * (f1[q] - f1[b]) - w * A1 * od) * itau;
        put(9 + q, f1[q] - re - ro + wdt * F1);
        put(9 + b, f1[b] - re + ro + wdt * F1);
      }
      {
        const C re = (C(0.5) * (f2[q] + f2[b]) - w * A2 * (C(1) + ev)) * itp;
        const C ro = (C(0.5) * (f2[q] - f2[b]) - w * A2 * od) * itau;
        put(18 + q, f2[q] - re - ro + wdt * F2);
        put(18 + b, f2[b] - re + ro + wdt * F2);
      }
    }
    // the rest population (even): its equilibrium is the moment minus the other eight, as for BGK
    const C wdt = WQ<C>(0) * dtc;
    put(0, f0[0] - (f0[0] - se0.rest(dA0)) * itp + wdt * F0);
    put(9, f1[0] - (f1[0] - se1.rest(A1)) * itp + wdt * F1);
    put(18, f2[0] - (f2[0] - se2.rest(A2)) * itp + wdt * F2);
  } else if (COLL == 3) {
    // multiple relaxation times: f - f_eq expanded in the orthogonal moments MB, each relaxed with
    // its rate (the fluxes with 1/tau, so D is that of BGK; the density moment of f - f_eq is
    // zero), then transformed back.  The equilibrium is BGK's, its rest population the moment
    // minus the other eight.
    const C rate[9] = {C(0), (C)p.mrt_se, (C)p.mrt_seps, itau, (C)p.mrt_sq, itau, (C)p.mrt_sq, (C)p.mrt_spi,
                       (C)p.mrt_spi};
    C Qq[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
      Qq[q] = C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
    }
    // lattice k: f its populations, mom its moment (for lattice 0 the deviation dA0, whose
    // equilibrium is w (dA0 + A0 Q)), F its source
    auto relax = [&](int k, const C (&f)[9], C mom, C F) {
      C e[9];
      SE sum;
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        e[q] = k == 0 ? WQ<C>(q) * (dA0 + A0 * Qq[q]) : WQ<C>(q) * mom * (C(1) + Qq[q]);
        sum.add(e[q]);
      }
      e[0] = sum.rest(mom);
      C c[9];
#pragma unroll
      for (int m = 1; m < 9; ++m) {
        C nm = C(0);
#pragma unroll
        for (int q = 0; q < 9; ++q)
          if (MB(m, q) != 0) nm += (C)MB(m, q) * (f[q] - e[q]);
        c[m] = rate[m] * nm / (C)MB_NORM2(m);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        C v = f[q];
#pragma unroll
        for (int m = 1; m < 9; ++m)
          if (MB(m, q) != 0) v -= (C)MB(m, q) * c[m];
        put(9 * k + q, v + WQ<C>(q) * dtc * F);
      }
    };
    relax(0, f0, dA0, F0);
    relax(1, f1, A1, F1);
    relax(2, f2, A2, F2);
  } else {
    // regularised: f - f_eq is replaced by its first-order Hermite projection
    // w xi . j_neq / c_s^2, j_neq = sum xi f - A u (the first moment of f_eq is A u), then
    // relaxed with 1/tau; every non-equilibrium moment above the first is dropped
    C jz0 = C(0), jr0 = C(0), jz1 = C(0), jr1 = C(0), jz2 = C(0), jr2 = C(0);
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (XZ(q) != 0) {
        jz0 += (C)XZ(q) * f0[q];
        jz1 += (C)XZ(q) * f1[q];
        jz2 += (C)XZ(q) * f2[q];
      }
      if (XR(q) != 0) {
        jr0 += (C)XR(q) * f0[q];
        jr1 += (C)XR(q) * f1[q];
        jr2 += (C)XR(q) * f2[q];
      }
    }
    const C k3 = C(3) * (C(1) - itau);
    jz0 = k3 * (jz0 - A0 * uz);
    jr0 = k3 * (jr0 - A0 * ur);
    jz1 = k3 * (jz1 - A1 * uz);
    jr1 = k3 * (jr1 - A1 * ur);
    jz2 = k3 * (jz2 - A2 * uz);
    jr2 = k3 * (jr2 - A2 * ur);
    SE se0, se1, se2;   // equilibria of the eight moving directions
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const C w = WQ<C>(q), wdt = w * dtc;
      const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
      const C Q = C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
      const C xz = (C)XZ(q), xr = (C)XR(q);
      const C e0 = w * (dA0 + A0 * Q), e1 = w * A1 * (C(1) + Q), e2 = w * A2 * (C(1) + Q);
      se0.add(e0);
      se1.add(e1);
      se2.add(e2);
      put(q, e0 + w * (xz * jz0 + xr * jr0) + wdt * F0);
      put(9 + q, e1 + w * (xz * jz1 + xr * jr1) + wdt * F1);
      put(18 + q, e2 + w * (xz * jz2 + xr * jr2) + wdt * F2);
    }
    // the rest population (no first-order part): the moment minus the other eight, as for BGK
    const C wdt = WQ<C>(0) * dtc;
    put(0, se0.rest(dA0) + wdt * F0);
    put(9, se1.rest(A1) + wdt * F1);
    put(18, se2.rest(A2) + wdt * F2);
  }
  bstore<A>(plane_rsrc<A>(Mout, plane, 0), oo, mo0);   // density moment stored as the deviation from n_bg
  bstore<A>(plane_rsrc<A>(Mout, plane, 1), oo, mo1);
  bstore<A>(plane_rsrc<A>(Mout, plane, 2), oo, mo2);

  if (FIELDS) {
    bstore<A>(plane_rsrc<A>(Eout, plane, 0), oo, (A)sEz[ty + 1][tx + 1]);
    bstore<A>(plane_rsrc<A>(Eout, plane, 1), oo, (A)sEr[ty + 1][tx + 1]);
    bstore<A>(plane_rsrc<A>(Eout, plane, 2), oo, (A)sBn[ty + 1][tx + 1]);
    if constexpr (COMP) {
      bstore<uint32_t>(plane_rsrc<uint32_t>(Eout, plane, 3), oo, sX[ty + 2][tx + 2]);
    } else if constexpr (XLO) {
      float eh, el, bh, bl;
      split_lo((double)sEr[ty + 1][tx + 1], eh, el);
      split_lo((double)sBn[ty + 1][tx + 1], bh, bl);
      bstore<uint32_t>(plane_rsrc<uint32_t>(Eout, plane, 3), oo, lo_pack(el, bl));
    }
  } else {
    const uint32_t io = j * pitch + i;
    for (int c = 0; c < 3; ++c) bstore<A>(plane_rsrc<A>(Eout, plane, c), oo, bload<A>(plane_rsrc<A>(Ein, plane, c), io));
    if constexpr (fields_lo(ST))
      bstore<uint32_t>(plane_rsrc<uint32_t>(Eout, plane, 3), oo, bload<uint32_t>(plane_rsrc<uint32_t>(Ein, plane, 3), io));
  }
}

// ------------------------------------------------------------------------------------------
// Initial state (FP64 arithmetic, rounded to the storage precision).
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ void init_fluid_kernel(Physics p, const double* n_pert, const double* p_init,
                                  void* gv, void* Mv) {
  using S = typename Mode<ST, false>::S;
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= p.nz || j >= p.nr) return;
  const long long u = (long long)j * p.nz + i;
  const long long oo = (long long)j * p.pitch + i;
  const double nb = nbg(p, (double)i * p.h);
  const double n = n_pert ? nb * (1.0 + n_pert[u]) : nb;
  const double a1 = p_init ? n * p_init[u] : 0.0;
  const double a2 = p_init ? n * p_init[(long long)p.nr * p.nz + u] : 0.0;
  double bz, br;
  velocity<double>(n, a1, a2, p.n_floor, bz, br);
  const double uz = p.lam * bz, ur = p.lam * br;
  S* g = (S*)gv;
  A* M = (A*)Mv;
  for (int q = 0; q < 9; ++q) {
    const double w = WQ<double>(q);
    const double cu = XZ(q) * uz + XR(q) * ur;
    const double Q = 3.0 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur);
    // storage 3 keeps the part off the equilibrium, zero here
    const bool z = neq_storage(ST);
    stv(g + q * p.plane + oo, z ? 0.0 : w * ((n - nb) + n * Q));
    stv(g + (9 + q) * p.plane + oo, z ? 0.0 : w * a1 * (1.0 + Q));
    stv(g + (18 + q) * p.plane + oo, z ? 0.0 : w * a2 * (1.0 + Q));
  }
  stv(M + oo, n - nb);
  stv(M + p.plane + oo, a1);
  stv(M + 2 * p.plane + oo, a2);
}

// Driver field from the discrete Gauss law: E_r^{-1} at (z_i, t = -dt), B^{-1/2} at
// (z_i + dz/2, t = -dt/2); E_z = 0.  One thread per column, serial cumulative sum over rows.
template <int ST>
__global__ void init_fields_kernel(Physics p, void* Ev) {
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nz) return;
  A* E = (A*)Ev;
  double ce = 0.0, cb = 0.0;
  const double z = (double)i * p.h;
  for (int j = 0; j < p.nr; ++j) {
    const long long oo = (long long)j * p.pitch + i;
    double er = 0.0, b = 0.0;
    if (p.fields_on && p.driver == 0) {   // a particle bunch sets its field with lbm_set_bunch
      const double r = (j + 0.5) * p.h;
      ce += (j + 0.5) * driver<double>(p, z, r, -p.dt);
      cb += (j + 0.5) * driver<double>(p, z + 0.5 * p.h, r, -0.5 * p.dt);
      er = -p.h * ce / (j + 1.0);
      b = -p.h * cb / (j + 1.0);
    }
    stv(E + oo, 0.0);
    stv(E + p.plane + oo, er);
    stv(E + 2 * p.plane + oo, b);
    if constexpr (fields_lo(ST)) {
      float eh, el, bh, bl;
      split_lo(er, eh, el);
      split_lo(b, bh, bl);
      ((uint32_t*)Ev)[3 * p.plane + oo] = lo_pack(el, bl);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Outputs, state view, diagnostics
// ------------------------------------------------------------------------------------------
template <int ST>
__global__ void moments_out_kernel(Physics p, long long s, const void* Mv, void* dst, int dst_f64) {
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= p.nz || j >= p.nr) return;
  const A* M = (const A*)Mv;
  const long long oo = (long long)j * p.pitch + i;
  const double n = (double)M[oo] + nbg(p, (double)(s + i) * p.h);
  const double a1 = (double)M[p.plane + oo], a2 = (double)M[2 * p.plane + oo];
  double bz, br;
  velocity<double>(n, a1, a2, p.n_floor, bz, br);
  const long long u = (long long)j * p.nz + i, pl = (long long)p.nr * p.nz;
  const double v[3] = {n, n * bz, n * br};
  for (int c = 0; c < 3; ++c) {
    if (dst_f64) ((double*)dst)[c * pl + u] = v[c];
    else ((float*)dst)[c * pl + u] = (float)v[c];
  }
}

template <int ST>
__global__ void fields_out_kernel(Physics p, const void* Ev, void* dst, int dst_f64) {
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= p.nz || j >= p.nr) return;
  const A* E = (const A*)Ev;
  const long long oo = (long long)j * p.pitch + i;
  const long long u = (long long)j * p.nz + i, pl = (long long)p.nr * p.nz;
  for (int c = 0; c < 3; ++c) {
    const double v = (double)E[c * p.plane + oo] + field_lo<ST>(Ev, p.plane, oo, c);
    if (dst_f64) ((double*)dst)[c * pl + u] = v;
    else ((float*)dst)[c * pl + u] = (float)v;
  }
}

// Storage 3: the equilibrium part of population c at a site, from the moments stored there
// (FP64 arithmetic; lattice 0 as the deviation from w n_bg).
template <typename A>
__device__ double neq_equilibrium(const Physics& p, long long s, int i, const A* M, long long oo, int c) {
  const double d0 = (double)M[oo], a1 = (double)M[p.plane + oo], a2 = (double)M[2 * p.plane + oo];
  const double m0 = nbg(p, (double)(s + i) * p.h) + d0;
  double bz, br;
  velocity<double>(m0, a1, a2, p.n_floor, bz, br);
  double e0, e1, e2;
  eq_dir<double>(c % 9, d0, m0, a1, a2, p.lam * bz, p.lam * br, e0, e1, e2);
  return c < 9 ? e0 : (c < 18 ? e1 : e2);
}

template <int ST>
__global__ void state_get_kernel(Physics p, long long s, const void* gv, const void* Mv,
                                 const void* Ev, int c, double* dst) {
  using S = typename Mode<ST, false>::S;
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= p.nz || j >= p.nr) return;
  const long long oo = (long long)j * p.pitch + i;
  double v;
  if (c < 27) {
    v = (double)ldv(((const S*)gv)[c * p.plane + oo]);
    if (neq_storage(ST)) v += neq_equilibrium<A>(p, s, i, (const A*)Mv, oo, c);
    if (c < 9) v += WQ<double>(c) * nbg(p, (double)(s + i) * p.h);
  } else if (c < 30) {
    v = (double)((const A*)Mv)[(c - 27) * p.plane + oo];
    if (c == 27) v += nbg(p, (double)(s + i) * p.h);
  } else {
    v = (double)((const A*)Ev)[(c - 30) * p.plane + oo] + field_lo<ST>(Ev, p.plane, oo, c - 30);
  }
  dst[(long long)j * p.nz + i] = v;
}

template <int ST>
__global__ void state_set_kernel(Physics p, long long s, void* gv, void* Mv, void* Ev, int c,
                                 const double* src) {
  using S = typename Mode<ST, false>::S;
  using A = typename Mode<ST, false>::A;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= p.nz || j >= p.nr) return;
  const long long oo = (long long)j * p.pitch + i;
  double v = src[(long long)j * p.nz + i];
  if (c < 27) {
    if (c < 9) v -= WQ<double>(c) * nbg(p, (double)(s + i) * p.h);
    // storage 3: the moments are set first (the caller's order), the part off their equilibrium here
    if (neq_storage(ST)) v -= neq_equilibrium<A>(p, s, i, (const A*)Mv, oo, c);
    stv(((S*)gv) + c * p.plane + oo, v);
  } else if (c < 30) {
    if (c == 27) v -= nbg(p, (double)(s + i) * p.h);
    stv(((A*)Mv) + (c - 27) * p.plane + oo, v);
  } else {
    stv(((A*)Ev) + (c - 30) * p.plane + oo, v);
    set_field_lo<ST>(Ev, p.plane, oo, c - 30, v);
  }
}

// Wavefront-then-block reduction of 5 FP64 quantities: 0 sum charge, 1 sum energy,
// 2 max |Gauss residual|, 3 max |u*|, 4 sum of non-finite counts.
__device__ __forceinline__ void block_reduce5(double v[5], double* out) {
  __shared__ double sred[RED_THREADS / 64][5];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  for (int off = 32; off > 0; off >>= 1) {
    v[0] += __shfl_down(v[0], off, 64);
    v[1] += __shfl_down(v[1], off, 64);
    v[2] = fmax(v[2], __shfl_down(v[2], off, 64));
    v[3] = fmax(v[3], __shfl_down(v[3], off, 64));
    v[4] += __shfl_down(v[4], off, 64);
  }
  if (lane == 0)
    for (int c = 0; c < 5; ++c) sred[wid][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < RED_THREADS / 64; ++w) {
      r[0] += sred[w][0];
      r[1] += sred[w][1];
      r[2] = fmax(r[2], sred[w][2]);
      r[3] = fmax(r[3], sred[w][3]);
      r[4] += sred[w][4];
    }
    for (int c = 0; c < 5; ++c) out[c] = r[c];
  }
}

// Each thread takes the sites u, u + stride, ... (stride = the whole grid of threads), so a fixed
// number of blocks (at most DIAG_MAX_BLOCKS) covers any lattice.
template <int ST>
__global__ __launch_bounds__(RED_THREADS) void diag_partial_kernel(Physics p, long long k,
                                                                  long long s, const void* Mv,
                                                                  const void* Ev, const double* drv,
                                                                  double* partials) {
  using A = typename Mode<ST, false>::A;
  const long long n = (long long)p.nz * p.nr;
  const long long stride = (long long)gridDim.x * RED_THREADS;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long u = (long long)blockIdx.x * RED_THREADS + threadIdx.x; u < n; u += stride) {
    const int i = (int)(u % p.nz), j = (int)(u / p.nz);
    const A* M = (const A*)Mv;
    const A* E = (const A*)Ev;
    const long long oo = (long long)j * p.pitch + i;
    const double h = p.h, r = (j + 0.5) * h, re = (j + 1.0) * h;
    const double z = (double)(s + i) * h;
    const double nb0 = nbg(p, z);
    const double m0 = (double)M[oo] + nb0, m1 = M[p.plane + oo], m2 = M[2 * p.plane + oo];
    const double ez = E[oo], er = (double)E[p.plane + oo] + field_lo<ST>(Ev, p.plane, oo, 1),
                 b = (double)E[2 * p.plane + oo] + field_lo<ST>(Ev, p.plane, oo, 2);
    const double twopi = 6.283185307179586;
    v[0] += twopi * r * h * h * m0;
    v[1] += 0.5 * twopi * h * h * (r * ez * ez + re * er * er + re * b * b);
    if (i >= 1) {
      const double ezl = E[oo - 1];
      const double erb = j > 0 ? (double)E[p.plane + oo - p.pitch] + field_lo<ST>(Ev, p.plane, oo - p.pitch, 1) : 0.0;
      const double div = (ez - ezl) / h + ((j + 1.0) * er - j * erb) / ((j + 0.5) * h);
      // driver density at t_{k-1}: the closed form, or the bunch density deposited at the nodes
      const double nd = drv ? drv[oo] : driver<double>(p, z, r, ((double)k - 1.0) * p.dt);
      const double rho = nb0 - m0 - nd;
      v[2] = fmax(v[2], fabs(div - rho));
    }
    double bz, br;
    velocity<double>(m0, m1, m2, p.n_floor, bz, br);
    v[3] = fmax(v[3], p.lam * sqrt(bz * bz + br * br));
    const double vals[6] = {(double)M[oo], m1, m2, ez, er, b};
    for (int c = 0; c < 6; ++c) v[4] += isfinite(vals[c]) ? 0.0 : 1.0;
  }
  block_reduce5(v, partials + (long long)blockIdx.x * 8);
}

__global__ __launch_bounds__(RED_THREADS) void diag_final_kernel(const double* partials,
                                                                int nblocks, double* out) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
    const double* q = partials + (long long)b * 8;
    v[0] += q[0];
    v[1] += q[1];
    v[2] = fmax(v[2], q[2]);
    v[3] = fmax(v[3], q[3]);
    v[4] += q[4];
  }
  block_reduce5(v, out);
}

// Bubble length (Sec. IV, Fig. 4): the sites of row `row` at lab positions z in [z0, z1] whose
// electron density is below n_star times the local background (vacuum sites excluded).  One
// block counts the whole row (an integer count: no atomics, exact).
template <int ST>
__global__ __launch_bounds__(RED_THREADS) void bubble_kernel(Physics p, long long s, const void* Mv, int row,
                                                            double n_star, double z0, double z1,
                                                            long long* out) {
  using A = typename Mode<ST, false>::A;
  const A* M = (const A*)Mv;
  long long cnt = 0;
  for (int i = threadIdx.x; i < p.nz; i += RED_THREADS) {
    const double z = (double)(s + i) * p.h;
    const double nb = nbg(p, z);
    const double n = (double)M[(long long)row * p.pitch + i] + nb;
    cnt += (z >= z0 && z <= z1 && nb > 0.0 && n < n_star * nb) ? 1 : 0;
  }
  __shared__ long long red[RED_THREADS / 64];
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
    *out = t;
  }
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
#define LBM_DISPATCH(storage, KERNEL, GRID, BLOCK, STREAM, ...)                      \
  do {                                                                               \
    if ((storage) == 0) KERNEL<0><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);    \
    else if ((storage) == 1) KERNEL<1><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__); \
    else if ((storage) == 2) KERNEL<2><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__); \
    else KERNEL<3><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);                   \
  } while (0)

static dim3 site_grid(const Physics& p) { return dim3((p.nz + 255) / 256, p.nr); }

// A grid that is not periodic takes the variant with the wrap code (an integer modulo by the grid
// size per index) compiled out.
template <int ST, bool M64, int COLL>
static void launch_step_c(const StepArgs& a, dim3 grid, hipStream_t st) {
  const bool np = !a.p.per_z && !a.p.per_r;
  const bool drv = a.p.driver == 1;
  if (a.p.fields_on && drv && np) step_kernel<ST, true, M64, false, COLL, false, 1><<<grid, dim3(NTHREADS), 0, st>>>(a);
  else if (a.p.fields_on && drv) step_kernel<ST, true, M64, false, COLL, true, 1><<<grid, dim3(NTHREADS), 0, st>>>(a);
  else if (a.p.fields_on && np) step_kernel<ST, true, M64, false, COLL, false, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
  else if (a.p.fields_on) step_kernel<ST, true, M64, false, COLL, true, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
  else if (np) step_kernel<ST, false, M64, false, COLL, false, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
  else step_kernel<ST, false, M64, false, COLL, true, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
}

// The site-record variant is the adjoint's forward recompute (no particle driver; FP64
// arithmetic on reduced storage for BGK only).  Without fields it takes the general (wrap)
// variant: that case is not on any timed path.
template <int ST, bool M64, int COLL>
static void launch_step_s(const StepArgs& a, dim3 grid, hipStream_t st) {
  if constexpr (!M64 || COLL == 0) {
    if (a.site_out) {
      if (!a.p.fields_on) step_kernel<ST, false, M64, true, COLL, true, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
      else if (!a.p.per_z && !a.p.per_r) step_kernel<ST, true, M64, true, COLL, false, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
      else step_kernel<ST, true, M64, true, COLL, true, 0><<<grid, dim3(NTHREADS), 0, st>>>(a);
      return;
    }
  }
  launch_step_c<ST, M64, COLL>(a, grid, st);
}

template <int ST, bool M64>
static void launch_step_t(const StepArgs& a, dim3 grid, hipStream_t st) {
  if (a.p.coll == 1) launch_step_s<ST, M64, 1>(a, grid, st);
  else if (a.p.coll == 2) launch_step_s<ST, M64, 2>(a, grid, st);
  else if (a.p.coll == 3) launch_step_s<ST, M64, 3>(a, grid, st);
  else launch_step_s<ST, M64, 0>(a, grid, st);
}

hipError_t launch_step(int storage, const StepArgs& a, hipStream_t st) {
  const int gx = (a.p.nz + TZ - 1) / TZ, gy = (a.p.nr + TR - 1) / TR;
  const dim3 grid(gx * gy);
  if (storage == 0) launch_step_t<0, false>(a, grid, st);
  else if (storage == 1 && a.p.fp64_math) launch_step_t<1, true>(a, grid, st);
  else if (storage == 1) launch_step_t<1, false>(a, grid, st);
  else if (storage == 2 && a.p.fp64_math) launch_step_t<2, true>(a, grid, st);
  else if (storage == 2) launch_step_t<2, false>(a, grid, st);
  else if (a.p.fp64_math) launch_step_t<3, true>(a, grid, st);
  else launch_step_t<3, false>(a, grid, st);
  return hipGetLastError();
}

hipError_t launch_bubble(int storage, const Physics& p, long long s, const void* M, int row, double n_star,
                         double z0, double z1, long long* out, hipStream_t st) {
  LBM_DISPATCH(storage, bubble_kernel, dim3(1), dim3(RED_THREADS), st, p, s, M, row, n_star, z0, z1, out);
  return hipGetLastError();
}

hipError_t launch_init_fluid(int storage, const Physics& p, const double* n_pert,
                             const double* p_init, void* g, void* M, hipStream_t st) {
  LBM_DISPATCH(storage, init_fluid_kernel, site_grid(p), dim3(256), st, p, n_pert, p_init, g, M);
  return hipGetLastError();
}

hipError_t launch_init_fields(int storage, const Physics& p, void* E, hipStream_t st) {
  LBM_DISPATCH(storage, init_fields_kernel, dim3((p.nz + 255) / 256), dim3(256), st, p, E);
  return hipGetLastError();
}

hipError_t launch_moments_out(int storage, const Physics& p, long long s, const void* M,
                              void* dst, int dst_f64, hipStream_t st) {
  LBM_DISPATCH(storage, moments_out_kernel, site_grid(p), dim3(256), st, p, s, M, dst, dst_f64);
  return hipGetLastError();
}

hipError_t launch_fields_out(int storage, const Physics& p, const void* E, void* dst,
                             int dst_f64, hipStream_t st) {
  LBM_DISPATCH(storage, fields_out_kernel, site_grid(p), dim3(256), st, p, E, dst, dst_f64);
  return hipGetLastError();
}

hipError_t launch_state_get(int storage, const Physics& p, long long s, const void* g,
                            const void* M, const void* E, int c, double* dst, hipStream_t st) {
  LBM_DISPATCH(storage, state_get_kernel, site_grid(p), dim3(256), st, p, s, g, M, E, c, dst);
  return hipGetLastError();
}

hipError_t launch_state_set(int storage, const Physics& p, long long s, void* g, void* M,
                            void* E, int c, const double* src, hipStream_t st) {
  LBM_DISPATCH(storage, state_set_kernel, site_grid(p), dim3(256), st, p, s, g, M, E, c, src);
  return hipGetLastError();
}

int diag_blocks(const Physics& p) {
  const long long n = (long long)p.nz * p.nr;
  const long long b = (n + RED_THREADS - 1) / RED_THREADS;
  return (int)(b < DIAG_MAX_BLOCKS ? b : DIAG_MAX_BLOCKS);
}

// Scratch of lbm_diagnostics_noalloc: the partial sums of DIAG_MAX_BLOCKS blocks (8 doubles each)
// and the 8 doubles of the final pass.  One copy per GPU, held until the process ends; every call
// on a GPU uses the same copy (each block overwrites its own partials, so nothing needs clearing).
static __device__ __align__(256) double scratch[(DIAG_MAX_BLOCKS + 1) * 8];

// Device address of the scratch on the current device, looked up once per device.  The array's
// name is a host-side stand-in in host code: kernels and copies take this address instead.
hipError_t diag_scratch(double** ptr) {
  static std::mutex mu;
  static void* addr[MAX_DEVICES] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = a;
  }
  *ptr = (double*)addr[dev];
  return hipSuccess;
}

size_t diag_scratch_doubles() { return sizeof(scratch) / sizeof(double); }

hipError_t launch_diagnostics(int storage, const Physics& p, long long k, long long s,
                              const void* M, const void* E, const double* drv, double* partials, double* out,
                              hipStream_t st) {
  const int nb = diag_blocks(p);
  LBM_DISPATCH(storage, diag_partial_kernel, dim3(nb), dim3(RED_THREADS), st, p, k, s, M, E, drv,
               partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  diag_final_kernel<<<1, RED_THREADS, 0, st>>>(partials, nb, out);
  return hipGetLastError();
}

}  // namespace lbm
