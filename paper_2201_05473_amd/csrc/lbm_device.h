// Device helpers shared by the forward and adjoint kernels of liblbmpwfa (gfx950).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------------------------------------
// Precision modes: population storage S, arithmetic C, auxiliary (moments, fields) storage A.
// ------------------------------------------------------------------------------------------
// C: arithmetic of the fluid phase; CF: arithmetic of the field phase and of the moment halo
// (LDS tiles).  M64 selects FP64 arithmetic for FP32 / FP16 storage (FP64 vector FMAs issue at
// the FP32 rate here, since packed FP32 is not used).
template <int ST, bool M64> struct Mode;
template <bool M64> struct Mode<0, M64> { using S = double; using C = double; using A = double; using CF = double; };
template <> struct Mode<1, false> { using S = float;  using C = float;  using A = float;  using CF = float; };
template <> struct Mode<1, true>  { using S = float;  using C = double; using A = float;  using CF = double; };
template <> struct Mode<2, false> { using S = __half; using C = float;  using A = float;  using CF = float; };
template <> struct Mode<2, true>  { using S = __half; using C = double; using A = float;  using CF = double; };
// FP16 storage of the populations' part off the equilibrium of their site's stored moments
template <> struct Mode<3, false> { using S = __half; using C = float;  using A = float;  using CF = float; };
template <> struct Mode<3, true>  { using S = __half; using C = double; using A = float;  using CF = double; };

// Storage mode 3 keeps, for each population g_q(x), only g_q(x) - f_eq_q(M(x)): its part off the
// equilibrium of the moments M(x) stored at the same site (FP32), in FP16.  That part is small
// next to g_q wherever the flow is near equilibrium, so its 11-bit significand loses far less
// than storing g_q (or its deviation from rest) does.
__host__ __device__ constexpr bool neq_storage(int ST) { return ST == 3; }

__device__ __forceinline__ double ldv(double x) { return x; }
__device__ __forceinline__ float ldv(float x) { return x; }
__device__ __forceinline__ float ldv(__half x) { return __half2float(x); }
__device__ __forceinline__ void stv(double* p, double v) { *p = v; }
__device__ __forceinline__ void stv(float* p, float v) { *p = v; }
__device__ __forceinline__ void stv(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void stv(__half* p, float v) { *p = __float2half_rn(v); }
__device__ __forceinline__ void stv(__half* p, double v) { *p = __float2half_rn((float)v); }

__device__ __forceinline__ float msqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double msqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float mexp(float x) { return expf(x); }
__device__ __forceinline__ double mexp(double x) { return exp(x); }

// D2Q9 velocity set (xi_z, xi_r) and weights; the paper's table (Fig. 2) is not in its text,
// the standard set is used.  Order: rest, +z, +r, -z, -r, (+z,+r), (-z,+r), (-z,-r), (+z,-r).
__host__ __device__ constexpr int XZ(int q) {
  return (q == 1 || q == 5 || q == 8) ? 1 : ((q == 3 || q == 6 || q == 7) ? -1 : 0);
}
__host__ __device__ constexpr int XR(int q) {
  return (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0);
}
// Index of the direction opposite to q.
__host__ __device__ constexpr int OPPQ(int q) { return q == 0 ? 0 : (q < 5 ? (q + 1) % 4 + 1 : (q - 3) % 4 + 5); }
template <typename C> __host__ __device__ constexpr C WQ(int q) {
  return q == 0 ? C(4) / C(9) : (q < 5 ? C(1) / C(9) : C(1) / C(36));
}

// Moment basis of the multiple-relaxation-time operator: value at velocity q of the m-th of the
// nine D2Q9 moment polynomials 1, 3|xi|^2 - 4, (9|xi|^4 - 21|xi|^2 + 8)/2, xi_z, (3|xi|^2 - 5) xi_z,
// xi_r, (3|xi|^2 - 5) xi_r, xi_z^2 - xi_r^2, xi_z xi_r (density, energy, energy square, flux and
// heat flux in z and r, two stresses; orthogonal on the nine velocities), and its squared norm.
__host__ __device__ constexpr int MB(int m, int q) {
  const int z = XZ(q), r = XR(q), q2 = z * z + r * r;
  return m == 0 ? 1 : m == 1 ? 3 * q2 - 4 : m == 2 ? (9 * q2 * q2 - 21 * q2 + 8) / 2 : m == 3 ? z
       : m == 4 ? (3 * q2 - 5) * z : m == 5 ? r : m == 6 ? (3 * q2 - 5) * r : m == 7 ? z * z - r * r : z * r;
}
__host__ __device__ constexpr int MB_NORM2(int m) {
  int sum = 0;
  for (int q = 0; q < 9; ++q) sum += MB(m, q) * MB(m, q);
  return sum;
}

// Sum of the eight moving equilibria of a lattice, from which the rest population's equilibrium
// is taken as the moment minus the sum (equal to Eq. (9) in exact arithmetic).  COMP: Kahan's
// compensated sum in the arithmetic type T, so that the difference is as close to the exact one as
// a sum in twice the precision would give (the running compensation c is the part of the sum lost
// to rounding so far, and the true sum is s - c).  The FP32 step uses it: a plain FP32 sum rounds
// with errors that are correlated between neighbouring sites and steps, and the drift of the
// density and momentum moments they cause grows over a run.
template <typename T, bool COMP>
struct EqSum {
  T s = T(0), c = T(0);
  __device__ __forceinline__ void add(T x) {
    if (COMP) {
      const T y = x - c;
      const T t = s + y;
      c = (t - s) - y;
      s = t;
    } else {
      s += x;
    }
  }
  // m minus the sum
  __device__ __forceinline__ T rest(T m) const { return COMP ? (m - s) + c : m - s; }
};

// Equilibrium of direction q (Eq. (9), standard D2Q9 coefficients) for the three lattices at
// moments with density deviation d0 from n_bg (density m0 = n_bg + d0), momenta a1, a2 and lattice
// velocity (uz, ur); lattice 0 as the deviation from w_q n_bg.
template <typename C>
__device__ __forceinline__ void eq_dir(int q, C d0, C m0, C a1, C a2, C uz, C ur, C& e0, C& e1, C& e2) {
  const C w = WQ<C>(q);
  const C cu = (C)XZ(q) * uz + (C)XR(q) * ur;
  const C Q = C(3) * cu + C(4.5) * cu * cu - C(1.5) * (uz * uz + ur * ur);
  e0 = w * (d0 + m0 * Q);
  e1 = w * a1 * (C(1) + Q);
  e2 = w * a2 * (C(1) + Q);
}

// Background (ion) density n_bg(z): uniform, linear ramp or tanh ramp (always FP64).
__device__ __forceinline__ double nbg(const Physics& p, double z) {
  if (p.ramp_kind == 0) return p.n0;
  const double x = (z - p.ramp_start) / p.ramp_len;
  if (p.ramp_kind == 1) return p.n0 * fmin(fmax(x, 0.0), 1.0);
  return p.n0 * 0.5 * (1.0 + tanh(2.0 * x - 1.0));
}

// Rigid bi-Gaussian driver moving at c, evaluated in arithmetic type C.
template <typename C>
__device__ __forceinline__ C driver(const Physics& p, double z, double r, double t) {
  const C dz = (C)(z - (p.zd0 + t));
  const C rr = (C)r;
  return (C)p.nb * mexp(-(dz * dz) / (C)(2.0 * p.sigma_z * p.sigma_z)) *
         mexp(-(rr * rr) / (C)(2.0 * p.sigma_r * p.sigma_r));
}

// beta = p / gamma from the moments (Eq. (2), third line); zero at or below the density floor.
__device__ __forceinline__ float mrsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double mrsqrt(double x) { return 1.0 / sqrt(x); }

template <typename C>
__device__ __forceinline__ bool velocity(C n, C a1, C a2, C floor_, C& bz, C& br) {
  if (!(n > floor_)) { bz = C(0); br = C(0); return false; }
  const C in = C(1) / n;
  const C pz = a1 * in, pr = a2 * in;
  const C ig = mrsqrt(C(1) + pz * pz + pr * pr);
  bz = pz * ig;
  br = pr * ig;
  return true;
}
// FP32: beta = p / sqrt(1 + p^2) with p = a / n is a / sqrt(n^2 + a^2) for n > 0, which needs one
// hardware reciprocal square root (1 ulp) and no division.  n > n_floor > 0 keeps n^2 normal for any
// floor above 1e-19.
template <>
__device__ __forceinline__ bool velocity<float>(float n, float a1, float a2, float floor_, float& bz, float& br) {
  if (!(n > floor_)) { bz = 0.f; br = 0.f; return false; }
  const float ig = __builtin_amdgcn_rsqf(n * n + a1 * a1 + a2 * a2);
  bz = a1 * ig;
  br = a2 * ig;
  return true;
}

// Buffer accesses.  A plane (or any array) is addressed through a buffer resource in scalar
// registers (its base and size, uniform) and a 32-bit byte offset per lane, so no lane computes a
// 64-bit address; an access past the resource's size reads zero and writes nothing.  Word 3 of
// the resource is the raw-buffer format of the gfx9 family.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc brsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// cache policy of a load: 0 default, 2 non-temporal
template <int POL = 0> __device__ __forceinline__ float bld(float*, Rsrc r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, POL));
}
template <int POL = 0> __device__ __forceinline__ double bld(double*, Rsrc r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, POL));
}
template <int POL = 0> __device__ __forceinline__ __half bld(__half*, Rsrc r, uint32_t off) {
  return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, POL));
}
template <int POL = 0> __device__ __forceinline__ uint32_t bld(uint32_t*, Rsrc r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, POL);
}
// load of element `idx` of an array of T through resource r
template <typename T, int POL = 0> __device__ __forceinline__ T bload(Rsrc r, uint32_t idx) {
  return bld<POL>((T*)nullptr, r, idx * (uint32_t)sizeof(T));
}
// Groups of planes under one resource: element idx of the plane that starts soff bytes into the
// group (soff uniform, a scalar operand of the instruction), so the planes of a group need no
// resource each.  FP32 and FP16 only (a group must stay under 4 GiB).
template <int POL = 0> __device__ __forceinline__ float bldg(float*, Rsrc r, uint32_t off, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, POL));
}
template <int POL = 0> __device__ __forceinline__ __half bldg(__half*, Rsrc r, uint32_t off, uint32_t soff) {
  return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, POL));
}
template <typename T, int POL = 0> __device__ __forceinline__ T bload_g(Rsrc r, uint32_t idx, uint32_t soff) {
  return bldg<POL>((T*)nullptr, r, idx * (uint32_t)sizeof(T), soff);
}
__device__ __forceinline__ void bputg(float*, Rsrc r, uint32_t idx, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(idx * 4u), (int)soff, 0);
}
__device__ __forceinline__ void bputg(float*, Rsrc r, uint32_t idx, uint32_t soff, double v) {
  bputg((float*)nullptr, r, idx, soff, (float)v);
}
__device__ __forceinline__ void bputg(__half*, Rsrc r, uint32_t idx, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(v)), r, (int)(idx * 2u),
                                        (int)soff, 0);
}
__device__ __forceinline__ void bputg(__half*, Rsrc r, uint32_t idx, uint32_t soff, double v) {
  bputg((__half*)nullptr, r, idx, soff, (float)v);
}
template <typename T, typename V> __device__ __forceinline__ void bstore_g(Rsrc r, uint32_t idx, uint32_t soff, V v) {
  bputg((T*)nullptr, r, idx, soff, v);
}
// store of v, rounded to the storage type T (round to nearest even), to element idx
__device__ __forceinline__ void bput(double*, Rsrc r, uint32_t idx, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                        (int)(idx * 8u), 0, 0);
}
__device__ __forceinline__ void bput(float*, Rsrc r, uint32_t idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(idx * 4u), 0, 0);
}
__device__ __forceinline__ void bput(float*, Rsrc r, uint32_t idx, double v) { bput((float*)nullptr, r, idx, (float)v); }
__device__ __forceinline__ void bput(__half*, Rsrc r, uint32_t idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(v)), r, (int)(idx * 2u), 0, 0);
}
__device__ __forceinline__ void bput(__half*, Rsrc r, uint32_t idx, double v) { bput((__half*)nullptr, r, idx, (float)v); }
__device__ __forceinline__ void bput(uint32_t*, Rsrc r, uint32_t idx, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)(idx * 4u), 0, 0);
}
template <typename T, typename V> __device__ __forceinline__ void bstore(Rsrc r, uint32_t idx, V v) {
  bput((T*)nullptr, r, idx, v);
}
// resource over plane c of a group of planes of `plane` elements of T starting at base
template <typename T> __device__ __forceinline__ Rsrc plane_rsrc(const void* base, long long plane, int c) {
  return brsrc((const T*)base + (long long)c * plane, (uint32_t)(plane * (long long)sizeof(T)));
}

// Compensated fields of FP32 storage.  E_r and B_theta are kept as an FP32 value plus the part
// that value misses, rounded to bfloat16 (8 more significand bits: 2^-32 relative together), so
// that the field update accumulates its increments without an FP32 rounding per step.  The two
// residuals of a cell share one 32-bit word of a fourth field plane: E_r's in the low half,
// B_theta's in the high half.  Without them, the FP32 rounding of the large driver fields E_r and
// B_theta, stored step after step, sets the E_z error of a young wake near 1e-5 (CPU emulation in
// the oracle: 1.0e-5 after 400 steps of C2's 512 x 128 copy; with the residuals, 6e-7).
// bfloat16 of x, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float lo_er(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float lo_b(uint32_t w) { return __builtin_bit_cast(float, w & 0xFFFF0000u); }
__device__ __forceinline__ uint32_t lo_pack(float er_lo, float b_lo) {
  return bf16_rne(er_lo) | (bf16_rne(b_lo) << 16);
}
// FP32 value and residual of a double
__device__ __forceinline__ void split_lo(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}
// (hi + lo) + d in FP32 without losing d's low bits: hi becomes the rounded sum, lo the part it
// misses (Knuth's two-sum of hi and d, the error added to lo, then renormalised).  No contraction
// into FMAs, which would change the error terms.
__device__ __forceinline__ void acc_comp(float& hi, float& lo, float d) {
#pragma clang fp contract(off)
  const float s = hi + d;
  const float bp = s - hi;
  const float err = (hi - (s - bp)) + (d - bp);
  const float l = lo + err;
  const float h2 = s + l;
  lo = l - (h2 - s);
  hi = h2;
}

// Residual of field component c (0 E_z, 1 E_r, 2 B_theta) of cell oo, in a field group of planes
// of `plane` elements (zero where the storage keeps none)
template <int ST>
__device__ __forceinline__ double field_lo(const void* E, long long plane, long long oo, int c) {
  if constexpr (fields_lo(ST)) {
    if (c == 0) return 0.0;
    const uint32_t w = ((const uint32_t*)E)[3 * plane + oo];
    return (double)(c == 1 ? lo_er(w) : lo_b(w));
  } else {
    return 0.0;
  }
}
// Store the residual of v (whose FP32 value the caller stores) for field component c of cell oo
template <int ST>
__device__ __forceinline__ void set_field_lo(void* E, long long plane, long long oo, int c, double v) {
  if constexpr (fields_lo(ST)) {
    if (c == 0) return;
    float hi, lo;
    split_lo(v, hi, lo);
    uint32_t* w = (uint32_t*)E + 3 * plane + oo;
    *w = c == 1 ? ((*w & 0xFFFF0000u) | bf16_rne(lo)) : ((*w & 0xFFFFu) | (bf16_rne(lo) << 16));
  }
}

// Population loads of the step: FP64 populations are read with non-temporal loads (measured on
// MI355X: FP64 step 110 -> 96.5 us on 2048 x 512; the same for FP32 loads is 25 % slower, so
// FP32 and FP16 use ordinary loads).
__device__ __forceinline__ float ldpop(const float* p) { return *p; }
__device__ __forceinline__ double ldpop(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ __half ldpop(const __half* p) { return *p; }

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// XCD-aware block -> tile map: consecutive tiles go to the same XCD (blocks are dispatched
// round-robin over the 8 XCDs), so halo and pull neighbours share an L2.  A bijection.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int per = nblocks / 8, rem = nblocks % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

}  // namespace lbm
