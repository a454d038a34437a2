// Memory-pattern ceiling of the FP32 step: the rate the chip sustains for the step's own access
// pattern when no arithmetic is attached to it, beside a plain float4 copy of the same bytes.
//
// The FP32 step moves 272 B per site: the 27 populations pulled from the neighbours along the
// lattice velocities (three D2Q9 lattices, pull offsets clamped to the grid), the 7 auxiliary words
// of the site (3 moments, E_z, E_r, B_theta and the residual word) read, and all 34 written back at
// the site.  The FP16 step moves 156 B (2-byte populations, 6 FP32 auxiliary words), the FP64 step
// 528 B (8-byte populations, 6 FP64 auxiliary words); they are measured on C3 as well.  pattern_kernel does exactly that with one site per thread on 64 x 4 tiles (the step's
// tile), in the step's layout (planes 256 bytes longer than their rows, so that the 34 streams of
// a site do not start on the same memory channels) and with the step's XCD-aware tile order; its
// rate bounds what any arrangement of the step's arithmetic around that pattern can reach.  The
// same kernel on unpadded planes in plain block order, and copy_kernel moving the same number of
// bytes as one contiguous float4 stream, are measured beside it.
//
// With --arith the FP32 pattern is measured again on both grids with 27 w dependent-free
// multiply-adds per site added between the loads and the stores (w = 0 .. 48; the step issues about
// 1,400 vector instructions per site): how much arithmetic the pattern's rate absorbs on a grid the
// MALL partly serves (C2) and on one it cannot (C3).
//
// With --zmarch the FP32 pattern is measured as a z-marching kernel instead: each block walks SEG
// consecutive tiles of one row strip along z (blocks in the XCD-aware order), issuing the next
// tile's loads before the current tile's stores.
//
// With --shift the FP32 pattern is measured with its pull offsets switched off (every load at the
// site: rows start 256-byte aligned), with the row offsets only (still aligned), with the full pull
// (the z offsets make 18 of the 27 loads start 4 bytes off a cache line), and with the z offsets
// taken by aligned row loads realigned across lanes (a wavefront DPP shift by one lane, the column
// past the wavefront's end from a single-lane load), and with the z offsets moved to the stores (each
// population plane stored shifted by its z velocity).  The realigned outputs are first checked
// against the full pull's bit for bit.
//
// With --pingpong the FP32 pattern runs as the step does, alternating between two buffer sets so
// that each launch reads what the previous one wrote (the other measurements read one input set
// every launch, which the MALL can keep), on C2, on a grid of the paper's size (2432 x 400, the
// paper's 2400 columns rounded up to the tile) and on C3.
//
// With --layout the FP32 pattern (full pull) is measured beside two other arrangements of the same
// 272 B per site, each with and without the pull's offsets: a chunked layout (the 3 lattices of a
// direction in one plane as [row][64-column chunk][lattice][64], the 7 auxiliary words in one plane
// likewise: 10 streams each way instead of 34) and four sites per lane with 16-byte accesses.
//
// Standalone program (not part of the library): prints one JSON line per measurement.  Every index
// is clamped into the arrays, and the grids are whole multiples of the tile.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
      exit(1);                                                                             \
    }                                                                                      \
  } while (0)

namespace {

constexpr int TZ = 64, TR = 4, NPOP = 27;

struct Grid {
  int nz, nr;
  long long plane;   // nz * nr plus the pad (nz is a multiple of 64: rows start 256-byte aligned)
};

// blocks are dispatched round-robin over the 8 XCDs; this bijection gives each XCD a run of
// consecutive tiles, so that pull neighbours share an L2 (the step's tile order)
__device__ __forceinline__ int xcd_order(int b, int nblocks) {
  const int per = nblocks / 8, rem = nblocks % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// D2Q9 velocity components of direction q (rest, 4 axis, 4 diagonal)
__device__ __forceinline__ int cz(int q) { return (q == 1 || q == 5 || q == 8) ? 1 : ((q == 3 || q == 6 || q == 7) ? -1 : 0); }
__device__ __forceinline__ int cr(int q) { return (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0); }
__device__ __forceinline__ int clampi(int x, int n) { return x < 0 ? 0 : (x >= n ? n - 1 : x); }

// WORK: rounds of 27 multiply-adds per site between the loads and the stores (0: the pure pattern).
// SHIFT: 0 no pull offsets, 1 row offsets only, 2 the full pull, 3 the full pull with the z offsets
// realigned across lanes (FP32; every lane active, as the DPP shift needs), 4 the z offsets on the
// stores instead
template <typename P, typename X, int NAUX, bool XCD, int WORK, int SHIFT = 2>
__global__ __launch_bounds__(TZ * TR) void pattern_kernel(Grid g, const P* __restrict__ pin, P* __restrict__ pout,
                                                          const X* __restrict__ ain, X* __restrict__ aout) {
  const int gx = g.nz / TZ;
  const int tile = XCD ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
  const int i = (tile % gx) * TZ + threadIdx.x % TZ;
  const int j = (tile / gx) * TR + threadIdx.x / TZ;
  X f[NPOP], a[NAUX];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if constexpr (SHIFT == 3 && sizeof(P) == 4) {
      // aligned row load, realigned across lanes with a wavefront DPP shift; the one column past the
      // row's end comes from a single-lane load
      const int lane = threadIdx.x % 64;
      const int i0 = i - lane;
      const long long rowb = (long long)clampi(j - cr(q), g.nr) * g.nz;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const P* src = pin + (9 * l + q) * g.plane + rowb;
        const int v = __builtin_bit_cast(int, (float)src[i]);
        if (cz(q) == 0) {
          f[9 * l + q] = (X)__builtin_bit_cast(float, v);
        } else {
          int e = 0;
          const int edge = cz(q) > 0 ? 0 : 63;
          if (lane == edge) e = __builtin_bit_cast(int, (float)src[clampi(cz(q) > 0 ? i0 - 1 : i0 + 64, g.nz)]);
          const int sh = cz(q) > 0 ? __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true)
                                   : __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
          f[9 * l + q] = (X)__builtin_bit_cast(float, sh | e);
        }
      }
    } else {
      const int dz = SHIFT == 2 ? cz(q) : 0, dr = SHIFT >= 1 ? cr(q) : 0;
      const long long off = (long long)clampi(j - dr, g.nr) * g.nz + clampi(i - dz, g.nz);
#pragma unroll
      for (int l = 0; l < 3; ++l) f[9 * l + q] = (X)pin[(9 * l + q) * g.plane + off];
    }
  }
  const long long o = (long long)j * g.nz + i;
#pragma unroll
  for (int c = 0; c < NAUX; ++c) a[c] = ain[c * g.plane + o];
  // a dependence of every output on every input keeps all loads; no other arithmetic
  X s = X(0);
#pragma unroll
  for (int c = 0; c < NPOP; ++c) s += f[c];
#pragma unroll 1
  for (int w = 0; w < WORK; ++w) {
#pragma unroll
    for (int c = 0; c < NPOP; ++c) f[c] = f[c] * X(0.999999) + X(1e-9) * s;
  }
#pragma unroll
  for (int c = 0; c < NPOP; ++c) {
    // SHIFT 4: each population plane stored shifted by its own z velocity, so that the pull's z
    // offsets move from the loads to the stores (rows still pulled)
    const long long oc = SHIFT == 4 ? (long long)j * g.nz + clampi(i + cz(c % 9), g.nz) : o;
    pout[c * g.plane + oc] = (P)(f[c] + X(1e-7) * s);
  }
#pragma unroll
  for (int c = 0; c < NAUX; ++c) aout[c * g.plane + o] = a[c] + X(1e-7) * s;
}

// z-marching: block b owns SEG consecutive tiles of one row strip and walks them along z, the next
// tile's 34 loads issued before the current tile's 34 stores (FP32 only)
template <int SEG>
__global__ __launch_bounds__(TZ * TR) void zmarch_kernel(Grid g, const float* __restrict__ pin, float* __restrict__ pout,
                                                         const float* __restrict__ ain, float* __restrict__ aout) {
  const int gx = g.nz / TZ;
  const int segs = gx / SEG;
  const int bid = xcd_order(blockIdx.x, gridDim.x);
  const int strip = bid / segs, seg = bid % segs;
  const int j = strip * TR + threadIdx.x / TZ;
  float f[NPOP], a[7], fn[NPOP], an[7];
  auto load = [&](int tile, float* ff, float* aa) {
    const int i = tile * TZ + threadIdx.x % TZ;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const long long off = (long long)clampi(j - cr(q), g.nr) * g.nz + clampi(i - cz(q), g.nz);
#pragma unroll
      for (int l = 0; l < 3; ++l) ff[9 * l + q] = pin[(9 * l + q) * g.plane + off];
    }
    const long long o = (long long)j * g.nz + i;
#pragma unroll
    for (int c = 0; c < 7; ++c) aa[c] = ain[c * g.plane + o];
  };
  const int t0 = seg * SEG;
  load(t0, f, a);
  for (int t = 0; t < SEG; ++t) {
    if (t + 1 < SEG) load(t0 + t + 1, fn, an);
    const int i = (t0 + t) * TZ + threadIdx.x % TZ;
    const long long o = (long long)j * g.nz + i;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NPOP; ++c) s += f[c];
#pragma unroll
    for (int c = 0; c < NPOP; ++c) pout[c * g.plane + o] = f[c] + 1e-7f * s;
#pragma unroll
    for (int c = 0; c < 7; ++c) aout[c * g.plane + o] = a[c] + 1e-7f * s;
#pragma unroll
    for (int c = 0; c < NPOP; ++c) f[c] = fn[c];
#pragma unroll
    for (int c = 0; c < 7; ++c) a[c] = an[c];
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ in, float4* __restrict__ out,
                                                   long long n4) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t < n4) {
    float4 v = in[t];
    v.x += 1e-7f;
    out[t] = v;
  }
}

}  // namespace

// One measurement: the pattern (step layout and order, then unpadded and in plain order) and the
// float4 copy of the same bytes, for population type P and NAUX auxiliary words of type X.
template <typename P, typename X, int NAUX, int WORK = 0>
void measure(const char* name, int nz, int nr, int iters, bool variants) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = (long long)nz * nr + 256 / (long long)sizeof(P);   // the step's pad: 256 bytes
  Grid gu = g;
  gu.plane = (long long)nz * nr;
  const long long sites = (long long)nz * nr;
  const int bps = 2 * (NPOP * (int)sizeof(P) + NAUX * (int)sizeof(X));
  const double bytes = (double)bps * sites;
  P *pin, *pout;
  X *ain, *aout;
  CK(hipMalloc(&pin, NPOP * g.plane * sizeof(P)));
  CK(hipMalloc(&pout, NPOP * g.plane * sizeof(P)));
  CK(hipMalloc(&ain, NAUX * g.plane * sizeof(X)));
  CK(hipMalloc(&aout, NAUX * g.plane * sizeof(X)));
  CK(hipMemset(pin, 0, NPOP * g.plane * sizeof(P)));
  CK(hipMemset(ain, 0, NAUX * g.plane * sizeof(X)));
  // the copy moves the same bytes: the population planes of pin to pout, then the auxiliary ones
  const long long n4p = NPOP * g.plane * (long long)sizeof(P) / 16, n4a = NAUX * g.plane * (long long)sizeof(X) / 16;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const int tiles = (nz / TZ) * (nr / TR);
  const char* kname[3] = {"step access pattern (pull, 64x4 tiles, step layout and tile order)",
                          "same pattern, unpadded planes, plain block order", "float4 copy, same bytes"};
  for (int k = 0; k < 3; ++k) {
    if (k == 1 && !variants) continue;
    auto launch = [&] {
      if (k == 0) {
        pattern_kernel<P, X, NAUX, true, WORK><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
      } else if (k == 1) {
        pattern_kernel<P, X, NAUX, false, WORK><<<tiles, TZ * TR>>>(gu, pin, pout, ain, aout);
      } else {
        copy_kernel<<<(unsigned)((n4p + 255) / 256), 256>>>((const float4*)pin, (float4*)pout, n4p);
        copy_kernel<<<(unsigned)((n4a + 255) / 256), 256>>>((const float4*)ain, (float4*)aout, n4a);
      }
    };
    for (int it = 0; it < 20; ++it) launch();
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int it = 0; it < iters; ++it) launch();
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipGetLastError());
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double us = ms * 1e3 / iters;
    printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"%s\", \"fma_per_site\": %d, \"bytes_per_site\": %d, "
           "\"us\": %.2f, \"GBps\": %.1f, \"frac_of_8TBps\": %.4f}\n",
           name, nz, nr, kname[k], k == 2 ? 0 : NPOP * WORK, bps, us, bytes / us / 1e3, bytes / us / 1e3 / 8000.0);
    fflush(stdout);
  }
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  CK(hipFree(pin));
  CK(hipFree(pout));
  CK(hipFree(ain));
  CK(hipFree(aout));
}

template <int SEG>
void measure_z(const char* name, int nz, int nr, int iters) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = (long long)nz * nr + 64;
  const double bytes = 272.0 * (double)nz * nr;
  float *pin, *pout, *ain, *aout;
  CK(hipMalloc(&pin, NPOP * g.plane * 4));
  CK(hipMalloc(&pout, NPOP * g.plane * 4));
  CK(hipMalloc(&ain, 7 * g.plane * 4));
  CK(hipMalloc(&aout, 7 * g.plane * 4));
  CK(hipMemset(pin, 0, NPOP * g.plane * 4));
  CK(hipMemset(ain, 0, 7 * g.plane * 4));
  const int blocks = (nr / TR) * (nz / TZ / SEG);
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int it = 0; it < 20; ++it) zmarch_kernel<SEG><<<blocks, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int it = 0; it < iters; ++it) zmarch_kernel<SEG><<<blocks, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipGetLastError());
  float ms;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = ms * 1e3 / iters;
  printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"z-march, %d tiles per block\", \"us\": %.2f, \"frac_of_8TBps\": %.4f}\n",
         name, nz, nr, SEG, us, bytes / us / 1e3 / 8000.0);
  fflush(stdout);
  CK(hipFree(pin));
  CK(hipFree(pout));
  CK(hipFree(ain));
  CK(hipFree(aout));
}

template <int SHIFT>
void measure_s(const char* name, int nz, int nr, int iters) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = (long long)nz * nr + 64;
  const double bytes = 272.0 * (double)nz * nr;
  float *pin, *pout, *ain, *aout;
  CK(hipMalloc(&pin, NPOP * g.plane * 4));
  CK(hipMalloc(&pout, NPOP * g.plane * 4));
  CK(hipMalloc(&ain, 7 * g.plane * 4));
  CK(hipMalloc(&aout, 7 * g.plane * 4));
  CK(hipMemset(pin, 0, NPOP * g.plane * 4));
  CK(hipMemset(ain, 0, 7 * g.plane * 4));
  const int tiles = (nz / TZ) * (nr / TR);
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int it = 0; it < 20; ++it) pattern_kernel<float, float, 7, true, 0, SHIFT><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int it = 0; it < iters; ++it) pattern_kernel<float, float, 7, true, 0, SHIFT><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipGetLastError());
  float ms;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = ms * 1e3 / iters;
  printf("{\"workload\": \"%s %dx%d\", \"shift_mode\": %d, \"us\": %.2f, \"frac_of_8TBps\": %.4f}\n",
         name, nz, nr, SHIFT, us, bytes / us / 1e3 / 8000.0);
  fflush(stdout);
  CK(hipFree(pin));
  CK(hipFree(pout));
  CK(hipFree(ain));
  CK(hipFree(aout));
}

// Chunked layout: the 3 lattices of one direction share a plane, [row][64-column chunk][lattice][64],
// and the 7 auxiliary words of a site share one plane, [row][chunk][word][64]: 10 streams each way.
template <int PULL>
__global__ __launch_bounds__(TZ * TR) void chunk_kernel(Grid g, const float* __restrict__ pin, float* __restrict__ pout,
                                                        const float* __restrict__ ain, float* __restrict__ aout) {
  const int gx = g.nz / TZ;
  const int tile = xcd_order(blockIdx.x, gridDim.x);
  const int i = (tile % gx) * TZ + threadIdx.x % TZ;
  const int j = (tile / gx) * TR + threadIdx.x / TZ;
  const long long qplane = 3LL * g.nz * g.nr + 64;
  float f[NPOP], a[7];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int jj = PULL ? clampi(j - cr(q), g.nr) : j, ii = PULL ? clampi(i - cz(q), g.nz) : i;
    const long long base = q * qplane + (long long)jj * 3 * g.nz + (ii / 64) * 192 + ii % 64;
#pragma unroll
    for (int l = 0; l < 3; ++l) f[9 * l + q] = pin[base + 64 * l];
  }
  const long long ob = (long long)j * 7 * g.nz + (i / 64) * 448 + i % 64;
#pragma unroll
  for (int c = 0; c < 7; ++c) a[c] = ain[ob + 64 * c];
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < NPOP; ++c) s += f[c];
  const long long pb = (long long)j * 3 * g.nz + (i / 64) * 192 + i % 64;
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int l = 0; l < 3; ++l) pout[q * qplane + pb + 64 * l] = f[9 * l + q] + 1e-7f * s;
#pragma unroll
  for (int c = 0; c < 7; ++c) aout[ob + 64 * c] = a[c] + 1e-7f * s;
}

template <int PULL>
void measure_c(const char* name, int nz, int nr, int iters) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = 0;   // unused: the chunked planes have their own strides
  const long long qplane = 3LL * nz * nr + 64;
  const double bytes = 272.0 * (double)nz * nr;
  float *pin, *pout, *ain, *aout;
  CK(hipMalloc(&pin, 9 * qplane * 4));
  CK(hipMalloc(&pout, 9 * qplane * 4));
  CK(hipMalloc(&ain, 7LL * nz * nr * 4));
  CK(hipMalloc(&aout, 7LL * nz * nr * 4));
  CK(hipMemset(pin, 0, 9 * qplane * 4));
  CK(hipMemset(ain, 0, 7LL * nz * nr * 4));
  const int tiles = (nz / TZ) * (nr / TR);
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int it = 0; it < 20; ++it) chunk_kernel<PULL><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int it = 0; it < iters; ++it) chunk_kernel<PULL><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipGetLastError());
  float ms;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = ms * 1e3 / iters;
  printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"chunked layout, pull %d\", \"us\": %.2f, \"frac_of_8TBps\": %.4f}\n",
         name, nz, nr, PULL, us, bytes / us / 1e3 / 8000.0);
  fflush(stdout);
  CK(hipFree(pin));
  CK(hipFree(pout));
  CK(hipFree(ain));
  CK(hipFree(aout));
}

// Four sites per lane: 16-byte loads and stores (a block: 256 columns x 4 rows), the planar layout
// of the step; the pulled loads start 4 bytes off 16 (the hardware takes dword-aligned 16-byte
// accesses), clamped so that all four columns lie in the row.
struct __attribute__((aligned(4))) F4 { float x, y, z, w; };
template <int PULL>
__global__ __launch_bounds__(256) void vec4_kernel(Grid g, const float* __restrict__ pin, float* __restrict__ pout,
                                                   const float* __restrict__ ain, float* __restrict__ aout) {
  const int gx = g.nz / 256;
  const int tile = xcd_order(blockIdx.x, gridDim.x);
  const int i = (tile % gx) * 256 + 4 * (threadIdx.x % 64);
  const int j = (tile / gx) * 4 + threadIdx.x / 64;
  F4 f[NPOP], a[7];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int jj = PULL ? clampi(j - cr(q), g.nr) : j;
    int ii = PULL ? i - cz(q) : i;
    ii = ii < 0 ? 0 : (ii > g.nz - 4 ? g.nz - 4 : ii);
    const long long off = (long long)jj * g.nz + ii;
#pragma unroll
    for (int l = 0; l < 3; ++l) f[9 * l + q] = *(const F4*)(pin + (9 * l + q) * g.plane + off);
  }
  const long long o = (long long)j * g.nz + i;
#pragma unroll
  for (int c = 0; c < 7; ++c) a[c] = *(const F4*)(ain + c * g.plane + o);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < NPOP; ++c) s += f[c].x + f[c].y + f[c].z + f[c].w;
#pragma unroll
  for (int c = 0; c < NPOP; ++c) {
    F4 v = f[c];
    v.x += 1e-7f * s; v.y += 1e-7f * s; v.z += 1e-7f * s; v.w += 1e-7f * s;
    *(F4*)(pout + c * g.plane + o) = v;
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    F4 v = a[c];
    v.x += 1e-7f * s; v.y += 1e-7f * s; v.z += 1e-7f * s; v.w += 1e-7f * s;
    *(F4*)(aout + c * g.plane + o) = v;
  }
}

template <int PULL>
void measure_v(const char* name, int nz, int nr, int iters) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = (long long)nz * nr + 64;
  const double bytes = 272.0 * (double)nz * nr;
  float *pin, *pout, *ain, *aout;
  CK(hipMalloc(&pin, NPOP * g.plane * 4));
  CK(hipMalloc(&pout, NPOP * g.plane * 4));
  CK(hipMalloc(&ain, 7 * g.plane * 4));
  CK(hipMalloc(&aout, 7 * g.plane * 4));
  CK(hipMemset(pin, 0, NPOP * g.plane * 4));
  CK(hipMemset(ain, 0, 7 * g.plane * 4));
  const int tiles = (nz / 256) * (nr / 4);
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int it = 0; it < 20; ++it) vec4_kernel<PULL><<<tiles, 256>>>(g, pin, pout, ain, aout);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int it = 0; it < iters; ++it) vec4_kernel<PULL><<<tiles, 256>>>(g, pin, pout, ain, aout);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipGetLastError());
  float ms;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = ms * 1e3 / iters;
  printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"4 sites per lane, pull %d\", \"us\": %.2f, \"frac_of_8TBps\": %.4f}\n",
         name, nz, nr, PULL, us, bytes / us / 1e3 / 8000.0);
  fflush(stdout);
  CK(hipFree(pin));
  CK(hipFree(pout));
  CK(hipFree(ain));
  CK(hipFree(aout));
}

// The FP32 pattern as the step runs it: two buffer sets, each launch reading the set the previous
// one wrote (the other measurements read the same input every launch).
void measure_pp(const char* name, int nz, int nr, int iters) {
  Grid g;
  g.nz = nz;
  g.nr = nr;
  g.plane = (long long)nz * nr + 64;
  const double bytes = 272.0 * (double)nz * nr;
  float *p0, *p1, *a0, *a1;
  CK(hipMalloc(&p0, NPOP * g.plane * 4));
  CK(hipMalloc(&p1, NPOP * g.plane * 4));
  CK(hipMalloc(&a0, 7 * g.plane * 4));
  CK(hipMalloc(&a1, 7 * g.plane * 4));
  CK(hipMemset(p0, 0, NPOP * g.plane * 4));
  CK(hipMemset(p1, 0, NPOP * g.plane * 4));
  CK(hipMemset(a0, 0, 7 * g.plane * 4));
  CK(hipMemset(a1, 0, 7 * g.plane * 4));
  const int tiles = (nz / TZ) * (nr / TR);
  auto launch = [&](int it) {
    if (it & 1) pattern_kernel<float, float, 7, true, 0, 2><<<tiles, TZ * TR>>>(g, p1, p0, a1, a0);
    else pattern_kernel<float, float, 7, true, 0, 2><<<tiles, TZ * TR>>>(g, p0, p1, a0, a1);
  };
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int it = 0; it < 20; ++it) launch(it);
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int it = 0; it < iters; ++it) launch(it);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipGetLastError());
  float ms;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double us = ms * 1e3 / iters;
  printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"step access pattern, ping-pong buffers\", \"us\": %.2f, "
         "\"frac_of_8TBps\": %.4f}\n", name, nz, nr, us, bytes / us / 1e3 / 8000.0);
  fflush(stdout);
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  CK(hipFree(p0));
  CK(hipFree(p1));
  CK(hipFree(a0));
  CK(hipFree(a1));
}

// The realigned pull (SHIFT 3) against the full pull (SHIFT 2) on the same input, C2's grid: the
// outputs must agree bit for bit.
bool realigned_pull_matches() {
  Grid g;
  g.nz = 2048;
  g.nr = 512;
  g.plane = (long long)g.nz * g.nr + 64;
  const size_t np = NPOP * g.plane, na = 7 * g.plane;
  float *pin, *o2, *o3, *ain, *aout;
  CK(hipMalloc(&pin, np * 4));
  CK(hipMalloc(&o2, np * 4));
  CK(hipMalloc(&o3, np * 4));
  CK(hipMalloc(&ain, na * 4));
  CK(hipMalloc(&aout, na * 4));
  float* h = (float*)malloc(np * 4);
  float* h2 = (float*)malloc(np * 4);
  if (!h || !h2) {
    fprintf(stderr, "host allocation failed\n");
    exit(1);
  }
  for (size_t t = 0; t < np; ++t) h[t] = (float)((t * 2654435761u) % 1000003u) * 1e-6f;
  CK(hipMemcpy(pin, h, np * 4, hipMemcpyHostToDevice));
  CK(hipMemset(ain, 0, na * 4));
  const int tiles = (g.nz / TZ) * (g.nr / TR);
  pattern_kernel<float, float, 7, true, 0, 2><<<tiles, TZ * TR>>>(g, pin, o2, ain, aout);
  pattern_kernel<float, float, 7, true, 0, 3><<<tiles, TZ * TR>>>(g, pin, o3, ain, aout);
  CK(hipDeviceSynchronize());
  CK(hipGetLastError());
  CK(hipMemcpy(h, o2, np * 4, hipMemcpyDeviceToHost));
  CK(hipMemcpy(h2, o3, np * 4, hipMemcpyDeviceToHost));
  long long bad = 0;
  for (size_t t = 0; t < np; ++t) bad += std::memcmp(&h[t], &h2[t], 4) != 0;
  printf("{\"check\": \"realigned pull against the full pull, C2 FP32\", \"mismatches\": %lld}\n", bad);
  fflush(stdout);
  free(h);
  free(h2);
  CK(hipFree(pin));
  CK(hipFree(o2));
  CK(hipFree(o3));
  CK(hipFree(ain));
  CK(hipFree(aout));
  return bad == 0;
}

int main(int argc, char** argv) {
  CK(hipSetDevice(0));
  if (argc > 1 && std::strcmp(argv[1], "--pingpong") == 0) {
    for (int rep = 0; rep < 3; ++rep) {
      measure_pp("C2 FP32", 2048, 512, 400);
      measure_pp("P-size FP32", 2432, 400, 400);
      measure_pp("C3 FP32", 4096, 1024, 100);
    }
    return 0;
  }
  if (argc > 1 && std::strcmp(argv[1], "--layout") == 0) {
    for (int rep = 0; rep < 2; ++rep) {
      measure_s<2>("C2 FP32", 2048, 512, 400);
      measure_c<1>("C2 FP32", 2048, 512, 400);
      measure_c<0>("C2 FP32", 2048, 512, 400);
      measure_v<1>("C2 FP32", 2048, 512, 400);
      measure_v<0>("C2 FP32", 2048, 512, 400);
      measure_s<2>("C3 FP32", 4096, 1024, 100);
      measure_c<1>("C3 FP32", 4096, 1024, 100);
      measure_c<0>("C3 FP32", 4096, 1024, 100);
      measure_v<1>("C3 FP32", 4096, 1024, 100);
      measure_v<0>("C3 FP32", 4096, 1024, 100);
    }
    return 0;
  }
  if (argc > 1 && std::strcmp(argv[1], "--shift") == 0) {
    if (!realigned_pull_matches()) return 1;
    for (int rep = 0; rep < 2; ++rep) {
      measure_s<0>("C2 FP32", 2048, 512, 400);
      measure_s<1>("C2 FP32", 2048, 512, 400);
      measure_s<2>("C2 FP32", 2048, 512, 400);
      measure_s<3>("C2 FP32", 2048, 512, 400);
      measure_s<4>("C2 FP32", 2048, 512, 400);
      measure_s<0>("C3 FP32", 4096, 1024, 100);
      measure_s<1>("C3 FP32", 4096, 1024, 100);
      measure_s<2>("C3 FP32", 4096, 1024, 100);
      measure_s<3>("C3 FP32", 4096, 1024, 100);
      measure_s<4>("C3 FP32", 4096, 1024, 100);
    }
    return 0;
  }
  if (argc > 1 && std::strcmp(argv[1], "--zmarch") == 0) {
    measure_z<2>("C2 FP32", 2048, 512, 400);
    measure_z<4>("C2 FP32", 2048, 512, 400);
    measure_z<8>("C2 FP32", 2048, 512, 400);
    measure_z<2>("C3 FP32", 4096, 1024, 100);
    measure_z<4>("C3 FP32", 4096, 1024, 100);
    measure_z<8>("C3 FP32", 4096, 1024, 100);
    measure_z<16>("C3 FP32", 4096, 1024, 100);
    return 0;
  }
  if (argc > 1 && std::strcmp(argv[1], "--arith") == 0) {
    measure<float, float, 7, 0>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 0>("C3 FP32", 4096, 1024, 100, false);
    measure<float, float, 7, 8>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 8>("C3 FP32", 4096, 1024, 100, false);
    measure<float, float, 7, 16>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 16>("C3 FP32", 4096, 1024, 100, false);
    measure<float, float, 7, 24>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 24>("C3 FP32", 4096, 1024, 100, false);
    measure<float, float, 7, 32>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 32>("C3 FP32", 4096, 1024, 100, false);
    measure<float, float, 7, 48>("C2 FP32", 2048, 512, 400, false);
    measure<float, float, 7, 48>("C3 FP32", 4096, 1024, 100, false);
    return 0;
  }
  measure<float, float, 7>("C2 FP32", 2048, 512, 400, true);
  measure<float, float, 7>("C3 FP32", 4096, 1024, 100, true);
  measure<_Float16, float, 6>("C3 FP16", 4096, 1024, 100, false);
  measure<double, double, 6>("C3 FP64", 4096, 1024, 50, false);
  return 0;
}
