// Memory-pattern ceiling of the FP32 step: the rate the chip sustains for the step's own access
// pattern when no arithmetic is attached to it, beside a plain float4 copy of the same bytes.
//
// The FP32 step moves 272 B per site: the 27 populations pulled from the neighbours along the
// lattice velocities (three D2Q9 lattices, pull offsets clamped to the grid), the 7 auxiliary words
// of the site (3 moments, E_z, E_r, B_theta and the residual word) read, and all 34 written back at
// the site.  pattern_kernel does exactly that with one site per thread on 64 x 4 tiles (the step's
// tile), in the step's layout (planes 256 bytes longer than their rows, so that the 34 streams of
// a site do not start on the same memory channels) and with the step's XCD-aware tile order; its
// rate bounds what any arrangement of the step's arithmetic around that pattern can reach.  The
// same kernel on unpadded planes in plain block order, and copy_kernel moving the same number of
// bytes as one contiguous float4 stream, are measured beside it.
//
// Standalone program (not part of the library): prints one JSON line per measurement.  Every index
// is clamped into the arrays, and the grids are whole multiples of the tile.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
      exit(1);                                                                             \
    }                                                                                      \
  } while (0)

namespace {

constexpr int TZ = 64, TR = 4, NPOP = 27, NAUX = 7;

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

template <bool XCD>
__global__ __launch_bounds__(TZ * TR) void pattern_kernel(Grid g, const float* __restrict__ pin,
                                                          float* __restrict__ pout, const float* __restrict__ ain,
                                                          float* __restrict__ aout) {
  const int gx = g.nz / TZ;
  const int tile = XCD ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
  const int i = (tile % gx) * TZ + threadIdx.x % TZ;
  const int j = (tile / gx) * TR + threadIdx.x / TZ;
  float f[NPOP], a[NAUX];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const long long off = (long long)clampi(j - cr(q), g.nr) * g.nz + clampi(i - cz(q), g.nz);
#pragma unroll
    for (int l = 0; l < 3; ++l) f[9 * l + q] = pin[(9 * l + q) * g.plane + off];
  }
  const long long o = (long long)j * g.nz + i;
#pragma unroll
  for (int c = 0; c < NAUX; ++c) a[c] = ain[c * g.plane + o];
  // a dependence of every output on every input keeps all loads; no other arithmetic
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < NPOP; ++c) s += f[c];
#pragma unroll
  for (int c = 0; c < NPOP; ++c) pout[c * g.plane + o] = f[c] + 1e-7f * s;
#pragma unroll
  for (int c = 0; c < NAUX; ++c) aout[c * g.plane + o] = a[c] + 1e-7f * s;
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

int main() {
  CK(hipSetDevice(0));
  const int sizes[2][2] = {{2048, 512}, {4096, 1024}};   // the C2 and C3 grids
  const char* names[2] = {"C2", "C3"};
  for (int w = 0; w < 2; ++w) {
    Grid g;
    g.nz = sizes[w][0];
    g.nr = sizes[w][1];
    g.plane = (long long)g.nz * g.nr + 64;   // the step's pad: 256 bytes of FP32
    Grid gu = g;
    gu.plane = (long long)g.nz * g.nr;       // unpadded
    const long long sites = (long long)g.nz * g.nr;
    const double bytes = 2.0 * 4.0 * (NPOP + NAUX) * (double)sites;   // 272 B per site
    float *pin, *pout, *ain, *aout;
    CK(hipMalloc(&pin, NPOP * g.plane * sizeof(float)));
    CK(hipMalloc(&pout, NPOP * g.plane * sizeof(float)));
    CK(hipMalloc(&ain, NAUX * g.plane * sizeof(float)));
    CK(hipMalloc(&aout, NAUX * g.plane * sizeof(float)));
    CK(hipMemset(pin, 0, NPOP * g.plane * sizeof(float)));
    CK(hipMemset(ain, 0, NAUX * g.plane * sizeof(float)));
    // the copy moves the same bytes: the 27 planes of pin to pout, then the 7 of ain to aout
    const long long n4p = NPOP * g.plane / 4, n4a = NAUX * g.plane / 4;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int iters = w == 0 ? 400 : 100;
    const int tiles = (g.nz / TZ) * (g.nr / TR);
    const char* kname[3] = {"step access pattern (pull, 64x4 tiles, step layout and tile order)",
                            "same pattern, unpadded planes, plain block order", "float4 copy, same bytes"};
    for (int k = 0; k < 3; ++k) {
      auto launch = [&] {
        if (k == 0) {
          pattern_kernel<true><<<tiles, TZ * TR>>>(g, pin, pout, ain, aout);
        } else if (k == 1) {
          pattern_kernel<false><<<tiles, TZ * TR>>>(gu, pin, pout, ain, aout);
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
      printf("{\"workload\": \"%s %dx%d\", \"kernel\": \"%s\", \"bytes_per_site\": 272, \"us\": %.2f, "
             "\"GBps\": %.1f, \"frac_of_8TBps\": %.4f}\n",
             names[w], g.nz, g.nr, kname[k], us, bytes / us / 1e3, bytes / us / 1e3 / 8000.0);
      fflush(stdout);
    }
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    CK(hipFree(pin));
    CK(hipFree(pout));
    CK(hipFree(ain));
    CK(hipFree(aout));
  }
  return 0;
}
