/* The C ABI used from plain C, with no Python: C1's grid and driver (256 x 64, dz = 0.05,
 * tau = 0.8, n_b = 0.01, sigma = 0.5, no density noise) in the storage given on the command line,
 * `steps` steps, then the FP64 diagnostics and the on-axis E_z at three columns as one JSON line.
 * Usage: lbm_c_run <steps> <storage 0..3>.  Exit status 0 on success, 1 on any library or HIP
 * error (the message goes to stderr). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lbmpwfa.h"

static int check(int rc, const char* what) {
  if (rc != LBM_OK) fprintf(stderr, "%s: %d %s\n", what, rc, lbm_last_error());
  return rc != LBM_OK;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <steps> <storage>\n", argv[0]);
    return 1;
  }
  const long long steps = atoll(argv[1]);
  lbm_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.nz = 256;
  cfg.nr = 64;
  cfg.dz = cfg.dr = 0.05;
  cfg.c_dt_over_dz = 0.2;
  cfg.tau = 0.8;
  cfg.storage = atoi(argv[2]);
  cfg.fields_on = 1;
  cfg.cyl_on = 1;
  cfg.n0 = 1.0;
  cfg.ramp_len = 1.0;
  cfg.nb = 0.01;
  cfg.sigma_z = cfg.sigma_r = 0.5;
  cfg.zd0 = 4.0;
  cfg.n_floor = 1e-10;
  cfg.trt_magic = 0.25;

  size_t bytes = 0;
  if (check(lbm_workspace_bytes(&cfg, &bytes), "lbm_workspace_bytes")) return 1;
  void* ws = NULL;
  hipStream_t st;
  if (hipMalloc(&ws, bytes) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
    fprintf(stderr, "HIP allocation failed\n");
    return 1;
  }
  lbm_ctx* ctx = NULL;
  int bad = check(lbm_init(&cfg, NULL, NULL, ws, bytes, st, &ctx), "lbm_init");
  lbm_diag d;
  double* f = (double*)malloc(3 * sizeof(double) * cfg.nz * cfg.nr);
  if (!bad) bad = check(lbm_step(ctx, steps), "lbm_step");
  if (!bad) bad = check(lbm_diagnostics(ctx, &d), "lbm_diagnostics");
  if (!bad) bad = check(lbm_fields(ctx, f, LBM_F64, 0), "lbm_fields");
  if (!bad)
    printf("{\"step\": %lld, \"shifts\": %lld, \"charge\": %.17g, \"field_energy\": %.17g, "
           "\"gauss_max\": %.17g, \"umax\": %.17g, \"nonfinite\": %d, \"ez_axis\": [%.17g, %.17g, %.17g]}\n",
           (long long)d.step, (long long)d.shifts, d.charge, d.field_energy, d.gauss_max, d.umax, d.nonfinite,
           f[40], f[80], f[120]);
  free(f);
  if (ctx) bad |= check(lbm_destroy(ctx), "lbm_destroy");
  hipStreamDestroy(st);
  hipFree(ws);
  return bad;
}
