/* One solve through the C ABI from C: the 32^3 one-bump workload (charge
 * (1 - rho^2)^4 of radius 0.35 at the centre, 8^3-cell patches, alpha 3,
 * beta 6, P 4, L19, float64 convolutions, DGF half-width 64), device
 * buffers from the HIP runtime.  The charge is sampled here, or read from
 * the file named by argv[1] (float64, (N+1)^3, C order) when given; phi is
 * written to argv[2] when given.  Prints the relative max-norm error against
 * the closed-form potential.  Built and run by tests/test_gpu_c_api.py. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mlc.h"

#define N 32

static double bump_charge(double r) { double u = 1.0 - r * r; return r < 1.0 ? u * u * u * u : 0.0; }
/* the potential of the unit-weight bump, in units of R^2 (Delta phi = f) */
static double bump_potential(double r) {
  if (r < 1.0) {
    double r2 = r * r;
    return r2 / 6 - r2 * r2 / 5 + r2 * r2 * r2 / 7 - r2 * r2 * r2 * r2 / 18 + r2 * r2 * r2 * r2 * r2 / 110 - 0.1;
  }
  return -128.0 / (3465.0 * r);
}

int main(int argc, char** argv) {
  const size_t nodes = (size_t)(N + 1) * (N + 1) * (N + 1);
  const double R = 0.35, h = 1.0 / N;
  double* f = malloc(nodes * sizeof(double));
  double* phi = malloc(nodes * sizeof(double));
  double* ex = malloc(nodes * sizeof(double));
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N; ++j)
      for (int k = 0; k <= N; ++k) {
        double x = i * h - 0.5, y = j * h - 0.5, z = k * h - 0.5;
        double r = sqrt(x * x + y * y + z * z) / R;
        size_t g = ((size_t)i * (N + 1) + j) * (N + 1) + k;
        f[g] = bump_charge(r);
        ex[g] = R * R * bump_potential(r);
      }
  if (argc > 1) {
    FILE* fp = fopen(argv[1], "rb");
    if (!fp || fread(f, sizeof(double), nodes, fp) != nodes) { printf("read failed\n"); return 2; }
    fclose(fp);
  }
  mlc_problem p;
  memset(&p, 0, sizeof p);
  p.n_cells = N; p.h = h; p.patch = 8; p.alpha = 3.0; p.beta = 6.0; p.P = 4; p.Q = 4;
  p.conv_precision = MLC_CONV_FP64; p.dgf_half_width = 64;
  mlc_context* ctx = NULL;
  mlc_plan* plan = NULL;
  char msg[256];
  if (mlc_context_create(0, 0, &ctx) != MLC_OK) { mlc_last_error(NULL, msg, sizeof msg); printf("context: %s\n", msg); return 2; }
  if (mlc_plan_create(ctx, &p, &plan) != MLC_OK) { mlc_last_error(ctx, msg, sizeof msg); printf("plan: %s\n", msg); return 2; }
  size_t ws_bytes = 0;
  mlc_plan_workspace_bytes(plan, &ws_bytes);
  void *df = NULL, *dphi = NULL, *ws = NULL;
  if (hipMalloc(&df, nodes * sizeof(double)) != hipSuccess || hipMalloc(&dphi, nodes * sizeof(double)) != hipSuccess ||
      hipMalloc(&ws, ws_bytes) != hipSuccess) { printf("allocation failed\n"); return 2; }
  hipMemcpy(df, f, nodes * sizeof(double), hipMemcpyHostToDevice);
  mlc_status s = mlc_solve(plan, df, dphi, ws, ws_bytes, NULL);
  if (s != MLC_OK) { mlc_last_error(ctx, msg, sizeof msg); printf("solve: %s\n", msg); return 2; }
  if (hipDeviceSynchronize() != hipSuccess) { printf("synchronize failed\n"); return 2; }
  hipMemcpy(phi, dphi, nodes * sizeof(double), hipMemcpyDeviceToHost);
  double emax = 0.0, pmax = 0.0;
  for (size_t g = 0; g < nodes; ++g) {
    emax = fmax(emax, fabs(phi[g] - ex[g]));
    pmax = fmax(pmax, fabs(ex[g]));
  }
  printf("relative max error against the closed form: %.3e\n", emax / pmax);
  if (argc > 2) {
    FILE* fp = fopen(argv[2], "wb");
    if (!fp || fwrite(phi, sizeof(double), nodes, fp) != nodes) { printf("write failed\n"); return 2; }
    fclose(fp);
  }
  hipFree(df); hipFree(dphi); hipFree(ws);
  mlc_plan_destroy(plan);
  mlc_context_destroy(ctx);
  free(f); free(phi); free(ex);
  return emax / pmax < 1e-3 ? 0 : 1;
}
