/*
 * A plain C caller of libtopoguard.so: only include/topoguard.h and the HIP
 * runtime's allocation calls, no Python and no torch.
 *
 *   guarded_solve host  nx ny nz            grid facts only (no device)
 *   guarded_solve gpu   nx ny nz rho.bin    the guarded floor policy on the
 *                                          density field in rho.bin (nx*ny*nz
 *                                          doubles, x fastest), default stream
 *
 * Prints one "key value" pair per line.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "topoguard.h"

#define TG(call)                                                              \
  do {                                                                        \
    int rc_ = (call);                                                         \
    if (rc_ != TG_OK) {                                                       \
      fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, tg_last_error());   \
      return 1;                                                               \
    }                                                                         \
  } while (0)
#define HIPC(call)                                                            \
  do {                                                                        \
    if ((call) != hipSuccess) {                                               \
      fprintf(stderr, "%s failed\n", #call);                                  \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 5) {
    fprintf(stderr, "usage: %s host|gpu nx ny nz [rho.bin]\n", argv[0]);
    return 2;
  }
  const int gpu = strcmp(argv[1], "gpu") == 0;
  const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
  tg_grid* g = NULL;
  TG(tg_setup_grid(nx, ny, nz, 1.0, 0.3, NULL, &g));
  tg_grid_info info;
  TG(tg_get_grid_info(g, &info));
  printf("n_elem %lld\nn_dof %lld\nn_free %lld\nn_levels %d\n", (long long)info.n_elem, (long long)info.n_dof,
         (long long)info.n_free, info.n_levels);
  const size_t nd = (size_t)info.n_dof, ne = (size_t)info.n_elem;
  double* f = (double*)malloc(nd * sizeof(double));
  TG(tg_edge_load(g, f));
  double fz = 0.0;
  for (size_t i = 2; i < nd; i += 3) fz += f[i];
  printf("load_z %.17g\n", fz);
  double ke[576];
  TG(tg_get_ke(g, ke));
  printf("ke_00 %.17g\n", ke[0]);
  if (!gpu) {
    free(f);
    tg_destroy(g);
    return 0;
  }
  if (argc < 6) return 2;
  double* rho = (double*)malloc(ne * sizeof(double));
  FILE* fh = fopen(argv[5], "rb");
  if (!fh || fread(rho, sizeof(double), ne, fh) != ne) {
    fprintf(stderr, "cannot read %s\n", argv[5]);
    return 1;
  }
  fclose(fh);
  size_t wb = 0;
  TG(tg_workspace_bytes(g, 100, &wb));
  void* ws = NULL;
  double *rho_d = NULL, *f_d = NULL, *u_d = NULL;
  HIPC(hipMalloc(&ws, wb));
  HIPC(hipMalloc((void**)&rho_d, ne * sizeof(double)));
  HIPC(hipMalloc((void**)&f_d, nd * sizeof(double)));
  HIPC(hipMalloc((void**)&u_d, nd * sizeof(double)));
  HIPC(hipMemcpy(rho_d, rho, ne * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(f_d, f, nd * sizeof(double), hipMemcpyHostToDevice));
  TG(tg_bind_workspace(g, ws, wb, 100));
  tg_policy pol;
  tg_default_policy(&pol);
  tg_policy_result out;
  TG(tg_select_floor(g, rho_d, f_d, &pol, u_d, &out, NULL));
  printf("rung %d\nfloor %.17g\nk0 %d\nr50 %.17g\nr100 %.17g\nattempts %d\n", out.rung, out.floor, out.k0, out.r50,
         out.r100, out.n_attempts);
  for (int a = 0; a < out.n_attempts; ++a)
    printf("attempt %d %d %d %.17g\n", out.attempts[a].rung, out.attempts[a].iterations, out.attempts[a].accepted,
           out.attempts[a].true_eta);
  double eta = -1.0, comp = 0.0;
  if (out.rung >= 0) {
    TG(tg_true_residual(g, f_d, u_d, &eta, NULL));
    TG(tg_compliance_sensitivity(g, NULL, pol.p, out.floor, f_d, u_d, NULL, NULL, &comp, NULL));
  }
  printf("true_eta %.17g\ncompliance %.17g\n", eta, comp);
  tg_destroy(g);
  hipFree(ws);
  hipFree(rho_d);
  hipFree(f_d);
  hipFree(u_d);
  free(rho);
  free(f);
  return 0;
}
