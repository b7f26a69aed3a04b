/*
 * A plain C caller of the lbm_axi C ABI (include/lbm_axi.h), with no Python
 * and no torch: it states a small porous annulus (the Fig. 3 problem with
 * R* = 2, phi = 0.6, Da = 1e-3, Ra = 1e5, Pr = 1, Ergun F_phi, 64 x 48),
 * creates it on the default device with the library's own stream, takes 101
 * steps (two residual checks), and writes to the file named by argv[1]:
 * u_z, u_r, p, T as [nz][nr] floats, the node classes as [nz][nr] bytes, then
 * res, Nu_i, Nu_o and max |psi| as doubles.  Exit status 0 on success; on a
 * library error it prints lbm_axi_last_error() and exits with 1.
 *
 * Built by the package build (gcc, linked against liblbm_axi.so); run by
 * tests/test_gpu_c_abi.py, which compares its output with the Python binding.
 */
#include <stdio.h>
#include <stdlib.h>

#include "lbm_axi.h"

#define CHECK(call)                                                            \
  do {                                                                         \
    if ((call) != LBM_AXI_OK) {                                                \
      fprintf(stderr, "%s failed: %s\n", #call, lbm_axi_last_error());        \
      return 1;                                                                \
    }                                                                          \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s <output file>\n", argv[0]);
    return 2;
  }
  lbm_axi_params p;
  lbm_axi_default_params(&p);
  p.nr = 64;
  p.nz = 48;
  p.side_rmin = p.side_rmax = p.side_z = LBM_SIDE_WALL;
  p.therm_rmin = p.therm_rmax = LBM_T_FIXED;
  p.therm_z = LBM_T_ADIABATIC;
  p.L = p.nr - 1;          /* wall nodes on the walls */
  p.r0 = p.L / (2.0 - 1.0); /* r_i = L / (R* - 1) */
  p.phi = 0.6;
  p.Da = 1e-3;
  p.F_phi = -1.0;          /* Ergun, Eq. (8) */
  p.Ra = 1e5;
  p.Pr = 1.0;
  p.T_rmin = 1.0;
  p.T_rmax = 0.0;
  p.T_ref = 0.5;
  p.T_init = 0.0;
  p.delta_T = 1.0;
  p.check_interval = 50;

  lbm_axi* h = NULL;
  CHECK(lbm_axi_create(&p, 1, NULL, NULL, NULL, &h));
  CHECK(lbm_axi_step(h, 101));
  const size_t n = (size_t)p.nr * p.nz;
  float* f = (float*)malloc(sizeof(float) * 4 * n);
  unsigned char* mask = (unsigned char*)malloc(n);
  if (!f || !mask) return 1;
  CHECK(lbm_axi_macros(h, 0, f, f + n, f + 2 * n, f + 3 * n, mask, 0));
  double out[4];
  int32_t status;
  CHECK(lbm_axi_residual(h, &out[0], &out[1], &out[2], &status));
  CHECK(lbm_axi_stream_function(h, 0, NULL, &out[3], 0));
  lbm_axi_destroy(h);

  FILE* fp = fopen(argv[1], "wb");
  if (!fp) return 1;
  int ok = fwrite(f, sizeof(float), 4 * n, fp) == 4 * n && fwrite(mask, 1, n, fp) == n &&
           fwrite(out, sizeof(double), 4, fp) == 4;
  ok = (fclose(fp) == 0) && ok;
  free(f);
  free(mask);
  printf("c_abi_driver: %dx%d, 101 steps, res %.3e Nu_i %.6f Nu_o %.6f max|psi| %.6e\n", p.nr, p.nz,
         out[0], out[1], out[2], out[3]);
  return ok ? 0 : 1;
}
