/*
 * A client of the library's C ABI alone (include/lbf.h): device memory and
 * the stream come from the HIP runtime, there is no Python.  It runs one
 * thermal lattice for a number of steps with the default schedule or the
 * fused two-step pass, checks it with lb_check, and writes the populations
 * (float32, q planes of nz * ny * nx values) to a file.
 *
 * usage: lb_client d3q19|d2q9 nx ny nz f32|f16|bf16 steps fused(0|1) out.bin
 * Parameters: rho0 = 1, kT = 1e-4, gamma_bulk = 0.5, gamma_shear = 0.8,
 * kinetic rates 0, seed 1234, thermal start at t = 0.
 */
#include <hip/hip_runtime_api.h>
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbf.h"

#define HIP_OR_FAIL(x)                                                              \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      fprintf(stderr, "lb_client: %s: %s\n", #x, hipGetErrorString(e_));            \
      return 2;                                                                     \
    }                                                                               \
  } while (0)
#define LB_OR_FAIL(x)                                                               \
  do {                                                                              \
    int rc_ = (x);                                                                  \
    if (rc_ != LB_OK) {                                                             \
      fprintf(stderr, "lb_client: %s: %s (%s)\n", #x, lb_strerror(rc_), lb_last_error()); \
      return 3;                                                                     \
    }                                                                               \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s d3q19|d2q9 nx ny nz f32|f16|bf16 steps fused(0|1) out.bin\n", argv[0]);
    return 1;
  }
  lb_params p;
  memset(&p, 0, sizeof(p));
  p.lattice = strcmp(argv[1], "d2q9") == 0 ? LB_D2Q9 : LB_D3Q19;
  p.nx = atoi(argv[2]);
  p.ny = atoi(argv[3]);
  p.nz = atoi(argv[4]);
  p.storage = strcmp(argv[5], "f16") == 0 ? LB_F16 : (strcmp(argv[5], "bf16") == 0 ? LB_BF16 : LB_F32);
  p.rho0 = 1.0;
  p.kT = 1e-4;
  p.gamma_bulk = 0.5;
  p.gamma_shear = 0.8;
  p.gamma_odd = 0.0;
  p.gamma_even = 0.0;
  p.seed = 1234;
  p.thermal_modes = LB_THERMAL_ALL;
  const int64_t steps = atoll(argv[6]);
  const int fused = atoi(argv[7]);

  const size_t q = p.lattice == LB_D2Q9 ? 9 : 19;
  const size_t es = p.storage == LB_F32 ? 4 : 2;
  const size_t nsites = (size_t)p.nx * (size_t)p.ny * (size_t)p.nz;

  void* d_state = NULL;
  float* d_pops = NULL;
  hipStream_t stream;
  HIP_OR_FAIL(hipMalloc(&d_state, q * nsites * es));
  HIP_OR_FAIL(hipMalloc((void**)&d_pops, q * nsites * sizeof(float)));
  HIP_OR_FAIL(hipStreamCreate(&stream));

  lb_ctx* ctx = NULL;
  LB_OR_FAIL(lb_init(&p, d_state, (void*)stream, LB_INIT_THERMAL, NULL, 0, &ctx));
  if (fused) {
    lb_schedule s;
    LB_OR_FAIL(lb_get_schedule(ctx, &s));
    s.fused = 1;
    LB_OR_FAIL(lb_set_schedule(ctx, &s));
  }
  LB_OR_FAIL(lb_step(ctx, steps));
  int64_t n_bad = -1;
  double sums[4] = {0, 0, 0, 0};
  LB_OR_FAIL(lb_check(ctx, &n_bad, sums));
  LB_OR_FAIL(lb_populations(ctx, d_pops));
  HIP_OR_FAIL(hipStreamSynchronize(stream));

  float* h = (float*)malloc(q * nsites * sizeof(float));
  if (!h) return 4;
  HIP_OR_FAIL(hipMemcpy(h, d_pops, q * nsites * sizeof(float), hipMemcpyDeviceToHost));
  FILE* f = fopen(argv[8], "wb");
  if (!f || fwrite(h, sizeof(float), q * nsites, f) != q * nsites) {
    fprintf(stderr, "lb_client: cannot write %s\n", argv[8]);
    return 5;
  }
  fclose(f);
  printf("lb_client: %s %dx%dx%d %s fused=%d t=%" PRId64 " bad=%" PRId64 " sums=%.17g %.17g %.17g %.17g\n",
         argv[1], p.nx, p.ny, p.nz, argv[5], fused, lb_step_count(ctx), n_bad, sums[0], sums[1], sums[2], sums[3]);
  free(h);
  lb_destroy(ctx);
  HIP_OR_FAIL(hipFree(d_pops));
  HIP_OR_FAIL(hipFree(d_state));
  HIP_OR_FAIL(hipStreamDestroy(stream));
  return 0;
}
