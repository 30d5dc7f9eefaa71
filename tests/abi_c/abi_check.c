/* Plain-C caller of libhwenou.so: device memory from hipMalloc, no Python.
 * Checks, through the C-ABI alone, that hwenou_advance keeps constant states
 * (1D and 2D Euler, FP64 and mixed, periodic and reflective sides where the
 * state is at rest) to round-off, reports t and the step count, and that
 * hwenou_stage and hwenou_create reject bad arguments.  Exit status 0 on
 * success.  Test infrastructure: built by __graft_entry__.build(), run by
 * tests/test_gpu_abi_c.py. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hwenou.h"

static int fail(const char* what, int rc) {
  fprintf(stderr, "FAIL %s: %s (%d)\n", what, hwenou_strerror(rc), rc);
  return 1;
}

/* Uniform Euler state (rho, velocity vel[dim], p) on nx*ny cells. */
static int run_constant(int dim, int precision, int nx, int ny, int bc, const double* vel) {
  const int nc = dim + 2;
  const size_t n = (size_t)nx * ny;
  const size_t melem = precision == HWENOU_MIXED ? sizeof(float) : sizeof(double);
  double rho = 1.3, p = 0.9, q2 = 0.0;
  for (int d = 0; d < dim; ++d) q2 += vel[d] * vel[d];
  double* u = (double*)malloc(nc * n * sizeof(double));
  for (size_t c = 0; c < n; ++c) {
    u[c] = rho;
    for (int d = 0; d < dim; ++d) u[(1 + d) * n + c] = rho * vel[d];
    u[(nc - 1) * n + c] = p / 0.4 + 0.5 * rho * q2;
  }
  double* du = NULL;
  void* dm = NULL;
  if (hipMalloc((void**)&du, nc * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&dm, dim * nc * n * melem) != hipSuccess)
    return fail("hipMalloc", HWENOU_ENOMEM);
  hipMemcpy(du, u, nc * n * sizeof(double), hipMemcpyHostToDevice);
  hipMemset(dm, 0, dim * nc * n * melem);

  hwenou_desc desc = {dim, HWENOU_EQ_EULER, precision, HWENOU_CHAR_SPLIT,
                      HWENOU_W_SCALE_INVARIANT, {0.0, 0.0}, 1.4, 1.0 / 400.0, 1e-10};
  hwenou_inst inst = {nx, ny, 0.0, 1.0, 0.0, 1.0, {bc, bc, bc, bc}, 0};
  hwenou_handle* h = NULL;
  int rc = hwenou_create(&desc, 1, &inst, NULL, &h);
  if (rc) return fail("hwenou_create", rc);
  double t = 0.0;
  int steps = 0;
  rc = hwenou_advance(h, du, dm, 0.6, 1e30, 20, &t, &steps);
  if (rc) return fail("hwenou_advance", rc);
  if (steps != 20 || !(t > 0.0)) {
    fprintf(stderr, "FAIL steps %d t %g\n", steps, t);
    return 1;
  }
  double* out = (double*)malloc(nc * n * sizeof(double));
  hipMemcpy(out, du, nc * n * sizeof(double), hipMemcpyDeviceToHost);
  double err = 0.0, scale = 0.0;
  for (size_t i = 0; i < nc * n; ++i) {
    err = fmax(err, fabs(out[i] - u[i]));
    scale = fmax(scale, fabs(u[i]));
  }
  /* bad stage arguments: s out of range; aliased input and output; stage 1
   * with no stage 0 recorded (hwenou_advance clears the record) */
  double *ddt = NULL, *dal = NULL, *du2 = NULL;
  void* dm2 = NULL;
  hipMalloc((void**)&ddt, sizeof(double));
  hipMalloc((void**)&dal, 2 * sizeof(double));
  hipMalloc((void**)&du2, nc * n * sizeof(double));
  hipMalloc(&dm2, dim * nc * n * melem);
  if (hwenou_stage(h, 3, ddt, dal, du, dm, du2, dm2) != HWENOU_EINVAL)
    return fail("stage 3 accepted", HWENOU_OK);
  if (hwenou_stage(h, 0, ddt, dal, du, dm, du, dm2) != HWENOU_EINVAL)
    return fail("aliased stage accepted", HWENOU_OK);
  if (hwenou_stage(h, 1, ddt, dal, du, dm, du2, dm2) != HWENOU_EINVAL)
    return fail("stage 1 before stage 0 accepted", HWENOU_OK);
  printf("dim %d precision %d bc %d: %d steps to t = %.6f, max |change| / scale = %.2e\n", dim,
         precision, bc, steps, t, err / scale);
  hwenou_destroy(h);
  hipFree(du);
  hipFree(dm);
  hipFree(ddt);
  hipFree(dal);
  hipFree(du2);
  hipFree(dm2);
  free(u);
  free(out);
  if (!(err <= 1e-13 * scale)) {
    fprintf(stderr, "FAIL constant state changed by %g\n", err / scale);
    return 1;
  }
  return 0;
}

int main(void) {
  const double v1[1] = {0.3}, v2[2] = {0.3, -0.2}, rest[2] = {0.0, 0.0};
  int bad = 0;
  bad |= run_constant(1, HWENOU_FP64, 300, 1, HWENOU_BC_PERIODIC, v1);
  bad |= run_constant(1, HWENOU_MIXED, 300, 1, HWENOU_BC_PERIODIC, v1);
  bad |= run_constant(2, HWENOU_FP64, 70, 45, HWENOU_BC_PERIODIC, v2);
  bad |= run_constant(2, HWENOU_MIXED, 70, 45, HWENOU_BC_TRANSMISSIVE, v2);
  bad |= run_constant(2, HWENOU_FP64, 70, 45, HWENOU_BC_REFLECTIVE, rest);
  /* hwenou_create argument checks */
  hwenou_desc desc = {2, HWENOU_EQ_BURGERS, HWENOU_FP64, HWENOU_CHAR_SPLIT,
                      HWENOU_W_SCALE_INVARIANT, {0.0, 0.0}, 1.4, 1.0 / 400.0, 1e-10};
  hwenou_inst inst = {10, 10, 0.0, 1.0, 0.0, 1.0, {HWENOU_BC_REFLECTIVE, 0, 0, 0}, 0};
  hwenou_handle* h = NULL;
  if (hwenou_create(&desc, 1, &inst, NULL, &h) != HWENOU_EINVAL || h != NULL) {
    fprintf(stderr, "FAIL reflective Burgers accepted\n");
    bad = 1;
  }
  printf(bad ? "abi_check: FAILED\n" : "abi_check: ok\n");
  return bad;
}
