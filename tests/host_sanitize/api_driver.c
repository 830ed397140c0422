/* Drives the host runtime's checks without a GPU (built with the host
 * sanitizers): invalid parameters, the addressable-pool limit, planning of a
 * padded and of a very large lattice, a refusing and a counting allocator,
 * NULL handles and batches.  Exit status 0 when every call returned what it
 * should. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"
#include "lbm_batch.h"

static int failures = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "line %d: %s failed\n", __LINE__, #cond);   \
      failures++;                                                 \
    }                                                             \
  } while (0)

static lbm_params base(int nx, int ny, int nz) {
  lbm_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx, p.ny = ny, p.nz = nz, p.block = 16, p.ncomp = 2, p.shell_width = 2;
  for (int f = 0; f < 6; ++f) p.bc[f] = LBM_BC_WALL;
  p.bc[0] = LBM_BC_INLET;
  p.bc[1] = LBM_BC_OUTLET;
  p.tau[0] = p.tau[1] = 1.0;
  p.eos_a = 2.0 / 49.0, p.eos_b = 2.0 / 21.0, p.eos_R = 1.0, p.eos_omega = 0.344, p.T_over_Tc = 0.7;
  p.g[0][0] = p.g[1][1] = -1.0;
  p.g[0][1] = p.g[1][0] = 0.1 / 6.0;
  p.beta = 1.16;
  p.inlet_rho[0] = 6.5, p.inlet_rho[1] = 0.1, p.inlet_u[0] = 0.02;
  p.bg_rho[0] = p.bg_rho[1] = 0.38;
  return p;
}

static int allocs = 0;
static void* refuse(size_t n, void* ctx) { (void)n; (void)ctx; allocs++; return NULL; }
static void release(void* p, void* ctx) { (void)ctx; free(p); }

int main(void) {
  lbm_t* h = NULL;
  int64_t bytes = 0;
  /* invalid parameters are refused before any device call */
  lbm_params p = base(48, 32, 32);
  p.tau[1] = 0.5;
  EXPECT(lbm_create(&p, NULL, NULL, &h) == LBM_EINVAL && h == NULL);
  EXPECT(strstr(lbm_last_error(NULL), "tau") != NULL);
  p = base(48, 32, 32);
  p.bc[0] = p.bc[1] = LBM_BC_PERIODIC;
  p.nx = 40;
  EXPECT(lbm_create(&p, NULL, NULL, &h) == LBM_EINVAL);
  p = base(48, 32, 32);
  p.pool_blocks = 65536; /* beyond the two-component FP32 limit; within the FP16 one */
  EXPECT(lbm_create(&p, NULL, NULL, &h) == LBM_EINVAL);
  p.store = LBM_STORE_F16DEV;
  EXPECT(lbm_plan_bytes(&p, NULL, &bytes) == LBM_OK && bytes > 0);
  EXPECT(lbm_create(NULL, NULL, NULL, &h) == LBM_EINVAL);
  EXPECT(lbm_plan_bytes(&p, NULL, NULL) == LBM_EINVAL);
  /* planning: a padded lattice with a solid array, and a lattice too large for the FP32 store */
  p = base(40, 24, 56);
  unsigned char* solid = calloc((size_t)40 * 24 * 56, 1);
  for (int k = 0; k < 40 * 24 * 56; k += 7) solid[k] = 1;
  EXPECT(lbm_plan_bytes(&p, solid, &bytes) == LBM_OK && bytes > 0);
  free(solid);
  p = base(1024, 1024, 512);
  EXPECT(lbm_plan_bytes(&p, NULL, &bytes) == LBM_EINVAL);
  /* a refusing allocator: LBM_ENOMEM, nothing leaked */
  p = base(48, 32, 32);
  lbm_allocator a = {refuse, release, NULL};
  EXPECT(lbm_create(&p, NULL, &a, &h) == LBM_ENOMEM && h == NULL && allocs >= 1);
  lbm_allocator half = {NULL, release, NULL};
  EXPECT(lbm_create(&p, NULL, &half, &h) == LBM_EINVAL);
  /* no device: lbm_create fails cleanly with the library's own allocation */
  int rc = lbm_create(&p, NULL, NULL, &h);
  EXPECT(rc != LBM_OK && h == NULL);
  /* NULL handles and batches */
  EXPECT(lbm_step(NULL, 1) == LBM_EINVAL);
  EXPECT(lbm_set_split(NULL, 8, 64) == LBM_EINVAL);
  EXPECT(lbm_moments_noalloc(NULL, NULL, NULL, NULL, NULL) == LBM_EINVAL);
  EXPECT(lbm_destroy(NULL) == LBM_OK);
  lbm_batch_t* b = NULL;
  EXPECT(lbm_batch_create(NULL, 1, &b) == LBM_EINVAL);
  lbm_t* hs[2] = {NULL, NULL};
  EXPECT(lbm_batch_create(hs, 2, &b) == LBM_EINVAL);
  EXPECT(lbm_batch_schedule(NULL, 1) == LBM_EINVAL);
  EXPECT(lbm_batch_destroy(NULL) == LBM_OK);
  printf("api driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
