/* Drives the FP64 oracle (built with the host sanitizers) through the calls
 * the tests use: a periodic droplet, a progressive porous injection on a
 * lattice with uneven edges (partial blocks), moments, the debug fields, the
 * trace and the counters.  Exit status 0 when the runs stay finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nx, ny, nz, ncomp, block, shell_width, bc[6];
  double tau[2], eos_a, eos_b, eos_R, eos_omega, T_over_Tc, g[2][2], beta, S, body[2][3];
  double inlet_rho[2], inlet_u[3], bg_rho[2];
} orc_params;
typedef struct orc_sim orc_sim;
orc_sim* orc_create(const orc_params*, const uint8_t*, const double*, const double*, const uint8_t*);
void orc_destroy(orc_sim*);
int orc_step(orc_sim*, int32_t);
void orc_moments(orc_sim*, double*, double*, double*, uint8_t*);
void orc_debug_fields(orc_sim*, double*, double*);
void orc_counters(orc_sim*, int64_t*);
void orc_trace(orc_sim*, int32_t*);

static orc_params fluid(int nx, int ny, int nz, int periodic) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx, p.ny = ny, p.nz = nz, p.ncomp = 2, p.block = 16, p.shell_width = 2;
  for (int f = 0; f < 6; ++f) p.bc[f] = periodic ? 0 : 1;
  if (!periodic) p.bc[0] = 2, p.bc[1] = 3;
  p.tau[0] = p.tau[1] = 1.0;
  p.eos_a = 2.0 / 49.0, p.eos_b = 2.0 / 21.0, p.eos_R = 1.0, p.eos_omega = 0.344, p.T_over_Tc = 0.7;
  p.g[0][0] = p.g[1][1] = -1.0;
  p.g[0][1] = p.g[1][0] = 0.1 / 6.0;
  p.beta = 1.16;
  p.inlet_rho[0] = 6.5, p.inlet_rho[1] = 0.1, p.inlet_u[0] = 0.02;
  p.bg_rho[0] = periodic ? 0.0556 : 0.38, p.bg_rho[1] = periodic ? 0.1 : 0.38;
  return p;
}

static int run(orc_params p, const uint8_t* solid, const double* rho0, const uint8_t* act, int steps) {
  const int64_t N = (int64_t)p.nx * p.ny * p.nz;
  orc_sim* s = orc_create(&p, solid, rho0, NULL, act);
  if (!s) return 1;
  orc_step(s, steps);
  double* rho = malloc(sizeof(double) * 2 * N);
  double* u = malloc(sizeof(double) * 6 * N);
  double* um = malloc(sizeof(double) * 3 * N);
  uint8_t* a = malloc(N);
  double* psi = malloc(sizeof(double) * 2 * N);
  double* F = malloc(sizeof(double) * 6 * N);
  orc_moments(s, rho, u, um, a);
  orc_debug_fields(s, psi, F);
  int64_t c[5];
  orc_counters(s, c);
  int32_t* tr = malloc(sizeof(int32_t) * 2 * (c[4] + 1));
  orc_trace(s, tr);
  int bad = 0;
  for (int64_t k = 0; k < 2 * N; ++k) bad |= !isfinite(rho[k]) || !isfinite(psi[k]);
  printf("oracle %dx%dx%d: %d steps, leak %lld, trace %lld\n", p.nx, p.ny, p.nz, steps, (long long)c[1],
         (long long)c[4]);
  free(rho), free(u), free(um), free(a), free(psi), free(F), free(tr);
  orc_destroy(s);
  return bad;
}

int main(void) {
  int bad = 0;
  /* periodic droplet, 16^3 */
  orc_params p = fluid(16, 16, 16, 1);
  double* rho0 = malloc(sizeof(double) * 2 * 4096);
  for (int k = 0; k < 4096; ++k) {
    const int x = k % 16, y = (k / 16) % 16, z = k / 256;
    const double d = sqrt((x - 8.0) * (x - 8.0) + (y - 8.0) * (y - 8.0) + (z - 8.0) * (z - 8.0));
    rho0[k] = 0.0556 + (8.08 - 0.0556) * 0.5 * (1.0 - tanh((d - 4.0) / 2.0));
    rho0[4096 + k] = 0.1;
  }
  bad |= run(p, NULL, rho0, NULL, 20);
  free(rho0);
  /* progressive porous injection on 40 x 24 x 56 (uneven edges: partial blocks) */
  p = fluid(40, 24, 56, 0);
  const int n = 40 * 24 * 56;
  uint8_t* solid = calloc(n, 1);
  for (int k = 0; k < n; ++k) {
    const int x = k % 40, y = (k / 40) % 24, z = k / 960;
    const double d = sqrt((x - 20.0) * (x - 20.0) + (y - 12.0) * (y - 12.0) + (z - 28.0) * (z - 28.0));
    solid[k] = (d < 7.0 && x >= 2 && x < 38) ? 1 : 0;
  }
  uint8_t act[3 * 2 * 4];
  memset(act, 0, sizeof act);
  for (int bz = 0; bz < 4; ++bz)
    for (int by = 0; by < 2; ++by) act[0 + 3 * (by + 2 * bz)] = 1;
  bad |= run(p, solid, NULL, act, 60);
  free(solid);
  printf("oracle driver: %s\n", bad ? "non-finite values" : "ok");
  return bad;
}
