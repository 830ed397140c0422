/*
 * Reference oracle for the two-component pseudo-potential lattice Boltzmann
 * update with a progressive (block-activated) mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, double-precision CPU
 * implementation used to check the GPU library.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the GPU library.
 *
 * Everything works on full-lattice arrays indexed n = x + nx*(y + ny*z) and
 * uses straightforward loops.  Each function cites the passage of Duchateau et
 * al., "A Progressive Mesh Method for Physical Simulations Using Lattice
 * Boltzmann Method on Single-Node multi-GPU Architectures" (arXiv 1510.03560)
 * that it follows.  Where the printed text is garbled or silent, the reading
 * used is stated at the point of use.
 *
 * Per time step t -> t+1 (paper section 2 and section 4.3):
 *   1. moments rho_a, u_a of f(t)                       (Eq 4-5)
 *   2. pseudo-potential psi_a(rho_a)                      (Eq 6-7)
 *   3. intra- and inter-component forces                  (Eq 8-9)
 *   4. BGK collision with exact-difference forcing        (Eq 10-12)
 *   5. streaming with half-way bounce-back
 *   6. moments of f(t+1)
 *   7. criterion on the boundaries of active blocks and creation of the
 *      neighbouring blocks                                (Eq 13, section 4.2-4.3)
 * Cells of inactive blocks are never updated: they hold the rest state.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19 velocity set (section 2.1, Fig 1b), listed so that direction 2k-1 and
 * 2k are opposite.  Weights are the standard D3Q19 values (the paper defers
 * them to its reference [1]). */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W[Q] = {1.0 / 3.0,
                            1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

/* lattice sound speed squared, Eq 3 with dx = dt = 1 */
static const double CS2 = 1.0 / 3.0;

/* Face boundary kinds, one per face in the order -x,+x,-y,+y,-z,+z. */
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_INLET = 2, ORC_OUTLET = 3 };
/* Cell kinds. */
enum { K_FLUID = 0, K_SOLID = 1, K_INLET = 2, K_OUTLET = 3 };

typedef struct orc_params {
  int32_t nx, ny, nz, ncomp;
  int32_t block;        /* edge of the cubic sub-domains (progressive mesh) */
  int32_t shell_width;  /* depth of the boundary shell the criterion scans */
  int32_t bc[6];
  double tau[2];
  double eos_a, eos_b, eos_R, eos_omega, T_over_Tc;
  double g[2][2];       /* g[a][a]: Eq 6 and 8; g[0][1] = g[1][0]: Eq 9 */
  double beta;          /* Eq 8 mixing weight */
  double S;             /* Eq 13 threshold */
  double body[2][3];    /* extra body force per unit density (gravity) */
  double inlet_rho[2], inlet_u[3], bg_rho[2];
} orc_params;

/* ---------------------------------------------------------------- lattice */

int orc_lattice(int32_t* ex, int32_t* ey, int32_t* ez, double* w, int32_t* opp) {
  for (int i = 0; i < Q; i++) {
    ex[i] = EX[i]; ey[i] = EY[i]; ez[i] = EZ[i]; w[i] = W[i]; opp[i] = opposite(i);
  }
  return Q;
}

/* Eq 2: second-order equilibrium, written with c_s^2 as printed. */
void orc_feq(double rho, const double u[3], double out[Q]) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; i++) {
    double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
    out[i] = W[i] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq 4-5: density and momentum of one cell's populations. */
static void cell_moments(const double f[Q], double* rho, double j[3]) {
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < Q; i++) {
    r += f[i];
    jx += f[i] * EX[i];
    jy += f[i] * EY[i];
    jz += f[i] * EZ[i];
  }
  *rho = r; j[0] = jx; j[1] = jy; j[2] = jz;
}

/* Velocity from Eq 5.  A non-positive density has no velocity (the paper is
 * silent; such cells are counted by the caller). */
static void cell_velocity(double rho, const double j[3], double u[3]) {
  if (rho > 0.0) { u[0] = j[0] / rho; u[1] = j[1] / rho; u[2] = j[2] / rho; }
  else { u[0] = u[1] = u[2] = 0.0; }
}

/* ------------------------------------------------------------------- EOS */

/* Eq 7, Peng-Robinson pressure.  The printed denominator "1 + 2b - b^2 rho^2"
 * is read as the standard 1 + 2 b rho - b^2 rho^2.  theta(T) is the
 * Peng-Robinson alpha function [1 + kappa (1 - sqrt(T/Tc))]^2 with
 * kappa = 0.37464 + 1.54226 w - 0.26992 w^2, and Tc = (0.07780/0.45724) a/(b R),
 * the critical temperature of this equation of state. */
typedef struct { double RT, a_theta, b, Tc, T, kappa, theta; } eos_consts;

static eos_consts eos_setup(const orc_params* p) {
  eos_consts e;
  const double Omega_a = 0.45724, Omega_b = 0.07780;
  e.Tc = (Omega_b / Omega_a) * p->eos_a / (p->eos_b * p->eos_R);
  e.T = p->T_over_Tc * e.Tc;
  double w = p->eos_omega;
  e.kappa = 0.37464 + 1.54226 * w - 0.26992 * w * w;
  double s = 1.0 + e.kappa * (1.0 - sqrt(e.T / e.Tc));
  e.theta = s * s;
  e.RT = p->eos_R * e.T;
  e.a_theta = p->eos_a * e.theta;
  e.b = p->eos_b;
  return e;
}

static double pr_pressure(const eos_consts* e, double rho) {
  return rho * e->RT / (1.0 - e->b * rho) -
         e->a_theta * rho * rho / (1.0 + 2.0 * e->b * rho - e->b * e->b * rho * rho);
}

/* Eq 6: psi = sqrt(2 (p - c_s^2 rho) / (c_s^2 g)).  A negative radicand (the
 * paper is silent) is clamped to zero and counted; g = 0 means no potential. */
static double pseudo_potential(const eos_consts* e, double g, double rho, int64_t* clamps) {
  if (g == 0.0) return 0.0;
  double rad = 2.0 * (pr_pressure(e, rho) - CS2 * rho) / (CS2 * g);
  if (rad < 0.0) { if (clamps) (*clamps)++; return 0.0; }
  return sqrt(rad);
}

/* Exposed for the equation-of-state pins. */
int orc_eos(const orc_params* p, int comp, const double* rho, int64_t n, double* pressure,
            double* psi, double* consts /* Tc, T, kappa, theta */) {
  eos_consts e = eos_setup(p);
  for (int64_t k = 0; k < n; k++) {
    if (pressure) pressure[k] = pr_pressure(&e, rho[k]);
    if (psi) psi[k] = pseudo_potential(&e, p->g[comp][comp], rho[k], NULL);
  }
  if (consts) { consts[0] = e.Tc; consts[1] = e.T; consts[2] = e.kappa; consts[3] = e.theta; }
  return 0;
}

/* ---------------------------------------------------------------- forces */

/* Eq 8 and Eq 9 for component a at one cell.
 *   psi_c[b]     : psi of component b at the cell itself
 *   psi_nb[b][i] : psi of component b at x + e_i, already substituted where
 *                  the neighbour is solid or outside the domain
 * Reading of the garbled prints: with the lattice weights w_i, the factor
 * (g/2) c_s^2 times the paper's weights equals g times w_i (the paper's
 * weights being 6 w_i), so
 *   F_aa  = -beta g_aa psi_a(x) sum_i w_i psi_a(x+e_i) e_i
 *           - (1-beta)/2 g_aa   sum_i w_i psi_a(x+e_i)^2 e_i
 *   F_ab  = -g_ab psi_a(x) sum_i w_i psi_b(x+e_i) e_i      (b the other component)
 * which together tend to -grad(p - c_s^2 rho) for smooth fields. */
void orc_cell_force(const orc_params* p, int a, const double psi_c[2], const double psi_nb[2][Q],
                    double F[3]) {
  double s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0}, s3[3] = {0, 0, 0};
  int b = 1 - a;
  for (int i = 1; i < Q; i++) {
    double e[3] = {EX[i], EY[i], EZ[i]};
    for (int d = 0; d < 3; d++) {
      s1[d] += W[i] * psi_nb[a][i] * e[d];
      s2[d] += W[i] * psi_nb[a][i] * psi_nb[a][i] * e[d];
      if (p->ncomp == 2) s3[d] += W[i] * psi_nb[b][i] * e[d];
    }
  }
  double gaa = p->g[a][a];
  for (int d = 0; d < 3; d++) {
    F[d] = -p->beta * gaa * psi_c[a] * s1[d] - 0.5 * (1.0 - p->beta) * gaa * s2[d];
    if (p->ncomp == 2) F[d] += -p->g[a][b] * psi_c[a] * s3[d];
  }
}

/* --------------------------------------------------------------- collide */

/* Eq 10-12 with the relaxation read as -(1/tau)(f - f_eq) (the printed "+" is
 * anti-damping): f* = f - (f - feq(rho,u))/tau + feq(rho,u+du) - feq(rho,u),
 * du = F/rho. */
void orc_collide(double tau, const double f[Q], const double F[3], double fstar[Q]) {
  double rho, j[3], u[3], ud[3], feq[Q], feqd[Q];
  cell_moments(f, &rho, j);
  cell_velocity(rho, j, u);
  for (int d = 0; d < 3; d++) ud[d] = u[d] + (rho > 0.0 ? F[d] / rho : 0.0);
  orc_feq(rho, u, feq);
  orc_feq(rho, ud, feqd);
  for (int i = 0; i < Q; i++) fstar[i] = f[i] - (f[i] - feq[i]) / tau + (feqd[i] - feq[i]);
}

/* ------------------------------------------------------------ rest state */

/* The state that a cell at rest with background density holds forever: start
 * from w_i rho_bg and apply the update of a cell whose neighbourhood is
 * identical to itself (so the force vanishes; no body force) until the
 * populations no longer change in the last bit.
 * The paper is silent on the initial state of a new sub-domain; this is the
 * exact rest state in this arithmetic, so a cell that is never reached by the
 * fluid is the same whether its block exists or not. */
int orc_rest_state(const orc_params* p, double frest[2][Q], double rho_rest[2], double psi_rest[2]) {
  eos_consts e = eos_setup(p);
  for (int a = 0; a < p->ncomp; a++) {
    double f[Q], fn[Q];
    for (int i = 0; i < Q; i++) f[i] = W[i] * p->bg_rho[a];
    int it;
    for (it = 0; it < 10000; it++) {
      /* psi of both components as the stencil sees it on a uniform lattice */
      double psi_c[2] = {0, 0}, psi_nb[2][Q], F[3], r, j[3];
      for (int b = 0; b < p->ncomp; b++) {
        double fb[Q];
        if (b == a) memcpy(fb, f, sizeof fb);
        else for (int i = 0; i < Q; i++) fb[i] = W[i] * p->bg_rho[b];
        cell_moments(fb, &r, j);
        psi_c[b] = pseudo_potential(&e, p->g[b][b], r, NULL);
        for (int i = 0; i < Q; i++) psi_nb[b][i] = psi_c[b];
      }
      orc_cell_force(p, a, psi_c, psi_nb, F);
      orc_collide(p->tau[a], f, F, fn);
      if (memcmp(fn, f, sizeof f) == 0) break;
      memcpy(f, fn, sizeof f);
    }
    if (it == 10000) return -1;
    double j[3];
    memcpy(frest[a], f, sizeof f);
    cell_moments(f, &rho_rest[a], j);
    psi_rest[a] = pseudo_potential(&e, p->g[a][a], rho_rest[a], NULL);
  }
  return 0;
}

/* ------------------------------------------------------------ simulation */

typedef struct orc_sim {
  orc_params p;
  eos_consts e;
  int64_t N;
  int nbx, nby, nbz, nb;
  uint8_t* kind;        /* per cell: K_FLUID, K_SOLID, K_INLET, K_OUTLET */
  uint8_t* bactive;     /* per block */
  uint8_t* bfluid;      /* per block: contains a non-solid cell */
  double* f;            /* [a][i][n] populations f(t) */
  double* fs;           /* [a][i][n] post-collision populations */
  double* psi;          /* [a][n] */
  double* u_old;        /* [a][3][n] velocity at t */
  double frest[2][Q], rho_rest[2], psi_rest[2], finlet[2][Q], psi_inlet[2];
  int64_t step, leak, clamps, nonpos;
  int32_t* trace;       /* pairs (step, block) */
  int64_t ntrace, cap_trace;
} orc_sim;

static int64_t cell_index(const orc_sim* s, int x, int y, int z) {
  return x + (int64_t)s->p.nx * (y + (int64_t)s->p.ny * z);
}
static int block_of(const orc_sim* s, int x, int y, int z) {
  int B = s->p.block;
  return x / B + s->nbx * (y / B + s->nby * (z / B));
}

/* Neighbour of (x,y,z) along (dx,dy,dz): wraps across periodic faces, returns
 * -1 when it leaves the domain across any other face. */
static int64_t neighbour(const orc_sim* s, int x, int y, int z, int dx, int dy, int dz) {
  int c[3] = {x + dx, y + dy, z + dz};
  int L[3] = {s->p.nx, s->p.ny, s->p.nz};
  for (int d = 0; d < 3; d++) {
    if (c[d] < 0 || c[d] >= L[d]) {
      int face = 2 * d + (c[d] < 0 ? 0 : 1);
      if (s->p.bc[face] != ORC_PERIODIC) return -1;
      c[d] = (c[d] + L[d]) % L[d];
    }
  }
  return cell_index(s, c[0], c[1], c[2]);
}

#define F_AT(arr, a, i, n) (arr)[((int64_t)(a) * Q + (i)) * s->N + (n)]

void orc_destroy(orc_sim* s) {
  if (!s) return;
  free(s->kind); free(s->bactive); free(s->bfluid); free(s->f); free(s->fs);
  free(s->psi); free(s->u_old); free(s->trace); free(s);
}

/* solid: per cell (nonzero = solid).  rho0: [ncomp][N] or NULL; u0: [3][N] or
 * NULL.  active_blocks: per block (nonzero = meshed at t = 0) or NULL for the
 * static mesh, where every block holding fluid is meshed.  Cells of blocks
 * meshed at t = 0 start at f_eq(rho0, u0) unless (rho0, u0) equals the
 * background rest state, which starts at the exact rest populations; every
 * other cell starts at the rest state. */
orc_sim* orc_create(const orc_params* p, const uint8_t* solid, const double* rho0, const double* u0,
                    const uint8_t* active_blocks) {
  if (p->ncomp < 1 || p->ncomp > 2 || p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || p->block <= 0) return NULL;
  /* a periodic axis wraps whole blocks; along the other axes the last block
   * may extend past the lattice (uneven edges: the cells it would hold
   * beyond the lattice do not exist, exactly as solid padding behaves) */
  {
    int n[3] = {p->nx, p->ny, p->nz};
    for (int d = 0; d < 3; d++)
      if (p->bc[2 * d] == ORC_PERIODIC && n[d] % p->block) return NULL;
  }
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->p = *p;
  s->e = eos_setup(p);
  s->N = (int64_t)p->nx * p->ny * p->nz;
  s->nbx = (p->nx + p->block - 1) / p->block;
  s->nby = (p->ny + p->block - 1) / p->block;
  s->nbz = (p->nz + p->block - 1) / p->block;
  s->nb = s->nbx * s->nby * s->nbz;
  int64_t N = s->N;
  int nc = p->ncomp;
  s->kind = (uint8_t*)calloc(N, 1);
  s->bactive = (uint8_t*)calloc(s->nb, 1);
  s->bfluid = (uint8_t*)calloc(s->nb, 1);
  s->f = (double*)malloc(sizeof(double) * nc * Q * N);
  s->fs = (double*)malloc(sizeof(double) * nc * Q * N);
  s->psi = (double*)malloc(sizeof(double) * nc * N);
  s->u_old = (double*)malloc(sizeof(double) * nc * 3 * N);
  s->cap_trace = 1024;
  s->trace = (int32_t*)malloc(sizeof(int32_t) * 2 * s->cap_trace);
  if (!s->kind || !s->bactive || !s->bfluid || !s->f || !s->fs || !s->psi || !s->u_old || !s->trace) {
    orc_destroy(s); return NULL;
  }
  if (orc_rest_state(p, s->frest, s->rho_rest, s->psi_rest) != 0) { orc_destroy(s); return NULL; }
  for (int a = 0; a < nc; a++) {
    double ui[3] = {p->inlet_u[0], p->inlet_u[1], p->inlet_u[2]};
    orc_feq(p->inlet_rho[a], ui, s->finlet[a]);
    s->psi_inlet[a] = pseudo_potential(&s->e, p->g[a][a], p->inlet_rho[a], NULL);
  }
  /* cell kinds: a non-solid cell on a face layer with an inlet (outlet)
   * condition is an inlet (outlet) node; inlet wins over outlet */
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        int64_t n = cell_index(s, x, y, z);
        uint8_t k = (solid && solid[n]) ? K_SOLID : K_FLUID;
        if (k == K_FLUID) {
          int on[6] = {x == 0, x == p->nx - 1, y == 0, y == p->ny - 1, z == 0, z == p->nz - 1};
          for (int fc = 0; fc < 6; fc++) if (on[fc] && p->bc[fc] == ORC_OUTLET) k = K_OUTLET;
          for (int fc = 0; fc < 6; fc++) if (on[fc] && p->bc[fc] == ORC_INLET) k = K_INLET;
          s->bfluid[block_of(s, x, y, z)] = 1;
        }
        s->kind[n] = k;
      }
  for (int b = 0; b < s->nb; b++)
    s->bactive[b] = active_blocks ? (active_blocks[b] && s->bfluid[b]) : s->bfluid[b];
  /* initial populations */
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        int64_t n = cell_index(s, x, y, z);
        int act = s->bactive[block_of(s, x, y, z)];
        double u[3] = {0, 0, 0};
        if (u0) { u[0] = u0[n]; u[1] = u0[N + n]; u[2] = u0[2 * N + n]; }
        for (int a = 0; a < nc; a++) {
          double r = rho0 ? rho0[a * N + n] : p->bg_rho[a];
          int at_rest = (r == p->bg_rho[a] && u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0);
          double fe[Q];
          if (act && !at_rest) orc_feq(r, u, fe);
          else memcpy(fe, s->frest[a], sizeof fe);
          for (int i = 0; i < Q; i++) F_AT(s->f, a, i, n) = fe[i];
        }
      }
  return s;
}

/* Moments of f at every non-solid cell. */
static void all_moments(orc_sim* s, double* rho, double* u) {
  int nc = s->p.ncomp;
  int64_t N = s->N;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; n++) {
    for (int a = 0; a < nc; a++) {
      double fc[Q], r, j[3], v[3];
      if (s->kind[n] == K_SOLID) {
        rho[a * N + n] = 0.0;
        u[(a * 3 + 0) * N + n] = u[(a * 3 + 1) * N + n] = u[(a * 3 + 2) * N + n] = 0.0;
        continue;
      }
      for (int i = 0; i < Q; i++) fc[i] = F_AT(s->f, a, i, n);
      cell_moments(fc, &r, j);
      cell_velocity(r, j, v);
      rho[a * N + n] = r;
      for (int d = 0; d < 3; d++) u[(a * 3 + d) * N + n] = v[d];
    }
  }
}

static void push_trace(orc_sim* s, int32_t step, int32_t block) {
  if (s->ntrace == s->cap_trace) {
    s->cap_trace *= 2;
    s->trace = (int32_t*)realloc(s->trace, sizeof(int32_t) * 2 * s->cap_trace);
  }
  s->trace[2 * s->ntrace] = step;
  s->trace[2 * s->ntrace + 1] = block;
  s->ntrace++;
}

/* One time step t -> t+1 over the meshed blocks. */
static void one_step(orc_sim* s) {
  const orc_params* p = &s->p;
  int nc = p->ncomp;
  int64_t N = s->N;
  double* rho = (double*)malloc(sizeof(double) * nc * N);
  double* u = (double*)malloc(sizeof(double) * nc * 3 * N);
  int64_t clamps = 0, nonpos = 0, leak = 0;

  /* 1. moments of f(t) (Eq 4-5) */
  all_moments(s, rho, u);

  /* 2. pseudo-potential (Eq 6-7); boundary nodes carry the potential of the
   * state they impose, cells of inactive blocks hold the rest state */
#pragma omp parallel for schedule(static) reduction(+ : clamps, nonpos)
  for (int64_t n = 0; n < N; n++) {
    for (int a = 0; a < nc; a++) {
      double v;
      switch (s->kind[n]) {
        case K_SOLID: v = 0.0; break;
        case K_INLET: v = s->psi_inlet[a]; break;
        case K_OUTLET: v = s->psi_rest[a]; break;
        default:
          if (rho[a * N + n] <= 0.0) nonpos++;
          v = pseudo_potential(&s->e, p->g[a][a], rho[a * N + n], &clamps);
      }
      s->psi[a * N + n] = v;
    }
  }

  /* 3-4. forces (Eq 8-9) and collision (Eq 10-12) */
#pragma omp parallel for schedule(static) reduction(+ : leak)
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        int64_t n = cell_index(s, x, y, z);
        int k = s->kind[n];
        if (k == K_SOLID) continue;
        if (!s->bactive[block_of(s, x, y, z)]) {
          for (int a = 0; a < nc; a++)
            for (int i = 0; i < Q; i++) F_AT(s->fs, a, i, n) = F_AT(s->f, a, i, n);
          /* an inlet node outside the mesh would inject in a full-mesh run */
          if (k == K_INLET) leak++;
          continue;
        }
        for (int a = 0; a < nc; a++) {
          double fst[Q];
          if (k == K_INLET) memcpy(fst, s->finlet[a], sizeof fst);
          else if (k == K_OUTLET) memcpy(fst, s->frest[a], sizeof fst);
          else {
            /* neighbour potentials; a solid neighbour, or one outside the
             * domain, contributes the centre cell's own potential of the same
             * component (neutral wetting; the paper leaves the solid
             * interaction to its reference [3]) */
            double psi_c[2] = {0, 0}, psi_nb[2][Q], F[3], fc[Q];
            for (int b = 0; b < nc; b++) psi_c[b] = s->psi[b * N + n];
            for (int i = 0; i < Q; i++) {
              int64_t m = neighbour(s, x, y, z, EX[i], EY[i], EZ[i]);
              for (int b = 0; b < nc; b++)
                psi_nb[b][i] = (m < 0 || s->kind[m] == K_SOLID) ? psi_c[b] : s->psi[b * N + m];
            }
            orc_cell_force(p, a, psi_c, psi_nb, F);
            for (int d = 0; d < 3; d++) F[d] += rho[a * N + n] * p->body[a][d];
            for (int i = 0; i < Q; i++) fc[i] = F_AT(s->f, a, i, n);
            orc_collide(p->tau[a], fc, F, fst);
          }
          for (int i = 0; i < Q; i++) F_AT(s->fs, a, i, n) = fst[i];
        }
        /* leak: what this active cell hands to a cell of an inactive block
         * must be the rest state, else the inactive block misses an update */
        for (int i = 1; i < Q; i++) {
          int64_t m = neighbour(s, x, y, z, EX[i], EY[i], EZ[i]);
          if (m < 0 || s->kind[m] == K_SOLID) continue;
          int mz = (int)(m / ((int64_t)p->nx * p->ny)), my = (int)((m / p->nx) % p->ny), mx = (int)(m % p->nx);
          if (s->bactive[block_of(s, mx, my, mz)]) continue;
          int bad = 0;
          for (int a = 0; a < nc; a++)
            if (F_AT(s->fs, a, i, n) != s->frest[a][i] || s->psi[a * N + n] != s->psi_rest[a]) bad = 1;
          leak += bad;
        }
      }

  /* 5. streaming (pull) with half-way bounce-back: a population arriving
   * from a solid cell, or across a non-periodic face, is the cell's own
   * post-collision population of the opposite direction */
#pragma omp parallel for schedule(static)
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        int64_t n = cell_index(s, x, y, z);
        if (s->kind[n] == K_SOLID || !s->bactive[block_of(s, x, y, z)]) continue;
        for (int i = 0; i < Q; i++) {
          int64_t m = neighbour(s, x, y, z, -EX[i], -EY[i], -EZ[i]);
          for (int a = 0; a < nc; a++) {
            if (m < 0 || s->kind[m] == K_SOLID) F_AT(s->f, a, i, n) = F_AT(s->fs, a, opposite(i), n);
            else F_AT(s->f, a, i, n) = F_AT(s->fs, a, i, m);
          }
        }
      }

  /* 6-7. moments of f(t+1) and the criterion of Eq 13 on the boundary of
   * every active block (section 4.2): a neighbouring block that holds fluid
   * and is not meshed yet is created when some fluid cell of the active block
   * within shell_width cells of it sees its velocity change by more than S for
   * any component.  "On the boundary" is read as this shell over all 26
   * neighbouring blocks: one step moves information two cells (one for the
   * potential stencil, one for streaming), so a thinner shell lets a change
   * reach a block before it exists.  Creation happens at the end of the step
   * (section 4.3), so the new blocks join the next step. */
  double* rho1 = (double*)malloc(sizeof(double) * nc * N);
  double* u1 = (double*)malloc(sizeof(double) * nc * 3 * N);
  all_moments(s, rho1, u1);
  int B = p->block, w = p->shell_width;
  uint8_t* create = (uint8_t*)calloc(s->nb, 1);
  for (int bz = 0; bz < s->nbz; bz++)
    for (int by = 0; by < s->nby; by++)
      for (int bx = 0; bx < s->nbx; bx++) {
        int b = bx + s->nbx * (by + s->nby * bz);
        if (!s->bactive[b]) continue;
        for (int dz = -1; dz <= 1; dz++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              if (!dx && !dy && !dz) continue;
              int c[3] = {bx + dx, by + dy, bz + dz}, nbl[3] = {s->nbx, s->nby, s->nbz}, ok = 1;
              for (int d = 0; d < 3; d++) {
                if (c[d] < 0 || c[d] >= nbl[d]) {
                  if (p->bc[2 * d + (c[d] < 0 ? 0 : 1)] != ORC_PERIODIC) ok = 0;
                  c[d] = (c[d] + nbl[d]) % nbl[d];
                }
              }
              if (!ok) continue;
              int nbk = c[0] + s->nbx * (c[1] + s->nby * c[2]);
              if (s->bactive[nbk] || !s->bfluid[nbk] || create[nbk]) continue;
              /* cells of block b within w cells of the neighbour block */
              int lo[3], hi[3], dd[3] = {dx, dy, dz};
              for (int d = 0; d < 3; d++) {
                lo[d] = dd[d] > 0 ? B - w : 0;
                hi[d] = dd[d] < 0 ? w - 1 : B - 1;
              }
              int fire = 0;
              for (int lz = lo[2]; lz <= hi[2] && !fire; lz++)
                for (int ly = lo[1]; ly <= hi[1] && !fire; ly++)
                  for (int lx = lo[0]; lx <= hi[0] && !fire; lx++) {
                    if (bx * B + lx >= p->nx || by * B + ly >= p->ny || bz * B + lz >= p->nz) continue;
                    int64_t n = cell_index(s, bx * B + lx, by * B + ly, bz * B + lz);
                    if (s->kind[n] == K_SOLID) continue;
                    for (int a = 0; a < nc && !fire; a++) {
                      double d0 = u1[(a * 3 + 0) * N + n] - u[(a * 3 + 0) * N + n];
                      double d1 = u1[(a * 3 + 1) * N + n] - u[(a * 3 + 1) * N + n];
                      double d2 = u1[(a * 3 + 2) * N + n] - u[(a * 3 + 2) * N + n];
                      /* ||C||_2 > S; for S = 0 this is "some component changed" */
                      if (p->S == 0.0) fire = (d0 != 0.0 || d1 != 0.0 || d2 != 0.0);
                      else fire = sqrt(d0 * d0 + d1 * d1 + d2 * d2) > p->S;
                    }
                  }
              if (fire) create[nbk] = 1;
            }
      }
  s->step++;
  for (int b = 0; b < s->nb; b++)
    if (create[b]) { s->bactive[b] = 1; push_trace(s, (int32_t)s->step, b); }
  s->leak += leak;
  s->clamps += clamps;
  s->nonpos += nonpos;
  free(create); free(rho); free(u); free(rho1); free(u1);
}

int orc_step(orc_sim* s, int32_t nsteps) {
  for (int32_t k = 0; k < nsteps; k++) one_step(s);
  return 0;
}

/* Blocks created by the solver after t = 0 (lbm_activate-style seeding is done
 * through active_blocks at creation or through this call between steps). */
int orc_activate(orc_sim* s, const int32_t* blocks, int32_t n) {
  for (int k = 0; k < n; k++) {
    int b = blocks[k];
    if (b < 0 || b >= s->nb) return -1;
    if (s->bfluid[b] && !s->bactive[b]) { s->bactive[b] = 1; push_trace(s, (int32_t)s->step, b); }
  }
  return 0;
}

/* Macroscopic output after the last step (Eq 4-5, section 2.2): rho_a and
 * u_a per cell, and the mixture velocity sum_a rho_a u_a / sum_a rho_a.
 * Solid cells report zeros.  active_cells marks cells of meshed blocks. */
int orc_moments(orc_sim* s, double* rho, double* u, double* umix, uint8_t* active_cells) {
  int nc = s->p.ncomp;
  int64_t N = s->N;
  double* uu = u ? u : (double*)malloc(sizeof(double) * nc * 3 * N);
  double* rr = rho ? rho : (double*)malloc(sizeof(double) * nc * N);
  all_moments(s, rr, uu);
  if (umix) {
    for (int64_t n = 0; n < N; n++) {
      double m = 0.0, jm[3] = {0, 0, 0};
      for (int a = 0; a < nc; a++) {
        m += rr[a * N + n];
        for (int d = 0; d < 3; d++) jm[d] += rr[a * N + n] * uu[(a * 3 + d) * N + n];
      }
      for (int d = 0; d < 3; d++) umix[d * N + n] = (m > 0.0) ? jm[d] / m : 0.0;
    }
  }
  if (active_cells) {
    for (int z = 0; z < s->p.nz; z++)
      for (int y = 0; y < s->p.ny; y++)
        for (int x = 0; x < s->p.nx; x++)
          active_cells[cell_index(s, x, y, z)] = s->bactive[block_of(s, x, y, z)];
  }
  if (!u) free(uu);
  if (!rho) free(rr);
  return 0;
}

/* Potential and total force of every non-solid cell in the current state,
 * for the stencil pins.  psi: [ncomp][N]; F: [ncomp][3][N]. */
int orc_debug_fields(orc_sim* s, double* psi, double* F) {
  const orc_params* p = &s->p;
  int nc = p->ncomp;
  int64_t N = s->N;
  double* rho = (double*)malloc(sizeof(double) * nc * N);
  double* u = (double*)malloc(sizeof(double) * nc * 3 * N);
  all_moments(s, rho, u);
  for (int64_t n = 0; n < N; n++)
    for (int a = 0; a < nc; a++) {
      double v;
      switch (s->kind[n]) {
        case K_SOLID: v = 0.0; break;
        case K_INLET: v = s->psi_inlet[a]; break;
        case K_OUTLET: v = s->psi_rest[a]; break;
        default: v = pseudo_potential(&s->e, p->g[a][a], rho[a * N + n], NULL);
      }
      psi[a * N + n] = v;
    }
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++)
      for (int x = 0; x < p->nx; x++) {
        int64_t n = cell_index(s, x, y, z);
        for (int a = 0; a < nc; a++) {
          double Fc[3] = {0, 0, 0};
          if (s->kind[n] == K_FLUID) {
            double psi_c[2] = {0, 0}, psi_nb[2][Q];
            for (int b = 0; b < nc; b++) psi_c[b] = psi[b * N + n];
            for (int i = 0; i < Q; i++) {
              int64_t m = neighbour(s, x, y, z, EX[i], EY[i], EZ[i]);
              for (int b = 0; b < nc; b++)
                psi_nb[b][i] = (m < 0 || s->kind[m] == K_SOLID) ? psi_c[b] : psi[b * N + m];
            }
            orc_cell_force(p, a, psi_c, psi_nb, Fc);
            for (int d = 0; d < 3; d++) Fc[d] += rho[a * N + n] * p->body[a][d];
          }
          for (int d = 0; d < 3; d++) F[(a * 3 + d) * N + n] = Fc[d];
        }
      }
  free(rho); free(u);
  return 0;
}

/* Counters: step, leak, clamps, non-positive densities, trace length. */
int orc_counters(const orc_sim* s, int64_t out[5]) {
  out[0] = s->step; out[1] = s->leak; out[2] = s->clamps; out[3] = s->nonpos; out[4] = s->ntrace;
  return 0;
}
int orc_trace(const orc_sim* s, int32_t* out) {
  memcpy(out, s->trace, sizeof(int32_t) * 2 * s->ntrace);
  return 0;
}
int orc_rest(const orc_sim* s, double* frest, double* rho_rest, double* psi_rest) {
  for (int a = 0; a < s->p.ncomp; a++) {
    memcpy(frest + a * Q, s->frest[a], sizeof(double) * Q);
    rho_rest[a] = s->rho_rest[a];
    psi_rest[a] = s->psi_rest[a];
  }
  return 0;
}
/* Raw populations f(t): [ncomp][19][N]. */
int orc_populations(const orc_sim* s, double* out) {
  memcpy(out, s->f, sizeof(double) * s->p.ncomp * Q * s->N);
  return 0;
}
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
