/*
 * lbm.h - C ABI of the progressive-mesh two-component lattice Boltzmann
 * library for AMD Instinct MI355X (gfx950).
 *
 * The library advances a D3Q19 two-component pseudo-potential lattice
 * Boltzmann model (Duchateau et al., arXiv 1510.03560, section 2) over the
 * 16^3 blocks of a lattice that a progressive mesh activates as the fluid
 * propagates (section 4.1-4.3).  One GPU holds the whole domain.
 *
 * Conventions for every call:
 *  - Lattice arrays on the host are indexed n = x + nx*(y + ny*z) (x fastest).
 *  - Block b covers cells [16*bx, 16*bx+16) x ... with b = bx + nbx*(by + nby*bz),
 *    nbx = ceil(nx/16) etc.  A non-periodic axis whose length is not a
 *    multiple of 16 is padded to whole blocks with solid cells, which act as
 *    the walls of that face would (bounce-back, and the neutral neighbour of
 *    Eq 8-9); host arrays keep the unpadded size.
 *  - All pointers in this header are HOST pointers unless stated otherwise.
 *    The caller owns them; the library copies what it needs during the call
 *    and keeps no pointer.
 *  - Every call returns LBM_OK (0) or a negative LBM_E* code and never throws.
 *    lbm_last_error() returns a text for the last failure on a handle.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - Work is enqueued on the HIP stream given to lbm_create.  lbm_step returns
 *    before the GPU has finished; a failure inside the GPU work (non-finite
 *    densities, pool exhaustion) is reported by the next call that waits for
 *    the stream (lbm_moments, lbm_stats, lbm_sync).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- error codes */
#define LBM_OK 0
#define LBM_EINVAL (-1)   /* invalid argument or parameter */
#define LBM_ESTATE (-2)   /* call out of order (e.g. lbm_step before lbm_set_geometry) */
#define LBM_ENOMEM (-3)   /* device allocation failed or the block pool is full */
#define LBM_EHIP (-4)     /* a HIP runtime call failed */
#define LBM_ENUMERIC (-5) /* a density became non-positive or non-finite */

/* ------------------------------------------------------------ face kinds */
/* Faces are ordered -x, +x, -y, +y, -z, +z. */
#define LBM_BC_PERIODIC 0 /* wraps to the opposite face */
#define LBM_BC_WALL 1     /* half-way bounce-back at the face */
#define LBM_BC_INLET 2    /* fluid cells of the face layer impose f_eq(inlet_rho, inlet_u) */
#define LBM_BC_OUTLET 3   /* fluid cells of the face layer impose the rest state */

/* ------------------------------------------------------ storage formats */
#define LBM_STORE_F32 0    /* populations stored as FP32 */
#define LBM_STORE_F16DEV 1 /* populations stored as FP16 deviations from w_i * rho (FP32 math) */

/* ------------------------------------------------------ access patterns */
/* LBM_PATTERN_AB: two population buffers; each step reads one and writes the
 *   other (pull streaming, one fused kernel per step).
 * LBM_PATTERN_AA: one population buffer updated in place (the A-A pattern of
 *   section 3, which halves the population memory): steps of even index
 *   read and write each cell's own populations with opposite directions
 *   swapped, steps of odd index read from and write to the neighbours.  Two
 *   kernels per step (psi, then collision and streaming).  Either storage
 *   format.  Results are bitwise those of LBM_PATTERN_AB with the same
 *   storage format. */
#define LBM_PATTERN_AB 0
#define LBM_PATTERN_AA 1

/*
 * Run parameters (copied at lbm_create).
 *
 * Physics (section 2): relaxation time tau of each component (Eq 1, 10);
 * Peng-Robinson equation of state (Eq 7) with a = eos_a, b = eos_b,
 * R = eos_R, acentric factor eos_omega and temperature T_over_Tc * Tc, where
 * Tc = (0.07780 / 0.45724) a / (b R); pseudo-potential of Eq 6 with
 * g_aa = g[a][a]; intra-component force of Eq 8 with weight beta;
 * inter-component force of Eq 9 with g_ab = g[0][1] (must equal g[1][0]).
 * body[a] is an extra force per unit density on component a (gravity).
 *
 * Progressive mesh (section 4.2): a block is activated when a fluid cell of
 * an active neighbouring block, within shell_width cells of it, changes its
 * velocity by more than S (Eq 13) between two steps, for any component.
 */
typedef struct lbm_params {
  int32_t nx, ny, nz;    /* lattice size; a periodic axis must be a multiple of block, other axes are padded */
  int32_t block;         /* block edge; must be 16 */
  int32_t ncomp;         /* number of components, 1 or 2 */
  int32_t shell_width;   /* criterion shell depth in cells, 1..8 (default 2) */
  int32_t bc[6];         /* LBM_BC_* per face; opposite faces must both be periodic or neither */
  int32_t store;         /* LBM_STORE_* */
  int32_t progressive;   /* 0: static mesh (every block holding fluid active); 1: progressive */
  int32_t pool_blocks;   /* block slots to reserve; 0 = number of blocks holding fluid.  At most
                            65535 with LBM_STORE_F32 and 131071 with LBM_STORE_F16DEV for two
                            components, 131071 and 262143 for one (the kernels address a pair of
                            population planes, every component of each link side by side, with
                            32-bit byte offsets); when the padded nx is a multiple of 256 (16
                            blocks) the slots are padded to 4160 cells and the limits are 64526,
                            129054, 129054 and 258110 */
  int32_t pattern;       /* LBM_PATTERN_* */
  double tau[2];         /* > 0.5 */
  double eos_a, eos_b, eos_R, eos_omega, T_over_Tc;
  double g[2][2];
  double beta;
  double S;              /* >= 0 */
  double body[2][3];
  double inlet_rho[2];   /* density imposed by LBM_BC_INLET nodes, per component */
  double inlet_u[3];     /* velocity imposed by LBM_BC_INLET nodes */
  double bg_rho[2];      /* background density: the rest state of cells outside the mesh */
} lbm_params;

/* Device allocator used for every device buffer of a handle.  alloc returns
 * NULL on failure, else memory aligned to 256 bytes (as hipMalloc's is; the
 * kernels make 16-byte accesses from the start of a buffer, and a misaligned
 * block is released and reported as LBM_EINVAL); free accepts what alloc
 * returned.  ctx is passed through. */
typedef struct lbm_allocator {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} lbm_allocator;

typedef struct lbm_stats {
  int64_t steps;            /* steps taken */
  int32_t n_active;         /* active blocks */
  int32_t n_fluid_blocks;   /* blocks holding fluid */
  int32_t capacity;         /* block slots reserved */
  int32_t store;            /* LBM_STORE_* */
  int64_t bytes_reserved;   /* device bytes held by the handle */
  int64_t bytes_active;     /* device bytes of the active blocks' slots */
  double mass[2];           /* sum of rho_a over all fluid cells (FP64 accumulation) */
  int64_t leak;             /* see below */
  int64_t clamps;           /* cells whose Eq 6 radicand was negative (psi set to 0) */
  int32_t numeric_error;    /* nonzero once a density was non-positive or non-finite */
  int32_t pool_full;        /* nonzero if an activation did not fit the pool */
  int64_t activations;      /* blocks activated so far, by lbm_activate or the criterion (trace entries) */
  int32_t repacked;         /* progressive mesh: nonzero once every block holding fluid was active and
                               lbm_step put the slots in block order (the static mesh's layout, which
                               its steps then run as fast as); the fields are unchanged by it */
  int32_t reserved;
} lbm_stats_t;
/* leak: number of (step, cell, direction) links in which an active cell
 * showed a non-solid cell of an inactive block a pseudo-potential other than
 * the rest one, or handed it a population other than the rest state (same
 * bits in the stored format) that the block did not take in by activating
 * at the next step.  It is 0 exactly when the progressive mesh reproduces the
 * static mesh.  Progressive mode only (0 on a static mesh). */

typedef struct lbm_handle lbm_t;

/* Creates a handle.  stream: a hipStream_t, or NULL for the null stream.
 * alloc: NULL for hipMalloc/hipFree.  Checks and copies *p, derives the
 * equation-of-state constants, and computes on the GPU the rest state of
 * each component: the populations of a cell at rest with density bg_rho that
 * the update leaves unchanged to the last bit.  Errors: LBM_EINVAL for an
 * invalid parameter (message names it), LBM_ENOMEM, LBM_EHIP. */
int lbm_create(const lbm_params* p, void* stream, const lbm_allocator* alloc, lbm_t** out);

/* Sets the geometry and the initial fields; call once, after lbm_create.
 * solid: N bytes, nonzero = solid cell (NULL: no solid).  rho0: ncomp*N
 * densities, component-major (NULL: bg_rho everywhere).  u0: 3*N velocities,
 * x-component first (NULL: zero).  A cell of a block that is active at t = 0
 * starts at f_eq(rho0, u0) (Eq 2), except that a cell whose rho0 equals bg_rho
 * and whose u0 is zero starts at the rest state; every other cell is at rest.
 * Static mesh: every block holding fluid is activated here.  Progressive
 * mesh: no block is active until lbm_activate.  Reserves the block pool.
 * Errors: LBM_ESTATE if called twice, LBM_EINVAL if the pool would need more
 * slots than the store can address (see pool_blocks), LBM_ENOMEM, LBM_EHIP. */
int lbm_set_geometry(lbm_t* h, const uint8_t* solid, const double* rho0, const double* u0);

/* Device bytes that lbm_create followed by lbm_set_geometry(solid) would hold
 * for these parameters (the block pool sized as lbm_set_geometry sizes it),
 * written to *bytes, without touching the device: for choosing a storage
 * format or access pattern that fits a memory budget.  The initial fields of
 * lbm_set_geometry (4*ncomp*N bytes, plus 12*N with velocities) come on top
 * until the first step.  solid: N bytes as in lbm_set_geometry (NULL: no
 * solid).  Errors: LBM_EINVAL (invalid parameters, as lbm_create, or a pool
 * beyond the addressable slots); lbm_last_error(NULL) has the text. */
int lbm_plan_bytes(const lbm_params* p, const uint8_t* solid, int64_t* bytes);

/* Activates blocks (the "first sub-domain" of section 4.1, or any block a
 * caller wants meshed early).  block_ids: n block indices.  Blocks holding no
 * fluid, and blocks already active, are skipped.  Before the first lbm_step a
 * block takes rho0/u0 from lbm_set_geometry; later it takes the rest state,
 * which is also what an inactive block stands for, so activating extra blocks
 * never changes the results.  Errors: LBM_EINVAL (id out of range),
 * LBM_ESTATE (before lbm_set_geometry), LBM_ENOMEM (pool full). */
int lbm_activate(lbm_t* h, const int32_t* block_ids, int32_t n);

/* Advances nsteps time steps (section 4.3): per step, the moments and
 * pseudo-potential of every active cell, the criterion of Eq 13 on the
 * boundary shell of every active block next to an inactive block holding
 * fluid, activation of the requested blocks (they join this step's
 * collision), then forces, collision and streaming.  Asynchronous.  Once
 * every block holding fluid is active the criterion has nothing left to
 * request and the step no longer runs it.  In progressive mode every block
 * holding an inlet node must be active before the first step.  Errors: LBM_ESTATE, LBM_EINVAL (nsteps < 0, or an inlet
 * node outside the mesh), LBM_EHIP. */
int lbm_step(lbm_t* h, int32_t nsteps);

/* Waits for the stream; reports LBM_ENUMERIC or LBM_ENOMEM raised by the GPU. */
int lbm_sync(lbm_t* h);

/* Macroscopic fields after the last step (Eq 4-5): rho: ncomp*N densities;
 * u: ncomp*3*N velocities of each component (component-major, then x,y,z);
 * umix: 3*N mixture velocity sum_a rho_a u_a / sum_a rho_a; active: N bytes,
 * 1 for cells of active blocks.  Any output may be NULL.  Cells outside the
 * mesh report the rest state (density rho_rest, velocity 0); solid cells
 * report zeros.  Values are computed in FP32 and widened to double.
 * Synchronous.  Errors: LBM_ESTATE, LBM_ENUMERIC, LBM_ENOMEM, LBM_EHIP. */
int lbm_moments(lbm_t* h, double* rho, double* u, double* umix, uint8_t* active);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same fields, values and errors as
 * lbm_moments, staged through a fixed device array that the library holds on
 * each GPU it runs on until the process ends (64 MiB, 16777216 floats), so
 * the call allocates and frees nothing.  The requested fields must fit it:
 * ncomp*N floats for rho, ncomp*3*N for u, 3*N for umix and N/4 for active,
 * each rounded up to 64 (every field of two components: about 1.49 million
 * cells, e.g. 112^3; densities alone: 8.38 million); a larger request returns LBM_EINVAL with the sizes in the message.
 * The array is shared by every handle on the GPU and keeps the last call's
 * contents (each call writes all it reads back): calls that overlap on one
 * GPU, from several threads or streams, race and must be serialised by the
 * caller.  Unlike lbm_moments it does not release the initial fields after
 * the first step (that happens at the next lbm_moments, lbm_sync or
 * lbm_destroy).  Synchronous.  Errors: LBM_EINVAL, LBM_ESTATE, LBM_ENUMERIC,
 * LBM_ENOMEM (pool full flag), LBM_EHIP. */
int lbm_moments_noalloc(lbm_t* h, double* rho, double* u, double* umix, uint8_t* active);

/* Same fields as lbm_moments, written as FP32 into caller-owned DEVICE
 * buffers (rho: ncomp*N, u: ncomp*3*N, umix: 3*N; any may be NULL), enqueued
 * on the handle's stream without waiting. */
int lbm_moments_device(lbm_t* h, float* rho, float* u, float* umix);

/* Counters and memory; synchronous (waits for the stream). */
int lbm_stats(lbm_t* h, lbm_stats_t* out);

/* Activation trace: up to cap pairs (step, block) written to out (2*cap
 * int32), in the order blocks were activated; returns the number of pairs
 * available (which may exceed cap) or a negative error.  step is the number
 * of completed steps when the block joined. */
int lbm_trace(lbm_t* h, int32_t* out, int32_t cap);

/* Field dumps for tests: which = LBM_DEBUG_PSI writes psi (Eq 6) as ncomp*N
 * doubles; LBM_DEBUG_FORCE writes the total force of Eq 8-9 plus body force
 * as ncomp*3*N doubles (zero at solid and boundary nodes).  Both are computed
 * from the current state exactly as the next step would. */
#define LBM_DEBUG_PSI 0
#define LBM_DEBUG_FORCE 1
int lbm_debug_fields(lbm_t* h, int which, double* out);

/* Per-kernel GPU timing.  lbm_timing_enable(h, 1) records HIP events around
 * every kernel lbm_step launches (on the handle's stream); lbm_timing_read
 * waits for the stream and returns, per kernel k < n (names from
 * lbm_kernel_name: criterion, activate, init_blocks, fused_step, propose,
 * inplace_psi, inplace_collide), the launch count and total milliseconds,
 * then resets. */
int lbm_timing_enable(lbm_t* h, int enable);

/* Work split of the step kernel (a performance setting; results are the
 * same bits for every choice).  The fused kernel of LBM_PATTERN_AB sweeps
 * each active block's planes with workgroups of one thread per column of
 * the block: planes_per_workgroup = 16 gives each block one workgroup
 * (16 cells per thread), 8 two (8 cells per thread, plus the two halo
 * planes each), 4 four.  0 (the default) chooses per step: the smallest
 * number of planes such that the active blocks, as last seen by the host,
 * times the workgroups per block stay within target_workgroups (default
 * 320, a little above one workgroup per compute unit: measured on MI355X,
 * splitting pays only while fewer blocks than compute units are active).  More workgroups per block fill the GPU when few blocks are active,
 * at the price of re-reading the halo planes.  lbm_batch.h batches use the
 * setting of their first member.  Errors: LBM_EINVAL. */
int lbm_set_split(lbm_t* h, int32_t planes_per_workgroup, int32_t target_workgroups);
int lbm_timing_read(lbm_t* h, int64_t* counts, double* total_ms, int32_t n);
const char* lbm_kernel_name(int32_t k);
#define LBM_NUM_KERNELS 7

/* Releases every resource of the handle (waits for the stream). */
int lbm_destroy(lbm_t* h);

/* Text of the last error on h (or of the last failed lbm_create when h is
 * NULL).  Valid until the next call on the same handle. */
const char* lbm_last_error(const lbm_t* h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
