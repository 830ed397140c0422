// Host runtime and C ABI of the progressive-mesh lattice Boltzmann library
// (declared in include/lbm.h).  Owns the device buffers of a handle, validates
// arguments, derives the constants of the run and enqueues the kernels of
// lbm_kernels.hip on the handle's stream.  The per-step loop never waits for
// the GPU: block counts live in device memory and every grid is sized to the
// pool capacity, with surplus workgroups exiting at once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_batch.h"
#include "lbm_internal.h"
#include "lbm_mlp.h"

using namespace lbm;

namespace {

constexpr int kTraceCap = 1 << 20;
const char* const kKernelNames[LBM_NUM_KERNELS] = {"criterion", "activate",    "init_blocks",    "fused_step",
                                                   "propose",   "inplace_psi", "inplace_collide"};

std::string g_create_error;

}  // namespace

struct lbm_handle {
  lbm_params user{};
  Params P{};
  Buffers D{};
  hipStream_t stream = nullptr;
  lbm_allocator alloc{};
  bool custom_alloc = false;
  bool geometry = false;
  int64_t step = 0;
  int rbuf = 0;
  int n_fluid_blocks = 0;
  int64_t fluid_cells = 0;
  int64_t bytes = 0;
  int64_t slot_bytes = 0;
  std::vector<uint8_t> bfluid_h;
  std::vector<uint8_t> binlet_h;  // block holds an inlet node
  std::vector<void*> owned;
  float* init_rho = nullptr;
  float* init_u = nullptr;
  int32_t* ids_dev = nullptr;
  std::vector<float> bfrac_h;     // fluid fraction per block
  float* mlp_dev = nullptr;       // proposal network parameters (LBM_MLP_NPARAMS)
  float prop_thr = 0.5f;
  bool prop_enabled = false;
  int prop_every = 1;             // the proposal runs on steps whose index is a multiple of this
  // once every block holding fluid is active the criterion has no candidates
  // left: the step then skips it (and activation), exactly
  bool mesh_complete = false;
  // once complete, the slots are put in block order (the static mesh's
  // layout) by one pass over the slot-indexed arrays
  bool repacked = false;
  bool misaligned = false;          // the caller's allocator returned memory not aligned to 256 bytes
  int32_t* nact_pinned = nullptr;  // pinned host copy of n_active
  hipEvent_t nact_ev = nullptr;
  bool nact_pending = false;
  int ids_cap = 0;
  double* mass_dev = nullptr;
  float* staging = nullptr;    // this device's copy of the static staging array (lbm_moments_noalloc)
  float* scratch_f = nullptr;  // small device scratch (rest state)
  int* scratch_i = nullptr;
  // step kernel workgroups per block: split_planes > 0 fixes the planes each
  // takes (16 / parts); 0 picks the most parts (1, 2, 4) that keep
  // n_est * parts within split_target workgroups
  int split_planes = 0;
  int split_target = 320;
  int n_est = 0;                   // active blocks, as last seen by the host (never above the truth)
  bool timing = false;
  std::vector<hipEvent_t> ev;   // pairs per launch
  std::vector<int> ev_kernel;
  int64_t t_count[LBM_NUM_KERNELS] = {};
  double t_ms[LBM_NUM_KERNELS] = {};
  std::string err;
};

namespace {

int fail(lbm_t* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_create_error = buf;
  return code;
}

#define HIP_TRY(h, call)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail((h), LBM_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void* dev_alloc(lbm_t* h, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 4;
  if (h->custom_alloc) {
    p = h->alloc.alloc(bytes, h->alloc.ctx);
    // the kernels use 16-byte accesses from the start of each buffer
    if (p && (reinterpret_cast<uintptr_t>(p) & 255u)) {
      h->alloc.free(p, h->alloc.ctx);
      p = nullptr;
      h->misaligned = true;
    }
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    h->owned.push_back(p);
    h->bytes += (int64_t)bytes;
  }
  return p;
}

// A device allocation that failed: LBM_EINVAL when the caller's allocator
// returned memory that is not aligned to 256 bytes (dev_alloc released it),
// else LBM_ENOMEM.
int alloc_failed(lbm_t* h, const char* what) {
  if (h->misaligned)
    return fail(h, LBM_EINVAL, "the allocator returned memory not aligned to 256 bytes (%s)", what);
  return fail(h, LBM_ENOMEM, "device allocation failed (%s)", what);
}

void dev_free_all(lbm_t* h) {
  for (void* p : h->owned) {
    if (h->custom_alloc)
      h->alloc.free(p, h->alloc.ctx);
    else
      (void)hipFree(p);
  }
  h->owned.clear();
}

void dev_free_one(lbm_t* h, void* p, size_t bytes) {
  for (size_t k = 0; k < h->owned.size(); ++k)
    if (h->owned[k] == p) {
      h->owned.erase(h->owned.begin() + (long)k);
      break;
    }
  if (h->custom_alloc)
    h->alloc.free(p, h->alloc.ctx);
  else
    (void)hipFree(p);
  h->bytes -= (int64_t)bytes;
}

// Peng-Robinson constants (Eq 7): Tc = (0.07780 / 0.45724) a / (b R),
// theta = [1 + kappa (1 - sqrt(T/Tc))]^2, kappa = 0.37464 + 1.54226 w - 0.26992 w^2.
void eos_constants(const lbm_params& p, double& RT, double& a_theta) {
  const double Tc = (0.07780 / 0.45724) * p.eos_a / (p.eos_b * p.eos_R);
  const double T = p.T_over_Tc * Tc;
  const double k = 0.37464 + 1.54226 * p.eos_omega - 0.26992 * p.eos_omega * p.eos_omega;
  const double s = 1.0 + k * (1.0 - std::sqrt(T / Tc));
  RT = p.eos_R * T;
  a_theta = p.eos_a * s * s;
}

double psi_host(const lbm_params& p, int a, double rho) {
  double RT, at;
  eos_constants(p, RT, at);
  const double g = p.g[a][a];
  if (g == 0.0) return 0.0;
  const double b = p.eos_b;
  const double pr = rho * RT / (1.0 - b * rho) - at * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
  const double rad = 2.0 * (pr - rho / 3.0) / (g / 3.0);
  return rad > 0.0 ? std::sqrt(rad) : 0.0;
}

const int kEx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
const int kEy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
const int kEz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

double w_host(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Non-periodic axes whose length is not a multiple of the block edge are
// rounded up to whole blocks; the padding cells are solid (section 8(c)
// reading of uneven edges: walls).
int padded(int n) { return (n + kB - 1) / kB * kB; }

// Cells a slot spans in every plane.  With a multiple of 16 blocks along x,
// the neighbours of a block along y sit 16 * k slots away, a power-of-two
// multiple of the slot's bytes, and the step kernel ran 7 % slower on such
// meshes (256^3: 1.75 against 1.63 ms); 64 cells of padding per slot (1.6 %
// more memory) remove that.  Other meshes run 1 % faster unpadded.
uint32_t slot_cells_for(const lbm_params& u) {
  const int nbx = padded(u.nx) / kB;
  return nbx % 16 == 0 ? (uint32_t)kCells + 64u : (uint32_t)kCells;
}

// Largest pool the kernels can address.  They form 32-bit byte offsets within
// the two planes of an opposite-direction pair, which hold every component of
// each link (2 * plane * ncomp * sizeof(population)), and within one mask,
// density or psi plane (4 * plane), with plane = (slots + 1) * slot_cells: the
// pool must keep both below 2^32.
int max_slots(const lbm_params& u) {
  const uint64_t lim = (uint64_t)1 << 32;
  const uint64_t fsz = u.store == LBM_STORE_F16DEV ? 2 : 4;
  const uint64_t nc = u.ncomp == 2 ? 2 : 1;
  const uint64_t pair = 2 * fsz * nc;
  const uint64_t per_slot = (uint64_t)slot_cells_for(u) * (pair > 4 ? pair : 4);
  return (int)(lim / per_slot) - 1;
}

// Device bytes of the buffers lbm_set_geometry reserves (each as dev_alloc
// rounds it), for a pool of cap slots over nb blocks and N cells.
struct GeometryLayout {
  size_t f, psi, rho, mask, uprev, per_block_i32, per_block_u8, per_slot_i32, solid, trace, init_rho, init_u;
  int64_t slot_bytes;  // bytes of one active block's slot
  int64_t total(const lbm_params& u) const {
    const bool aa = u.pattern == LBM_PATTERN_AA, f16 = u.store == LBM_STORE_F16DEV;
    return (int64_t)((aa ? 1 : 2) * f + (aa ? psi : 0) + (f16 ? 2 * rho : 0) + mask + (u.progressive ? uprev : 0) +
                     6 * per_block_i32 + per_block_u8 + 3 * per_slot_i32 + solid + trace);
  }
};

size_t at_least_4(size_t b) { return b == 0 ? 4 : b; }

GeometryLayout geometry_layout(const lbm_params& u, int cap, int nb, int64_t N) {
  const size_t plane = (size_t)(cap + 1) * slot_cells_for(u);
  const size_t fsz = u.store == LBM_STORE_F16DEV ? 2 : 4;
  const bool f16 = u.store == LBM_STORE_F16DEV, aa = u.pattern == LBM_PATTERN_AA;
  GeometryLayout L;
  L.f = at_least_4(fsz * u.ncomp * kQ * plane);
  L.psi = at_least_4(sizeof(float) * u.ncomp * plane);
  L.rho = L.psi;
  L.mask = at_least_4(sizeof(uint32_t) * plane);
  L.uprev = at_least_4(sizeof(float) * u.ncomp * 3 * plane);
  L.per_block_i32 = at_least_4(sizeof(int32_t) * (size_t)nb);
  L.per_block_u8 = at_least_4((size_t)nb);
  L.per_slot_i32 = at_least_4(sizeof(int32_t) * (size_t)cap);
  L.solid = at_least_4((size_t)N);
  L.trace = at_least_4(sizeof(int32_t) * 2 * (size_t)kTraceCap);
  L.init_rho = at_least_4(sizeof(float) * u.ncomp * (size_t)N);
  L.init_u = at_least_4(sizeof(float) * 3 * (size_t)N);
  L.slot_bytes = (int64_t)slot_cells_for(u) * ((int64_t)(aa ? 1 : 2) * fsz * u.ncomp * kQ + (f16 ? 8 * u.ncomp : 0) +
                                    (aa ? 4 * u.ncomp : 0) + 4 + (u.progressive ? 12 * u.ncomp : 0));
  return L;
}

// Per block of the padded block grid: holds a non-solid cell, holds an inlet
// node, fraction of its 4096 cells that are non-solid.  Returns the number of
// non-solid cells.
int64_t classify_blocks(const lbm_params& p, const uint8_t* solid, std::vector<uint8_t>& bfluid,
                        std::vector<uint8_t>& binlet, std::vector<float>& bfrac) {
  const int nbx = padded(p.nx) / kB, nby = padded(p.ny) / kB, nbz = padded(p.nz) / kB;
  const int nb = nbx * nby * nbz;
  bfluid.assign(nb, 0);
  binlet.assign(nb, 0);
  bfrac.assign(nb, 0.0f);
  int64_t cells = 0;
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const int64_t n = x + (int64_t)p.nx * (y + (int64_t)p.ny * z);
        if (solid && solid[n]) continue;
        const int b = x / kB + nbx * (y / kB + nby * (z / kB));
        bfluid[b] = 1;
        bfrac[b] += 1.0f / (float)kCells;
        cells++;
        const bool on[6] = {x == 0, x == p.nx - 1, y == 0, y == p.ny - 1, z == 0, z == p.nz - 1};
        for (int f = 0; f < 6; ++f)
          if (on[f] && p.bc[f] == LBM_BC_INLET) binlet[b] = 1;
      }
  return cells;
}

int pool_capacity(const lbm_params& p, int n_fluid_blocks, int nb) {
  int cap = p.pool_blocks > 0 ? p.pool_blocks : n_fluid_blocks;
  if (cap > nb) cap = nb;
  if (cap < 1) cap = 1;
  return cap;
}

// Bytes lbm_create reserves before any geometry.
constexpr int64_t kCreateBytes = sizeof(float) * 128 + sizeof(int) * 4 + sizeof(double) * 4 +
                                 sizeof(int32_t) * kNumCtrl + sizeof(unsigned long long) * 4;

int validate(const lbm_params* p) {
  if (!p) return fail(nullptr, LBM_EINVAL, "params is NULL");
  if (p->block != kB) return fail(nullptr, LBM_EINVAL, "block must be 16 (got %d)", p->block);
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0)
    return fail(nullptr, LBM_EINVAL, "nx, ny, nz must be positive (got %d %d %d)", p->nx, p->ny, p->nz);
  {
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int d = 0; d < 3; ++d)
      if (p->bc[2 * d] == LBM_BC_PERIODIC && n[d] % kB)
        return fail(nullptr, LBM_EINVAL,
                    "a periodic axis must be a multiple of 16 (axis %d has %d cells); only non-periodic axes "
                    "are padded with solid cells", d, n[d]);
  }
  if ((int64_t)padded(p->nx) * padded(p->ny) * padded(p->nz) > (int64_t)1 << 31)
    return fail(nullptr, LBM_EINVAL, "lattice larger than 2^31 cells (after padding to whole blocks)");
  if (p->ncomp != 1 && p->ncomp != 2) return fail(nullptr, LBM_EINVAL, "ncomp must be 1 or 2 (got %d)", p->ncomp);
  if (p->shell_width < 1 || p->shell_width > kB / 2)
    return fail(nullptr, LBM_EINVAL, "shell_width must be in 1..8 (got %d)", p->shell_width);
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] < 0 || p->bc[f] > 3) return fail(nullptr, LBM_EINVAL, "bc[%d] invalid (%d)", f, p->bc[f]);
  for (int d = 0; d < 3; ++d)
    if ((p->bc[2 * d] == LBM_BC_PERIODIC) != (p->bc[2 * d + 1] == LBM_BC_PERIODIC))
      return fail(nullptr, LBM_EINVAL, "faces %d and %d: periodic must be set on both or neither", 2 * d, 2 * d + 1);
  if (p->store != LBM_STORE_F32 && p->store != LBM_STORE_F16DEV)
    return fail(nullptr, LBM_EINVAL, "store must be LBM_STORE_F32 or LBM_STORE_F16DEV (got %d)", p->store);
  if (p->progressive != 0 && p->progressive != 1) return fail(nullptr, LBM_EINVAL, "progressive must be 0 or 1");
  if (p->pool_blocks < 0) return fail(nullptr, LBM_EINVAL, "pool_blocks must be >= 0");
  if (p->store == LBM_STORE_F32 || p->store == LBM_STORE_F16DEV) {
    const int lim = max_slots(*p);
    if (p->pool_blocks > lim)
      return fail(nullptr, LBM_EINVAL, "pool_blocks %d exceeds the %d block slots the kernels can address with this "
                  "store and component count", p->pool_blocks, lim);
  }
  if (p->pattern != LBM_PATTERN_AB && p->pattern != LBM_PATTERN_AA)
    return fail(nullptr, LBM_EINVAL, "pattern must be LBM_PATTERN_AB or LBM_PATTERN_AA");
  for (int a = 0; a < p->ncomp; ++a) {
    if (!(p->tau[a] > 0.5)) return fail(nullptr, LBM_EINVAL, "tau[%d] must exceed 0.5 (got %g)", a, p->tau[a]);
    if (!(p->bg_rho[a] > 0.0)) return fail(nullptr, LBM_EINVAL, "bg_rho[%d] must be positive", a);
  }
  if (!(p->eos_b > 0.0) || !(p->eos_R > 0.0) || !(p->eos_a > 0.0) || !(p->T_over_Tc > 0.0))
    return fail(nullptr, LBM_EINVAL, "equation of state constants must be positive");
  if (p->ncomp == 2 && p->g[0][1] != p->g[1][0]) return fail(nullptr, LBM_EINVAL, "g[0][1] must equal g[1][0]");
  if (!(p->S >= 0.0)) return fail(nullptr, LBM_EINVAL, "S must be >= 0");
  return LBM_OK;
}

int check_device_flags(lbm_t* h) {
  int32_t ctrl[kNumCtrl];
  HIP_TRY(h, hipMemcpy(ctrl, h->D.ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
  h->n_est = ctrl[kNActive];
  if (ctrl[kNumeric]) return fail(h, LBM_ENUMERIC, "a density became non-positive or non-finite");
  if (ctrl[kPoolFull])
    return fail(h, LBM_ENOMEM, "block pool full (%d slots); raise pool_blocks", h->P.capacity);
  return LBM_OK;
}

bool in_place(const lbm_t* h) { return h->user.pattern == LBM_PATTERN_AA; }

// Workgroups per block of the fused step kernel for about n active blocks.
int step_parts(int split_planes, int split_target, int n) {
  if (split_planes > 0) return kB / split_planes;
  if (n < 1) n = 1;
  int parts = 1;
  while (parts < 4 && (int64_t)n * parts * 2 <= split_target) parts *= 2;
  return parts;
}

// Where the populations of the current state are read (ReadMode).
int read_mode(const lbm_t* h) {
  if (h->step == 0) return kRdOwn;
  if (!in_place(h)) return kRdPull;
  return (h->step & 1) ? kRdAAOdd : kRdAAEven;
}

// How blocks that join before the current step are initialised (InitMode).
int init_mode(const lbm_t* h) {
  if (!in_place(h) || h->step == 0) return kInitNatural;
  return (h->step & 1) ? kInitSwapped : kInitStash;
}

int sync(lbm_t* h) {
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (h->step > 0 && h->init_rho) {
    const int64_t N = (int64_t)h->P.nx * h->P.ny * h->P.nz;
    dev_free_one(h, h->init_rho, sizeof(float) * h->P.ncomp * N);
    h->init_rho = nullptr;
    h->D.init_rho = nullptr;
    if (h->init_u) {
      dev_free_one(h, h->init_u, sizeof(float) * 3 * N);
      h->init_u = nullptr;
      h->D.init_u = nullptr;
    }
  }
  return check_device_flags(h);
}

// Timed launch helper: records events around the launch when timing is on.
template <typename Fn>
int timed(lbm_t* h, int kernel, Fn&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (h->timing) {
    HIP_TRY(h, hipEventCreate(&a));
    HIP_TRY(h, hipEventCreate(&b));
    HIP_TRY(h, hipEventRecord(a, h->stream));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return fail(h, LBM_EHIP, "launch of %s: %s", kKernelNames[kernel], hipGetErrorString(e));
  if (h->timing) {
    HIP_TRY(h, hipEventRecord(b, h->stream));
    h->ev.push_back(a);
    h->ev.push_back(b);
    h->ev_kernel.push_back(kernel);
  }
  return LBM_OK;
}

int collect_timing(lbm_t* h) {
  for (size_t k = 0; k < h->ev_kernel.size(); ++k) {
    float ms = 0.0f;
    HIP_TRY(h, hipEventSynchronize(h->ev[2 * k + 1]));
    HIP_TRY(h, hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]));
    h->t_ms[h->ev_kernel[k]] += ms;
    h->t_count[h->ev_kernel[k]] += 1;
    (void)hipEventDestroy(h->ev[2 * k]);
    (void)hipEventDestroy(h->ev[2 * k + 1]);
  }
  h->ev.clear();
  h->ev_kernel.clear();
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_create(const lbm_params* p, void* stream, const lbm_allocator* alloc, lbm_t** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, LBM_EINVAL, "allocator needs alloc and free");
  lbm_t* h = new lbm_handle();
  h->user = *p;
  h->stream = (hipStream_t)stream;
  if (alloc) {
    h->alloc = *alloc;
    h->custom_alloc = true;
  }
  Params& P = h->P;
  P.nx = p->nx;
  P.ny = p->ny;
  P.nz = p->nz;
  P.nbx = padded(p->nx) / kB;
  P.slot_cells = slot_cells_for(*p);
  P.nby = padded(p->ny) / kB;
  P.nbz = padded(p->nz) / kB;
  P.nb = P.nbx * P.nby * P.nbz;
  P.ncomp = p->ncomp;
  P.shell = p->shell_width;
  for (int f = 0; f < 6; ++f) P.bc[f] = p->bc[f];
  P.trace_cap = kTraceCap;
  P.store = p->store;
  P.s_zero = p->S == 0.0 ? 1 : 0;
  P.S = (float)p->S;
  double RT, at;
  eos_constants(*p, RT, at);
  P.RT = (float)RT;
  P.a_theta = (float)at;
  P.b = (float)p->eos_b;
  P.beta = (float)p->beta;
  P.g_cross = p->ncomp == 2 ? (float)p->g[0][1] : 0.0f;
  for (int a = 0; a < kMaxComp; ++a) {
    const int aa = a < p->ncomp ? a : 0;
    P.omega[a] = (float)(1.0 / p->tau[aa]);
    P.g_self[a] = (float)p->g[aa][aa];
    for (int d = 0; d < 3; ++d) P.body[a][d] = (float)p->body[aa][d];
    P.psi_in[a] = (float)psi_host(*p, aa, p->inlet_rho[aa]);
    // inlet populations: Eq 2 at (inlet_rho, inlet_u), FP64 then rounded
    const double* u = p->inlet_u;
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < kQ; ++i) {
      const double eu = kEx[i] * u[0] + kEy[i] * u[1] + kEz[i] * u[2];
      P.f_in[a][i] = (float)(w_host(i) * p->inlet_rho[aa] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    }
  }
  // rest state on the device with the kernels' own arithmetic
  h->scratch_f = (float*)dev_alloc(h, sizeof(float) * 128);
  h->scratch_i = (int*)dev_alloc(h, sizeof(int) * 4);
  h->mass_dev = (double*)dev_alloc(h, sizeof(double) * 4);
  h->D.ctrl = (int32_t*)dev_alloc(h, sizeof(int32_t) * kNumCtrl);
  h->D.counters = (unsigned long long*)dev_alloc(h, sizeof(unsigned long long) * 4);
  if (!h->scratch_f || !h->scratch_i || !h->mass_dev || !h->D.ctrl || !h->D.counters) {
    const bool misaligned = h->misaligned;
    dev_free_all(h);
    delete h;
    if (misaligned) return fail(nullptr, LBM_EINVAL, "the allocator returned memory not aligned to 256 bytes");
    return fail(nullptr, LBM_ENOMEM, "device allocation failed");
  }
  float bg[2] = {(float)p->bg_rho[0], (float)(p->ncomp == 2 ? p->bg_rho[1] : p->bg_rho[0])};
  float res[128];
  int iters = 0;
  hipError_t e = hipMemcpyAsync(h->scratch_f + 120, bg, sizeof bg, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = launch_rest_state(P, h->scratch_f + 120, h->scratch_f, h->scratch_i, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(res, h->scratch_f, sizeof(float) * 96, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&iters, h->scratch_i, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->D.ctrl, 0, sizeof(int32_t) * kNumCtrl, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->D.counters, 0, sizeof(unsigned long long) * 4, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    std::string msg = hipGetErrorString(e);
    dev_free_all(h);
    delete h;
    return fail(nullptr, LBM_EHIP, "rest state: %s", msg.c_str());
  }
  if (iters >= 100000) {
    dev_free_all(h);
    delete h;
    return fail(nullptr, LBM_EINVAL, "the rest state did not converge (body force?)");
  }
  // the static staging array of lbm_moments_noalloc on this device (looked
  // up once per device with that device current)
  e = static_staging(&h->staging);
  if (e != hipSuccess) {
    std::string msg = hipGetErrorString(e);
    dev_free_all(h);
    delete h;
    return fail(nullptr, LBM_EHIP, "static staging lookup: %s", msg.c_str());
  }
  for (int a = 0; a < kMaxComp; ++a) {
    const int aa = a < p->ncomp ? a : 0;
    for (int i = 0; i < kQ; ++i) {
      uint32_t bits;
      std::memcpy(&bits, &res[aa * kQ + i], 4);
      P.f_rest_bits[a][i] = bits;
      P.f_rest[a][i] = res[2 * kQ + aa * kQ + i];
    }
    P.rho_ref_rest[a] = res[4 * kQ + aa];
    P.rho_rest[a] = res[4 * kQ + 2 + aa];
    P.psi_rest[a] = res[4 * kQ + 4 + aa];
  }
  *out = h;
  return LBM_OK;
}

int lbm_plan_bytes(const lbm_params* p, const uint8_t* solid, int64_t* bytes) {
  g_create_error.clear();
  if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
  *bytes = 0;
  const int rc = validate(p);
  if (rc) return rc;
  std::vector<uint8_t> bfluid, binlet;
  std::vector<float> bfrac;
  classify_blocks(*p, solid, bfluid, binlet, bfrac);
  int n_fluid = 0;
  for (uint8_t v : bfluid) n_fluid += v;
  const int nb = (int)bfluid.size();
  const int cap = pool_capacity(*p, n_fluid, nb);
  if (cap > max_slots(*p))
    return fail(nullptr, LBM_EINVAL, "%d block slots needed, but the kernels address at most %d with this store", cap,
                max_slots(*p));
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  *bytes = kCreateBytes + geometry_layout(*p, cap, nb, N).total(*p);
  return LBM_OK;
}

int lbm_set_geometry(lbm_t* h, const uint8_t* solid, const double* rho0, const double* u0) {
  if (!h) return LBM_EINVAL;
  if (h->geometry) return fail(h, LBM_ESTATE, "lbm_set_geometry called twice");
  Params& P = h->P;
  Buffers& D = h->D;
  const int64_t N = (int64_t)P.nx * P.ny * P.nz;
  // block classification on the host
  h->fluid_cells = classify_blocks(h->user, solid, h->bfluid_h, h->binlet_h, h->bfrac_h);
  h->n_fluid_blocks = 0;
  for (int b = 0; b < P.nb; ++b) h->n_fluid_blocks += h->bfluid_h[b];
  const int cap = pool_capacity(h->user, h->n_fluid_blocks, P.nb);
  if (cap > max_slots(h->user))
    return fail(h, LBM_EINVAL,
                "%d block slots needed, but the kernels address at most %d with this store (32-bit offsets "
                "within a pair of population planes); use the FP16-deviation store or a smaller lattice",
                cap, max_slots(h->user));
  P.capacity = cap;
  P.slot_cells = slot_cells_for(h->user);
  P.plane = (uint32_t)((int64_t)(cap + 1) * P.slot_cells);
  const GeometryLayout L = geometry_layout(h->user, cap, P.nb, N);
  const bool f16 = h->user.store == LBM_STORE_F16DEV;
  const bool aa = in_place(h);
  D.f[0] = dev_alloc(h, L.f);
  D.f[1] = aa ? D.f[0] : dev_alloc(h, L.f);
  D.psi = aa ? (float*)dev_alloc(h, L.psi) : nullptr;
  D.rho[0] = f16 ? (float*)dev_alloc(h, L.rho) : nullptr;
  D.rho[1] = f16 ? (float*)dev_alloc(h, L.rho) : nullptr;
  D.mask = (uint32_t*)dev_alloc(h, L.mask);
  D.uprev = h->user.progressive ? (float*)dev_alloc(h, L.uprev) : nullptr;
  D.block_slot = (int32_t*)dev_alloc(h, L.per_block_i32);
  D.slot_block = (int32_t*)dev_alloc(h, L.per_slot_i32);
  D.order = (int32_t*)dev_alloc(h, L.per_slot_i32);
  D.frontier = (int32_t*)dev_alloc(h, L.per_slot_i32);
  D.bfluid = (uint8_t*)dev_alloc(h, L.per_block_u8);
  D.solid = (uint8_t*)dev_alloc(h, L.solid);
  D.request = (int32_t*)dev_alloc(h, L.per_block_i32);
  D.expose = (int32_t*)dev_alloc(h, L.per_block_i32);
  D.act_step = (int32_t*)dev_alloc(h, L.per_block_i32);
  D.bfrac = (float*)dev_alloc(h, L.per_block_i32);
  D.cand = (int32_t*)dev_alloc(h, L.per_block_i32);
  D.trace = (int32_t*)dev_alloc(h, L.trace);
  if (!D.f[0] || !D.f[1] || (aa && !D.psi) || (f16 && (!D.rho[0] || !D.rho[1])) || !D.mask ||
      (h->user.progressive && !D.uprev) || !D.block_slot ||
      !D.slot_block || !D.order || !D.frontier || !D.bfluid || !D.solid || !D.request || !D.expose || !D.act_step || !D.bfrac ||
      !D.cand || !D.trace) {
    return alloc_failed(h, "block pool");
  }
  h->slot_bytes = L.slot_bytes;
  // initial fields, FP32; NaN marks a component of a cell at the rest state
  if (rho0 || u0) {
    std::vector<float> r((size_t)P.ncomp * N), u(u0 ? (size_t)3 * N : 0);
    const float nan = std::nanf("");
    for (int a = 0; a < P.ncomp; ++a)
      for (int64_t n = 0; n < N; ++n) {
        const double rv = rho0 ? rho0[a * N + n] : h->user.bg_rho[a];
        const bool zero_u = !u0 || (u0[n] == 0.0 && u0[N + n] == 0.0 && u0[2 * N + n] == 0.0);
        r[a * N + n] = (rv == h->user.bg_rho[a] && zero_u) ? nan : (float)rv;
      }
    if (u0)
      for (int64_t k = 0; k < 3 * N; ++k) u[k] = (float)u0[k];
    h->init_rho = (float*)dev_alloc(h, L.init_rho);
    if (!h->init_rho) return alloc_failed(h, "initial fields");
    HIP_TRY(h, hipMemcpy(h->init_rho, r.data(), sizeof(float) * r.size(), hipMemcpyHostToDevice));
    D.init_rho = h->init_rho;
    if (u0) {
      h->init_u = (float*)dev_alloc(h, L.init_u);
      if (!h->init_u) return alloc_failed(h, "initial fields");
      HIP_TRY(h, hipMemcpy(h->init_u, u.data(), sizeof(float) * u.size(), hipMemcpyHostToDevice));
      D.init_u = h->init_u;
    }
  }
  std::vector<uint8_t> sol((size_t)N, 0);
  if (solid)
    for (int64_t n = 0; n < N; ++n) sol[n] = solid[n] ? 1 : 0;
  HIP_TRY(h, hipMemcpy(D.solid, sol.data(), (size_t)N, hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(D.bfluid, h->bfluid_h.data(), P.nb, hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemsetAsync(D.request, 0, sizeof(int32_t) * P.nb, h->stream));
  HIP_TRY(h, hipMemsetAsync(D.expose, 0, sizeof(int32_t) * P.nb, h->stream));
  HIP_TRY(h, hipMemsetAsync(D.act_step, 0xFF, sizeof(int32_t) * P.nb, h->stream));  // -1: never activated
  if (h->user.progressive) {
    HIP_TRY(h, hipHostMalloc((void**)&h->nact_pinned, sizeof(int32_t), hipHostMallocDefault));
    *h->nact_pinned = 0;
    HIP_TRY(h, hipEventCreateWithFlags(&h->nact_ev, hipEventDisableTiming));
  }
  HIP_TRY(h, hipMemcpy(D.bfrac, h->bfrac_h.data(), sizeof(float) * P.nb, hipMemcpyHostToDevice));
  // the rest slot, in both population buffers (in place: the one buffer,
  // holding the rest state as post-collision values, opposite pairs swapped)
  for (int b = 0; b < (aa ? 1 : 2); ++b) {
    hipError_t e = launch_init_slots(P, D, b, P.capacity, 1, false, false, h->stream,
                                     aa ? kInitSwapped : kInitNatural, -1);
    if (e != hipSuccess) return fail(h, LBM_EHIP, "init rest slot: %s", hipGetErrorString(e));
  }
  std::vector<int32_t> bslot(P.nb, -1), sblock;
  if (!h->user.progressive) {
    for (int b = 0; b < P.nb; ++b)
      if (h->bfluid_h[b]) {
        bslot[b] = (int32_t)sblock.size();
        sblock.push_back(b);
      }
    if ((int)sblock.size() > cap) return fail(h, LBM_ENOMEM, "pool_blocks smaller than the blocks holding fluid");
  }
  HIP_TRY(h, hipMemcpy(D.block_slot, bslot.data(), sizeof(int32_t) * P.nb, hipMemcpyHostToDevice));
  if (!sblock.empty()) {
    HIP_TRY(h, hipMemcpy(D.slot_block, sblock.data(), sizeof(int32_t) * sblock.size(), hipMemcpyHostToDevice));
    // static mesh: slots were assigned in block order
    std::vector<int32_t> ord(sblock.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int32_t)k;
    HIP_TRY(h, hipMemcpy(D.order, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice));
  }
  int32_t ctrl[kNumCtrl] = {0};
  ctrl[kNActive] = (int32_t)sblock.size();
  h->n_est = (int)sblock.size();
  HIP_TRY(h, hipMemcpy(D.ctrl, ctrl, sizeof ctrl, hipMemcpyHostToDevice));
  if (!sblock.empty()) {
    hipError_t e = launch_init_slots(P, D, 0, 0, (int)sblock.size(), false, true, h->stream);
    if (e != hipSuccess) return fail(h, LBM_EHIP, "init blocks: %s", hipGetErrorString(e));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->geometry = true;
  return LBM_OK;
}

int lbm_activate(lbm_t* h, const int32_t* ids, int32_t n) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_activate before lbm_set_geometry");
  if (n < 0 || (n > 0 && !ids)) return fail(h, LBM_EINVAL, "bad block list");
  if (n == 0) return LBM_OK;
  for (int k = 0; k < n; ++k)
    if (ids[k] < 0 || ids[k] >= h->P.nb) return fail(h, LBM_EINVAL, "block id %d out of range", ids[k]);
  // mark requests on the host side of a small upload, then compact on the GPU
  std::vector<int32_t> req(h->P.nb, 0);
  HIP_TRY(h, hipMemcpyAsync(req.data(), h->D.request, sizeof(int32_t) * h->P.nb, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (int k = 0; k < n; ++k) req[ids[k]] = 1;
  HIP_TRY(h, hipMemcpy(h->D.request, req.data(), sizeof(int32_t) * h->P.nb, hipMemcpyHostToDevice));
  const int32_t pending = 1;
  HIP_TRY(h, hipMemcpy(h->D.ctrl + kPending, &pending, sizeof pending, hipMemcpyHostToDevice));
  hipError_t e = launch_activate(h->P, h->D, (int)h->step, h->stream);
  if (e == hipSuccess)
    e = launch_init_slots(h->P, h->D, h->rbuf, 0, 0, true, h->step == 0, h->stream, init_mode(h), (int)h->step);
  if (e != hipSuccess) return fail(h, LBM_EHIP, "activation: %s", hipGetErrorString(e));
  return sync(h);
}

namespace {
// A progressive run starts from blocks the caller activated: every block with
// inlet nodes must be among them (the criterion only looks at active blocks).
int check_inlet_blocks(lbm_t* h) {
  const Params& P = h->P;
  std::vector<int32_t> bslot(P.nb);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemcpy(bslot.data(), h->D.block_slot, sizeof(int32_t) * P.nb, hipMemcpyDeviceToHost));
  for (int b = 0; b < P.nb; ++b)
    if (h->binlet_h[b] && bslot[b] < 0)
      return fail(h, LBM_EINVAL, "block %d holds inlet nodes but is not active at t = 0", b);
  return LBM_OK;
}
}  // namespace

int lbm_step(lbm_t* h, int32_t nsteps) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_step before lbm_set_geometry");
  if (nsteps < 0) return fail(h, LBM_EINVAL, "nsteps < 0");
  const Params& P = h->P;
  if (h->step == 0 && nsteps > 0 && h->user.progressive) {
    const int rc = check_inlet_blocks(h);
    if (rc) return rc;
  }
  const bool aa = in_place(h);
  for (int32_t k = 0; k < nsteps; ++k) {
    const bool pull = h->step > 0;
    const int rd = read_mode(h);
    const int rb = h->rbuf;
    int rc;
    if (h->user.progressive && h->nact_pending && hipEventQuery(h->nact_ev) == hipSuccess) {
      h->nact_pending = false;
      if (*h->nact_pinned > h->n_est) h->n_est = *h->nact_pinned;
      if (*h->nact_pinned >= h->n_fluid_blocks) h->mesh_complete = true;
      if (h->mesh_complete && !h->repacked) {
        // slots in block order from here on: the layout of the static mesh
        const hipError_t e = launch_repack(P, h->D, rb, aa, h->stream);
        if (e != hipSuccess) return fail(h, LBM_EHIP, "repack: %s", hipGetErrorString(e));
        h->repacked = true;
      }
    }
    if (h->user.progressive && !h->mesh_complete) {
      // criterion and leak checks on the frontier, then the requested blocks
      // join this step
      const int flags = h->step == 0 ? (kCritRecord | kCritExposure)
                                     : (kCritRecord | kCritEval | kCritExposure | kCritEmission);
      rc = timed(h, 0, [&] { return launch_criterion(P, h->D, rb, rd, flags, h->stream); });
      if (rc) return rc;
      if (h->prop_enabled && h->step % h->prop_every == 0) {
        // the learned proposal requests more blocks, ahead of the criterion
        rc = timed(h, 4, [&] {
          hipError_t e = launch_candidates(P, h->D, h->stream);
          if (e == hipSuccess)
            e = launch_propose(P, h->D, rb, rd, (int)h->step, h->mlp_dev, h->prop_thr, nullptr, nullptr, 0,
                               h->stream);
          return e;
        });
        if (rc) return rc;
      }
      rc = timed(h, 1, [&] { return launch_activate(P, h->D, (int)h->step, h->stream); });
      if (rc) return rc;
      rc = timed(h, 2, [&] {
        return launch_init_slots(P, h->D, rb, 0, 0, true, false, h->stream, init_mode(h), (int)h->step);
      });
      if (rc) return rc;
    }
    if (aa) {
      rc = timed(h, 5, [&] { return launch_inplace_psi(P, h->D, rb, rd, h->stream); });
      if (rc) return rc;
      rc = timed(h, 6, [&] { return launch_inplace_collide(P, h->D, rb, rd, h->stream); });
      if (rc) return rc;
    } else {
      const int parts = step_parts(h->split_planes, h->split_target, h->n_est);
      rc = timed(h, 3, [&] { return launch_fused(P, h->D, rb, pull, parts, h->stream); });
      if (rc) return rc;
    }
    if (h->user.progressive && !h->mesh_complete && !h->nact_pending && h->step % 16 == 0 && h->nact_pinned) {
      HIP_TRY(h, hipMemcpyAsync(h->nact_pinned, h->D.ctrl + kNActive, sizeof(int32_t), hipMemcpyDeviceToHost,
                                h->stream));
      HIP_TRY(h, hipEventRecord(h->nact_ev, h->stream));
      h->nact_pending = true;
    }
    h->rbuf ^= 1;  // in place: both indices name the one population buffer
    h->step++;
  }
  return LBM_OK;
}

int lbm_sync(lbm_t* h) {
  if (!h) return LBM_EINVAL;
  return sync(h);
}

int lbm_moments_device(lbm_t* h, float* rho, float* u, float* umix) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_moments before lbm_set_geometry");
  hipError_t e = launch_export(h->P, h->D, h->rbuf, read_mode(h), rho, u, umix, h->stream);
  if (e != hipSuccess) return fail(h, LBM_EHIP, "export: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_moments(lbm_t* h, double* rho, double* u, double* umix, uint8_t* active) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_moments before lbm_set_geometry");
  int rc = sync(h);
  if (rc) return rc;
  const Params& P = h->P;
  const int64_t N = (int64_t)P.nx * P.ny * P.nz;
  const size_t nr = (size_t)P.ncomp * N, nu = (size_t)P.ncomp * 3 * N, nm = (size_t)3 * N;
  float* d_r = rho ? (float*)dev_alloc(h, sizeof(float) * nr) : nullptr;
  float* d_u = u ? (float*)dev_alloc(h, sizeof(float) * nu) : nullptr;
  float* d_m = umix ? (float*)dev_alloc(h, sizeof(float) * nm) : nullptr;
  if ((rho && !d_r) || (u && !d_u) || (umix && !d_m)) {
    if (d_r) dev_free_one(h, d_r, sizeof(float) * nr);
    if (d_u) dev_free_one(h, d_u, sizeof(float) * nu);
    if (d_m) dev_free_one(h, d_m, sizeof(float) * nm);
    return alloc_failed(h, "moments");
  }
  rc = lbm_moments_device(h, d_r, d_u, d_m);
  std::vector<float> tmp;
  auto fetch = [&](float* d, double* out, size_t n) -> int {
    if (!d) return LBM_OK;
    tmp.resize(n);
    HIP_TRY(h, hipMemcpyAsync(tmp.data(), d, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (size_t k = 0; k < n; ++k) out[k] = (double)tmp[k];
    return LBM_OK;
  };
  if (!rc) rc = fetch(d_r, rho, nr);
  if (!rc) rc = fetch(d_u, u, nu);
  if (!rc) rc = fetch(d_m, umix, nm);
  if (d_r) dev_free_one(h, d_r, sizeof(float) * nr);
  if (d_u) dev_free_one(h, d_u, sizeof(float) * nu);
  if (d_m) dev_free_one(h, d_m, sizeof(float) * nm);
  if (rc) return rc;
  if (active) {
    std::vector<int32_t> bslot(P.nb);
    HIP_TRY(h, hipMemcpy(bslot.data(), h->D.block_slot, sizeof(int32_t) * P.nb, hipMemcpyDeviceToHost));
    for (int z = 0; z < P.nz; ++z)
      for (int y = 0; y < P.ny; ++y)
        for (int x = 0; x < P.nx; ++x)
          active[x + (int64_t)P.nx * (y + (int64_t)P.ny * z)] =
              bslot[x / kB + P.nbx * (y / kB + P.nby * (z / kB))] >= 0 ? 1 : 0;
  }
  return check_device_flags(h);
}

namespace {
// Widens n FP32 values to FP64 in place: the floats occupy the upper half
// of out's 8n bytes.  Ascending order reads each float before the double
// written at the same index (or a lower one) can overwrite it.
void widen_in_place(double* out, size_t n) {
  const char* src = reinterpret_cast<const char*>(out) + 4 * n;
  for (size_t k = 0; k < n; ++k) {
    float v;
    std::memcpy(&v, src + 4 * k, sizeof v);
    out[k] = (double)v;
  }
}
}  // namespace

int lbm_moments_noalloc(lbm_t* h, double* rho, double* u, double* umix, uint8_t* active) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_moments_noalloc before lbm_set_geometry");
  const Params& P = h->P;
  const size_t N = (size_t)P.nx * P.ny * P.nz;
  const size_t nr = rho ? (size_t)P.ncomp * N : 0, nu = u ? (size_t)P.ncomp * 3 * N : 0, nm = umix ? 3 * N : 0;
  const size_t na = active ? (N + 3) / 4 : 0;  // N bytes
  auto up = [](size_t n) { return (n + 63) & ~(size_t)63; };  // 256-byte aligned segments
  const size_t need = up(nr) + up(nu) + up(nm) + up(na);
  if (need > kStaticStagingFloats)
    return fail(h, LBM_EINVAL,
                "lbm_moments_noalloc: the requested fields need %zu floats of staging, the static array holds %zu "
                "(about %zu cells with every field of two components)",
                need, (size_t)kStaticStagingFloats, (size_t)kStaticStagingFloats * 4 / 45);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  int rc = check_device_flags(h);
  if (rc) return rc;
  float* next = h->staging;
  float* d_r = rho ? next : nullptr;
  next += up(nr);
  float* d_u = u ? next : nullptr;
  next += up(nu);
  float* d_m = umix ? next : nullptr;
  next += up(nm);
  uint8_t* d_a = active ? reinterpret_cast<uint8_t*>(next) : nullptr;
  // every element copied out is written first (the default fill covers the
  // whole lattice), so the array's previous contents never show
  hipError_t e = hipSuccess;
  if (rho || u || umix) e = launch_export(P, h->D, h->rbuf, read_mode(h), d_r, d_u, d_m, h->stream);
  if (e == hipSuccess && active) e = launch_active_cells(P, h->D, d_a, h->stream);
  if (e != hipSuccess) return fail(h, LBM_EHIP, "export: %s", hipGetErrorString(e));
  // FP32 fields land in the upper half of the caller's FP64 arrays
  if (rho) HIP_TRY(h, hipMemcpyAsync((char*)rho + 4 * nr, d_r, 4 * nr, hipMemcpyDeviceToHost, h->stream));
  if (u) HIP_TRY(h, hipMemcpyAsync((char*)u + 4 * nu, d_u, 4 * nu, hipMemcpyDeviceToHost, h->stream));
  if (umix) HIP_TRY(h, hipMemcpyAsync((char*)umix + 4 * nm, d_m, 4 * nm, hipMemcpyDeviceToHost, h->stream));
  if (active) HIP_TRY(h, hipMemcpyAsync(active, d_a, N, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (rho) widen_in_place(rho, nr);
  if (u) widen_in_place(u, nu);
  if (umix) widen_in_place(umix, nm);
  return LBM_OK;
}

int lbm_stats(lbm_t* h, lbm_stats_t* out) {
  if (!h || !out) return LBM_EINVAL;
  std::memset(out, 0, sizeof *out);
  int rc = LBM_OK;
  if (h->geometry) {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  int32_t ctrl[kNumCtrl] = {0};
  unsigned long long cnt[4] = {0, 0, 0, 0};
  HIP_TRY(h, hipMemcpy(ctrl, h->D.ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(cnt, h->D.counters, sizeof cnt, hipMemcpyDeviceToHost));
  out->steps = h->step;
  out->n_active = ctrl[kNActive];
  out->n_fluid_blocks = h->n_fluid_blocks;
  out->capacity = h->P.capacity;
  out->store = h->user.store;
  out->bytes_reserved = h->bytes;
  out->bytes_active = h->slot_bytes * ctrl[kNActive];
  out->leak = (int64_t)cnt[0];
  out->clamps = (int64_t)cnt[1];
  out->numeric_error = ctrl[kNumeric];
  out->pool_full = ctrl[kPoolFull];
  out->activations = ctrl[kTraceLen];
  out->repacked = h->repacked ? 1 : 0;
  out->reserved = 0;
  if (h->geometry) {
    double m[4] = {0, 0, 0, 0};
    HIP_TRY(h, hipMemsetAsync(h->mass_dev, 0, sizeof m, h->stream));
    hipError_t e = launch_mass(h->P, h->D, h->rbuf, read_mode(h), h->mass_dev, h->stream);
    if (e != hipSuccess) return fail(h, LBM_EHIP, "mass: %s", hipGetErrorString(e));
    HIP_TRY(h, hipMemcpyAsync(m, h->mass_dev, sizeof m, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const double inactive_cells = (double)h->fluid_cells - m[2];
    for (int a = 0; a < h->P.ncomp; ++a) out->mass[a] = m[a] + inactive_cells * (double)h->P.rho_rest[a];
  }
  return rc;
}

int lbm_trace(lbm_t* h, int32_t* out, int32_t cap) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return 0;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  int32_t ctrl[kNumCtrl];
  HIP_TRY(h, hipMemcpy(ctrl, h->D.ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
  int32_t n = ctrl[kTraceLen];
  int32_t avail = n < h->P.trace_cap ? n : h->P.trace_cap;
  int32_t k = avail < cap ? avail : cap;
  if (k > 0 && out) HIP_TRY(h, hipMemcpy(out, h->D.trace, sizeof(int32_t) * 2 * k, hipMemcpyDeviceToHost));
  return n;
}

int lbm_debug_fields(lbm_t* h, int which, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_debug_fields before lbm_set_geometry");
  if (which != LBM_DEBUG_PSI && which != LBM_DEBUG_FORCE) return fail(h, LBM_EINVAL, "which must be 0 or 1");
  int rc = sync(h);
  if (rc) return rc;
  const Params& P = h->P;
  const int64_t N = (int64_t)P.nx * P.ny * P.nz;
  const size_t np = (size_t)P.ncomp * N, nf = (size_t)P.ncomp * 3 * N;
  const size_t ns = (size_t)P.ncomp * P.plane;  // psi per slot
  float* d_p = (float*)dev_alloc(h, sizeof(float) * np);
  float* d_f = (float*)dev_alloc(h, sizeof(float) * nf);
  float* d_s = (float*)dev_alloc(h, sizeof(float) * ns);
  if (!d_p || !d_f || !d_s) {
    if (d_p) dev_free_one(h, d_p, sizeof(float) * np);
    if (d_f) dev_free_one(h, d_f, sizeof(float) * nf);
    if (d_s) dev_free_one(h, d_s, sizeof(float) * ns);
    return alloc_failed(h, "debug");
  }
  hipError_t e = hipMemsetAsync(d_p, 0, sizeof(float) * np, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d_f, 0, sizeof(float) * nf, h->stream);
  if (e == hipSuccess) e = launch_debug_fields(P, h->D, h->rbuf, read_mode(h), d_s, d_p, d_f, h->stream);
  std::vector<float> tmp(which == LBM_DEBUG_PSI ? np : nf);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tmp.data(), which == LBM_DEBUG_PSI ? d_p : d_f, sizeof(float) * tmp.size(),
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  dev_free_one(h, d_p, sizeof(float) * np);
  dev_free_one(h, d_f, sizeof(float) * nf);
  dev_free_one(h, d_s, sizeof(float) * ns);
  if (e != hipSuccess) return fail(h, LBM_EHIP, "debug fields: %s", hipGetErrorString(e));
  for (size_t k = 0; k < tmp.size(); ++k) out[k] = (double)tmp[k];
  return LBM_OK;
}

int lbm_timing_enable(lbm_t* h, int enable) {
  if (!h) return LBM_EINVAL;
  h->timing = enable != 0;
  return LBM_OK;
}

int lbm_set_split(lbm_t* h, int32_t planes_per_workgroup, int32_t target_workgroups) {
  if (!h) return LBM_EINVAL;
  if (planes_per_workgroup != 0 && planes_per_workgroup != 4 && planes_per_workgroup != 8 &&
      planes_per_workgroup != 16)
    return fail(h, LBM_EINVAL, "planes_per_workgroup must be 0, 4, 8 or 16 (got %d)", planes_per_workgroup);
  if (target_workgroups < 1) return fail(h, LBM_EINVAL, "target_workgroups must be positive");
  h->split_planes = planes_per_workgroup;
  h->split_target = target_workgroups;
  return LBM_OK;
}

int lbm_timing_read(lbm_t* h, int64_t* counts, double* total_ms, int32_t n) {
  if (!h) return LBM_EINVAL;
  int rc = collect_timing(h);
  if (rc) return rc;
  for (int k = 0; k < n && k < LBM_NUM_KERNELS; ++k) {
    if (counts) counts[k] = h->t_count[k];
    if (total_ms) total_ms[k] = h->t_ms[k];
    h->t_count[k] = 0;
    h->t_ms[k] = 0.0;
  }
  return LBM_OK;
}

const char* lbm_kernel_name(int32_t k) { return (k >= 0 && k < LBM_NUM_KERNELS) ? kKernelNames[k] : ""; }

int lbm_proposal_features(lbm_t* h, float* feat, int32_t* block, int32_t cap) {
  if (!h) return LBM_EINVAL;
  if (!h->geometry) return fail(h, LBM_ESTATE, "lbm_proposal_features before lbm_set_geometry");
  if (cap < 0 || (cap > 0 && (!feat || !block))) return fail(h, LBM_EINVAL, "bad feature buffers");
  hipError_t e = launch_candidates(h->P, h->D, h->stream);
  if (e == hipSuccess)
    e = launch_propose(h->P, h->D, h->rbuf, read_mode(h), (int)h->step, nullptr, 0.0f, feat, block, cap, h->stream);
  if (e != hipSuccess) return fail(h, LBM_EHIP, "proposal features: %s", hipGetErrorString(e));
  int32_t ctrl[kNumCtrl];
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemcpy(ctrl, h->D.ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
  return ctrl[kCandCount];
}

int lbm_set_proposal(lbm_t* h, const float* params, float threshold, int32_t enable) {
  if (!h) return LBM_EINVAL;
  if (enable <= 0) {
    h->prop_enabled = false;
    return LBM_OK;
  }
  if (!params) return fail(h, LBM_EINVAL, "proposal parameters missing");
  if (!h->user.progressive) return fail(h, LBM_EINVAL, "the proposal needs a progressive mesh");
  if (!h->mlp_dev) {
    h->mlp_dev = (float*)dev_alloc(h, sizeof(float) * LBM_MLP_NPARAMS);
    if (!h->mlp_dev) return alloc_failed(h, "proposal");
  }
  HIP_TRY(h, hipMemcpy(h->mlp_dev, params, sizeof(float) * LBM_MLP_NPARAMS, hipMemcpyHostToDevice));
  h->prop_thr = threshold;
  h->prop_every = enable;
  h->prop_enabled = true;
  return LBM_OK;
}

// ------------------------------------------------------------------ batch
struct lbm_batch {
  std::vector<lbm_t*> members;
  hipStream_t stream = nullptr;  // own stream: graphs cannot be captured on the null stream
  hipEvent_t done = nullptr;
  Batch B{};
  Params* P_dev = nullptr;
  Buffers* D_dev = nullptr;
  int32_t* off_dev = nullptr;
  bool progressive = false;
  bool in_place = false;                          // members use LBM_PATTERN_AA
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two steps starting at buffer parity 0 / 1
  int parts = 0;                                 // step-kernel split the graphs were captured with
  int32_t* heads = nullptr;                      // [8] queue heads of the persistent step kernel
  bool persistent = false;                       // step kernel as a resident work-taking grid
  bool graph_persistent = false;                 // schedule the graphs were captured with
};

namespace {
int batch_fail(const char* what, hipError_t e) {
  g_create_error = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}
}  // namespace

int lbm_batch_create(lbm_t* const* hs, int32_t n, lbm_batch_t** out) {
  if (!hs || n < 1 || !out) return fail(nullptr, LBM_EINVAL, "batch: NULL argument or n < 1");
  *out = nullptr;
  lbm_t* h0 = hs[0];
  for (int i = 0; i < n; ++i) {
    lbm_t* h = hs[i];
    if (!h) return fail(nullptr, LBM_EINVAL, "batch: member %d is NULL", i);
    if (!h->geometry) return fail(nullptr, LBM_ESTATE, "batch: member %d has no geometry", i);
    if (h->P.store != h0->P.store || h->P.ncomp != h0->P.ncomp || h->user.progressive != h0->user.progressive ||
        h->user.pattern != h0->user.pattern)
      return fail(nullptr, LBM_EINVAL, "batch: member %d differs in store, ncomp, mesh mode or pattern", i);
    if (h->step != h0->step || h->rbuf != h0->rbuf)
      return fail(nullptr, LBM_EINVAL, "batch: member %d is at another step", i);
    if (h->prop_enabled) return fail(nullptr, LBM_EINVAL, "batch: member %d has the proposal enabled", i);
    // one member twice would have two workgroups update its blocks and
    // tables unsynchronised, and would advance its step count twice
    for (int j = 0; j < i; ++j)
      if (hs[j] == h) return fail(nullptr, LBM_EINVAL, "batch: members %d and %d are the same handle", j, i);
  }
  lbm_batch* b = new lbm_batch();
  b->members.assign(hs, hs + n);
  b->progressive = h0->user.progressive != 0;
  b->in_place = in_place(h0);
  std::vector<Params> P(n);
  std::vector<Buffers> D(n);
  int total = 0;
  for (int i = 0; i < n; ++i) {
    P[i] = hs[i]->P;
    D[i] = hs[i]->D;
    total += hs[i]->P.capacity;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&b->P_dev, sizeof(Params) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->D_dev, sizeof(Buffers) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->off_dev, sizeof(int32_t) * (n + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->heads, sizeof(int32_t) * 8);
  if (e == hipSuccess) e = hipMemset(b->heads, 0, sizeof(int32_t) * 8);
  if (e == hipSuccess) e = hipMemcpy(b->P_dev, P.data(), sizeof(Params) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->D_dev, D.data(), sizeof(Buffers) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    lbm_batch_destroy(b);
    return batch_fail("batch create", e);
  }
  b->B = Batch{b->P_dev, b->D_dev, b->off_dev, n, total, b->heads};
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch_t* b, int32_t nsteps, int32_t use_graph) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (nsteps == 0) return LBM_OK;
  lbm_t* h0 = b->members[0];
  for (lbm_t* h : b->members)
    if (h->step != h0->step || h->rbuf != h0->rbuf) return LBM_ESTATE;
  const Params& P0 = h0->P;
  if (h0->step == 0 && b->progressive)
    for (lbm_t* h : b->members) {
      const int rc = check_inlet_blocks(h);
      if (rc) return rc;
    }
  // order after the members' queued work; the device step counters follow
  // the members' step counts
  for (lbm_t* h : b->members) {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int32_t st = (int32_t)h->step;
    HIP_TRY(h, hipMemcpy(h->D.ctrl + kStepCount, &st, sizeof st, hipMemcpyHostToDevice));
    int32_t na = 0;
    HIP_TRY(h, hipMemcpy(&na, h->D.ctrl + kNActive, sizeof na, hipMemcpyDeviceToHost));
    h->n_est = na;
  }
  hipError_t e = launch_batch_offsets(b->B, P0, b->stream);
  int64_t step = h0->step;
  int rbuf = h0->rbuf;
  int32_t k = 0;
  int n_sum = 0;
  for (lbm_t* h : b->members) n_sum += h->n_est;
  const int parts = step_parts(h0->split_planes, h0->split_target, n_sum);
  if (parts != b->parts || b->persistent != b->graph_persistent) {  // captured for another schedule
    for (hipGraphExec_t& g : b->graph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
    b->parts = parts;
    b->graph_persistent = b->persistent;
  }
  auto eager = [&](bool first) {
    const hipError_t r =
        launch_batch_step(b->B, P0, rbuf, first, b->progressive, b->in_place, parts, b->persistent, b->stream);
    if (r == hipSuccess) {
      rbuf ^= 1;
      step++;
      k++;
    }
    return r;
  };
  if (e == hipSuccess && step == 0) e = eager(true);
  while (e == hipSuccess && k + 2 <= nsteps && use_graph) {
    hipGraphExec_t& g = b->graph[rbuf];
    if (!g) {
      hipGraph_t graph = nullptr;
      e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess)
        e = launch_batch_step(b->B, P0, rbuf, false, b->progressive, b->in_place, parts, b->persistent, b->stream);
      if (e == hipSuccess)
        e = launch_batch_step(b->B, P0, rbuf ^ 1, false, b->progressive, b->in_place, parts, b->persistent,
                              b->stream);
      hipError_t ec = hipStreamEndCapture(b->stream, &graph);
      if (e == hipSuccess) e = ec;
      if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) break;
    }
    e = hipGraphLaunch(g, b->stream);
    if (e == hipSuccess) {
      step += 2;
      k += 2;
    }
  }
  while (e == hipSuccess && k < nsteps) e = eager(false);
  // the members advance by the steps actually enqueued (all of them unless a
  // launch failed)
  const hipError_t e_steps = e;
  e = hipEventRecord(b->done, b->stream);
  for (lbm_t* h : b->members) {
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, b->done, 0);
    h->step += k;
    h->rbuf ^= (k & 1);
  }
  if (e_steps != hipSuccess) e = e_steps;
  if (e != hipSuccess) return fail(h0, LBM_EHIP, "batch step: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_batch_schedule(lbm_batch_t* b, int32_t persistent) {
  if (!b || (persistent != 0 && persistent != 1)) return LBM_EINVAL;
  b->persistent = persistent != 0;
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch_t* b) {
  if (!b) return LBM_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipGraphExec_t g : b->graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (b->P_dev) (void)hipFree(b->P_dev);
  if (b->D_dev) (void)hipFree(b->D_dev);
  if (b->off_dev) (void)hipFree(b->off_dev);
  if (b->heads) (void)hipFree(b->heads);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBM_OK;
}

int lbm_destroy(lbm_t* h) {
  if (!h) return LBM_OK;
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->nact_ev) (void)hipEventDestroy(h->nact_ev);
  if (h->nact_pinned) (void)hipHostFree(h->nact_pinned);
  dev_free_all(h);
  delete h;
  return LBM_OK;
}

const char* lbm_last_error(const lbm_t* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
