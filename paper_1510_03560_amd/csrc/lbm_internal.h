// Internal interface between the host runtime (lbm_api.cpp) and the HIP
// kernels (lbm_kernels.hip) of the progressive-mesh lattice Boltzmann library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;          // D3Q19 directions
constexpr int kB = 16;          // block edge
constexpr int kCells = kB * kB * kB;
constexpr int kMaxComp = 2;

// Cell kinds, stored in bits 24..25 of the per-cell mask word.
enum CellKind : uint32_t { kFluid = 0, kSolid = 1, kInlet = 2, kOutlet = 3 };
constexpr int kKindShift = 24;

// Where a kernel reads the populations f(t) arriving at a cell.
//  kRdOwn:    at the cell itself, plane i (the initial state, before the first step)
//  kRdPull:   two buffers: f*_i(x - e_i) at (x - e_i, plane i) of the buffer read
//  kRdAAEven: one buffer updated in place, after an even number (> 0) of
//             steps: at (x, plane i), where the last step streamed them
//  kRdAAOdd:  one buffer, after an odd number of steps: f*_i(x - e_i) at
//             (x - e_i, plane of the opposite direction), where the last
//             step left it
// A bounced link reads the cell's own post-collision value of the opposite
// direction in every mode.
enum ReadMode : int { kRdOwn = 0, kRdPull = 1, kRdAAEven = 2, kRdAAOdd = 3 };

// How k_init writes the populations of the slots it initialises.
//  kInitNatural: f(t) at (x, plane i) (two buffers; in place before the first step)
//  kInitSwapped: in place, before an odd step: the rest state as post-collision
//                values, f*_i at (x, opposite plane); also the rest slot
//  kInitStash:   in place, before an even step (> 0): the rest state at
//                (x, plane i), except links from a cell of a block that took
//                part in the last step, which take the value that cell
//                streamed towards x and kept at its own (x - e_i, opposite
//                plane); the rest state is left there in its place
enum InitMode : int { kInitNatural = 0, kInitSwapped = 1, kInitStash = 2 };

// Face kinds (same values as LBM_BC_*).
enum FaceKind : int { kPeriodic = 0, kWall = 1, kInletFace = 2, kOutletFace = 3 };

// Control words in device memory.
enum Ctrl : int {
  kNActive = 0,     // active blocks (== slots in use)
  kNewFirst = 1,    // first slot activated by the last activation pass
  kNewCount = 2,    // number of slots activated by the last activation pass
  kPoolFull = 3,    // set when a request did not fit the pool
  kNumeric = 4,     // set when a density was non-positive or non-finite
  kTraceLen = 5,    // activation trace entries written
  kCandCount = 6,   // proposal candidates listed by the last k_candidates
  kStepCount = 7,   // steps taken (maintained on the device by batched stepping)
  kPending = 8,     // requests or failing links recorded since the last activation pass
  kNumCtrl = 9
};

// Constants of one run, passed by value to every kernel.
struct Params {
  int nx, ny, nz;
  int nbx, nby, nbz, nb;
  int ncomp;
  int shell;
  int bc[6];
  int capacity;      // usable slots; slot index `capacity` is the rest slot
  uint32_t plane;    // cells per plane: (capacity + 1) * slot_cells
  uint32_t slot_cells;  // cells a slot spans in every plane: 4096, or 4160 (padded; see the kernels' header)
  int store;         // 0: FP32 populations, 1: FP16 deviations
  int trace_cap;
  int s_zero;        // criterion threshold is exactly zero
  float S;
  float omega[kMaxComp];   // 1/tau
  float RT, a_theta, b;    // Peng-Robinson constants
  float g_self[kMaxComp];
  float g_cross;
  float beta;
  float body[kMaxComp][3];
  float psi_in[kMaxComp];
  float psi_rest[kMaxComp];
  float rho_rest[kMaxComp];
  float rho_ref_rest[kMaxComp];        // reference density of the stored rest state (FP16 store)
  float f_in[kMaxComp][kQ];            // populations imposed by inlet nodes
  float f_rest[kMaxComp][kQ];          // rest populations, decoded (bitwise fixed point)
  uint32_t f_rest_bits[kMaxComp][kQ];  // rest populations in the stored format
};

// Device buffers of one handle.
// A "plane" holds one value per cell of every slot: index slot*slot_cells + cell.
struct Buffers {
  void* f[2];             // populations: [ncomp*19 planes] of float or __half (in place: f[1] == f[0],
                          // and the buffer index only selects the reference densities)
  float* psi;             // in place only: [ncomp planes] pseudo-potential of the step being taken
  float* rho[2];          // FP16 store only: [ncomp planes] reference densities, double-buffered
  uint32_t* mask;         // [1 plane]: bit i = link i bounces; kind in bits 24..25
  float* uprev;           // [ncomp*3 planes] velocity of the previous step (criterion; progressive only)
  int32_t* block_slot;    // [nb] slot of a block, -1 when inactive
  int32_t* slot_block;    // [capacity] block of a slot (the active list)
  int32_t* order;         // [capacity] the active slots in block order (scheduling order of the step)
  int32_t* frontier;      // [capacity] nonzero while the slot's block may have an inactive neighbour holding
                          // fluid (set when the slot is initialised, cleared by the criterion once it has none)
  uint8_t* bfluid;        // [nb] block holds a non-solid cell
  uint8_t* solid;         // [nx*ny*nz] solid flags of the whole lattice
  int32_t* request;       // [nb] activation requests
  int32_t* expose;        // [nb] links that showed a non-rest psi to the block this step
  int32_t* act_step;      // [nb] step at which the block was last activated, -1 never
  float* bfrac;           // [nb] fraction of the block's cells that are fluid
  int32_t* cand;          // [nb] proposal candidates (inactive, fluid, an active neighbour), block order
  int32_t* ctrl;          // [kNumCtrl]
  unsigned long long* counters;  // [0] leak, [1] clamps
  int32_t* trace;         // [trace_cap][2] (step, block)
  const float* init_rho;  // [ncomp][N] initial densities, or null (used before the first step)
  const float* init_u;    // [3][N] initial velocity, or null
};

// Batched stepping: several simulations advanced by the same launches.  P
// and D are device tables (one entry per simulation); off[nsims + 1] holds
// the prefix sums of their active block counts (the merged active list).
struct Batch {
  const Params* P;
  const Buffers* D;
  int32_t* off;
  int32_t nsims;
  int32_t total_capacity;
  int32_t* heads;  // [8] queue heads of the persistent step kernel (one queue per XCD), zero between steps
};

// Launchers (lbm_kernels.hip).  All enqueue on `stream` and return the
// launch status.
// Rest state: bg = device [2] background densities; out = device
// [2*19 stored bits][2*19 decoded populations][2 reference densities]
// [2 densities][2 potentials]; iters = device int.
hipError_t launch_rest_state(const Params& P, const float* bg, float* out, int* iters, hipStream_t stream);
// mode: InitMode; born: the step the slots join (blocks activated then are
// read as rest by kInitStash).
hipError_t launch_init_slots(const Params& P, const Buffers& D, int buf, int first_slot_host, int count_host,
                             bool from_device_counts, bool use_initial_fields, hipStream_t stream,
                             int mode = kInitNatural, int born = -1);
hipError_t launch_activate(const Params& P, const Buffers& D, int step, hipStream_t stream);
// Fused step kernel: moments, psi, forces, collision and streaming.  parts
// (1, 2 or 4) workgroups share each block, each taking 16 / parts planes.
hipError_t launch_fused(const Params& P, const Buffers& D, int rbuf, bool pull, int parts, hipStream_t stream);
// Criterion of Eq 13 and leak checks on the shell cells of frontier blocks.
enum : int {
  kCritRecord = 1,    // store this step's velocities for the next comparison
  kCritEval = 2,      // compare with the stored velocities, request blocks
  kCritExposure = 4,  // check the psi shown to inactive blocks
  kCritEmission = 8,  // check the populations the last step handed to inactive blocks
};
hipError_t launch_criterion(const Params& P, const Buffers& D, int rbuf, int rd, int flags,
                            hipStream_t stream);
// In-place step (one population buffer): psi of every cell of the active
// blocks into D.psi, then forces, collision and streaming in place.
// rd: kRdOwn for the first step, then kRdAAOdd / kRdAAEven by step parity;
// rbuf: the reference densities read (FP16 store; this step writes rbuf ^ 1).
hipError_t launch_inplace_psi(const Params& P, const Buffers& D, int rbuf, int rd, hipStream_t stream);
hipError_t launch_inplace_collide(const Params& P, const Buffers& D, int rbuf, int rd, hipStream_t stream);
// Learned activation proposal: list the candidate blocks, then per candidate
// gather its 12 features; with mlp != nullptr also run the network and request
// the block when its probability exceeds thr, else write feat[cap][12] and
// block[cap] for the first cap candidates.
hipError_t launch_candidates(const Params& P, const Buffers& D, hipStream_t stream);
hipError_t launch_propose(const Params& P, const Buffers& D, int rbuf, int rd, int step, const float* mlp,
                          float thr, float* feat, int32_t* block, int cap, hipStream_t stream);
// Batched step: criterion (progressive), activation, initialisation,
// merged list, fused step, step counters; `first` selects the first step
// of a run (populations read in place).  Every member must share store,
// component count, mode and step parity.
hipError_t launch_batch_offsets(const Batch& B, const Params& P0, hipStream_t stream);
// persistent: the step kernel as a resident grid taking work items (A-B
// pattern; the in-place kernels always use one workgroup per item).
hipError_t launch_batch_step(const Batch& B, const Params& P0, int rbuf, bool first, bool progressive,
                             bool in_place, int parts, bool persistent, hipStream_t stream);
hipError_t launch_export(const Params& P, const Buffers& D, int rbuf, int rd, float* rho, float* u,
                         float* umix, hipStream_t stream);
// Puts the slots in block order (slot j takes the block of D.order[j]) once
// every block holding fluid is active: every slot-indexed plane is permuted
// through the buffer the next step writes (two buffers) or the psi planes
// (in place); rbuf: the population buffer the next step reads.
hipError_t launch_repack(const Params& P, const Buffers& D, int rbuf, bool in_place, hipStream_t stream);
// out[n] = 1 for cells of active blocks (lattice-wide, N bytes).
hipError_t launch_active_cells(const Params& P, const Buffers& D, uint8_t* out, hipStream_t stream);
// Staging for lbm_moments_noalloc: a fixed device array of
// kStaticStagingFloats floats, one per GPU.  Returns its address on the
// current device (looked up once per device, thread-safe).
constexpr size_t kStaticStagingFloats = size_t(16) << 20;  // 64 MiB
hipError_t static_staging(float** out);
hipError_t launch_mass(const Params& P, const Buffers& D, int rbuf, int rd, double* out2,
                       hipStream_t stream);
// Test dump: psi_slots = device scratch of ncomp planes; psi (ncomp*N) and
// force (ncomp*3*N) lattice-wide device outputs.
hipError_t launch_debug_fields(const Params& P, const Buffers& D, int rbuf, int rd, float* psi_slots,
                               float* psi, float* force, hipStream_t stream);

}  // namespace lbm
