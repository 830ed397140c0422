// HIP kernels for gfx950 (CDNA4, wave64) of the progressive-mesh two-component
// pseudo-potential lattice Boltzmann update (Duchateau et al., arXiv
// 1510.03560, sections 2 and 4).
//
// Data layout: the lattice is cut into 16^3 blocks; an active block owns a
// slot of the pool.  Inside a slot everything is structure-of-arrays
// (section 3): f[slot][comp][dir][cell] with cell = x + 16*(y + 16*z), so the
// 64 lanes of a wave touch four consecutive x-rows, 256 contiguous bytes.
// The extra slot `capacity` holds the rest state everywhere and stands in for
// every inactive block and for the outside of the domain.
//
// One time step (section 4.3) runs
//   k_moments  : pull f(t) -> rho, u; psi (Eq 4-7); criterion of Eq 13 on the
//                boundary shell of frontier blocks -> activation requests
//   k_activate : compact requests into new slots (wave ballot + scan)
//   k_init     : new slots take the rest state
//   k_collide  : psi halo staged in LDS -> forces (Eq 8-9); BGK collision with
//                exact-difference forcing (Eq 10-12); pull streaming with
//                half-way bounce-back; aligned store of f*(t)
// The state between steps is the post-collision f*; the first step of a run
// reads the initial populations in place instead of pulling.
//
// Every floating-point expression is written out explicitly and the library
// is compiled without floating-point contraction, so the same inputs give the
// same bits in every kernel.  That makes the rest state computed by
// k_rest_state an exact fixed point of k_moments + k_collide, which is what
// lets a progressive run reproduce the static run bit for bit.

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

// ----------------------------------------------------------------- lattice
// D3Q19 (section 2.1, Fig 1b) with opposite directions adjacent: 2k-1 and 2k.
__host__ __device__ constexpr int dir_ex(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int dir_ey(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int dir_ez(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int dir_opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// weights: rest 1/3, axis 1/18, diagonal 1/36
__host__ __device__ constexpr float dir_w(int i) {
  return i == 0 ? (1.0f / 3.0f) : (i <= 6 ? (1.0f / 18.0f) : (1.0f / 36.0f));
}

constexpr float kThird = 1.0f / 3.0f;

template <int N, typename F>
__device__ __forceinline__ void unroll(F&& fn) {
  if constexpr (N > 0) {
    unroll<N - 1>(fn);
    fn(std::integral_constant<int, N - 1>{});
  }
}

// --------------------------------------------------------------- moments
// Eq 4-5.  Momentum is accumulated over opposite pairs so that a population
// set symmetric under reflection gives exactly zero.
struct Mom {
  float rho, jx, jy, jz;
};

__device__ __forceinline__ Mom moments(const float f[kQ]) {
  Mom m;
  float r = f[0];
  r = r + (f[1] + f[2]);
  r = r + (f[3] + f[4]);
  r = r + (f[5] + f[6]);
  r = r + (f[7] + f[8]);
  r = r + (f[9] + f[10]);
  r = r + (f[11] + f[12]);
  r = r + (f[13] + f[14]);
  r = r + (f[15] + f[16]);
  r = r + (f[17] + f[18]);
  const float d1 = f[1] - f[2], d3 = f[3] - f[4], d5 = f[5] - f[6];
  const float d7 = f[7] - f[8], d9 = f[9] - f[10], d11 = f[11] - f[12];
  const float d13 = f[13] - f[14], d15 = f[15] - f[16], d17 = f[17] - f[18];
  m.rho = r;
  m.jx = (((d1 + d7) + d9) + d11) + d13;
  m.jy = (((d3 + d7) - d9) + d15) + d17;
  m.jz = (((d5 + d11) - d13) + d15) - d17;
  return m;
}

// ------------------------------------------------------------------- EOS
// Eq 7 (Peng-Robinson, denominator 1 + 2 b rho - b^2 rho^2) and Eq 6.  A
// negative radicand gives psi = 0 and is reported through `clamped`.
__device__ __forceinline__ float pseudo_potential(const Params& P, int a, float rho, bool& clamped) {
  const float g = P.g_self[a];
  clamped = false;
  if (g == 0.0f) return 0.0f;
  const float brho = P.b * rho;
  const float p = (rho * P.RT) / (1.0f - brho) - (P.a_theta * rho * rho) / ((1.0f + 2.0f * brho) - brho * brho);
  const float rad = (2.0f * (p - kThird * rho)) / (kThird * g);
  if (!(rad >= 0.0f)) {
    clamped = true;
    return 0.0f;
  }
  return sqrtf(rad);
}

// -------------------------------------------------------------- forcing
// Stencil sum over opposite pairs: sum_i w_i v_i e_i with v_i the value at
// x + e_i.  Exactly zero when v is uniform.
struct Vec3 {
  float x, y, z;
};

__device__ __forceinline__ Vec3 pair_gradient(const float v[kQ]) {
  const float a = 1.0f / 18.0f, d = 1.0f / 36.0f;
  const float p1 = v[1] - v[2], p3 = v[3] - v[4], p5 = v[5] - v[6];
  const float p7 = v[7] - v[8], p9 = v[9] - v[10], p11 = v[11] - v[12];
  const float p13 = v[13] - v[14], p15 = v[15] - v[16], p17 = v[17] - v[18];
  Vec3 s;
  s.x = a * p1 + d * ((((p7 + p9) + p11) + p13));
  s.y = a * p3 + d * ((((p7 - p9) + p15) + p17));
  s.z = a * p5 + d * ((((p11 - p13) + p15) - p17));
  return s;
}

// Eq 8-9 read with lattice weights (the paper's weights being 6 w_i):
//   F_a = -beta g_aa psi_a(x) sum w_i psi_a(x+e_i) e_i
//         - (1-beta)/2 g_aa sum w_i psi_a(x+e_i)^2 e_i
//         - g_ab psi_a(x) sum w_i psi_b(x+e_i) e_i + rho_a body_a
// nb_self[i] / nb_other[i]: psi of this / the other component at x + e_i,
// already replaced by the centre value where x + e_i is solid or outside.
__device__ __forceinline__ Vec3 interaction_force(const Params& P, int a, float psi_c, const float nb_self[kQ],
                                                  const float nb_other[kQ], float rho) {
  float sq[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) sq[i] = nb_self[i] * nb_self[i];
  const Vec3 s1 = pair_gradient(nb_self);
  const Vec3 s2 = pair_gradient(sq);
  const float c1 = -P.beta * P.g_self[a] * psi_c;
  const float c2 = -0.5f * (1.0f - P.beta) * P.g_self[a];
  Vec3 F;
  F.x = c1 * s1.x + c2 * s2.x;
  F.y = c1 * s1.y + c2 * s2.y;
  F.z = c1 * s1.z + c2 * s2.z;
  if (P.ncomp == 2) {
    const Vec3 s3 = pair_gradient(nb_other);
    const float c3 = -P.g_cross * psi_c;
    F.x = F.x + c3 * s3.x;
    F.y = F.y + c3 * s3.y;
    F.z = F.z + c3 * s3.z;
  }
  F.x = F.x + rho * P.body[a][0];
  F.y = F.y + rho * P.body[a][1];
  F.z = F.z + rho * P.body[a][2];
  return F;
}

// ------------------------------------------------------------- collision
// Eq 10-12, relaxation toward equilibrium:
//   f* = f + omega (feq(rho,u) - f) + [feq(rho,u+du) - feq(rho,u)],  du = F/rho
// Eq 2 with c_s^2 = 1/3: feq_i = w_i rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u).
// The forcing bracket is evaluated in its factored form
//   w_i rho (3 e.du + 4.5 (e.du)(e.(u+v)) - 1.5 du.(u+v)),  v = u + du,
// which is the same quantity without the cancellation of two equilibria.
// The collision conserves the cell's mass exactly, so the rest population is
// taken as the remainder rho - sum_{i>0} f*_i: with FP32 weights (whose sum
// exceeds 1 by 1.5e-8) the direct formula would add that much mass per step.
__device__ __forceinline__ void collide(float omega, const float f[kQ], const Mom& m, const Vec3& F,
                                        float out[kQ]) {
  float inv = 0.0f;
  if (m.rho > 0.0f) inv = 1.0f / m.rho;
  const float ux = m.jx * inv, uy = m.jy * inv, uz = m.jz * inv;
  const float dx = F.x * inv, dy = F.y * inv, dz = F.z * inv;
  const float sx = (ux + ux) + dx, sy = (uy + uy) + dy, sz = (uz + uz) + dz;  // u + v
  const float usq = (ux * ux + uy * uy) + uz * uz;
  const float dus = (dx * sx + dy * sy) + dz * sz;
  unroll<kQ>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int ex = dir_ex(i), ey = dir_ey(i), ez = dir_ez(i);
    constexpr float w = dir_w(i);
    const float eu = float(ex) * ux + float(ey) * uy + float(ez) * uz;
    const float ed = float(ex) * dx + float(ey) * dy + float(ez) * dz;
    const float es = float(ex) * sx + float(ey) * sy + float(ez) * sz;
    const float wr = w * m.rho;
    const float feq = wr * (((1.0f + 3.0f * eu) + 4.5f * (eu * eu)) - 1.5f * usq);
    const float df = wr * ((3.0f * ed + 4.5f * (ed * es)) - 1.5f * dus);
    out[i] = (f[i] + omega * (feq - f[i])) + df;
  });
  float rest = (out[1] + out[2]) + (out[3] + out[4]);
  rest = rest + (out[5] + out[6]);
  rest = rest + (out[7] + out[8]);
  rest = rest + (out[9] + out[10]);
  rest = rest + (out[11] + out[12]);
  rest = rest + (out[13] + out[14]);
  rest = rest + (out[15] + out[16]);
  rest = rest + (out[17] + out[18]);
  out[0] = m.rho - rest;
}

__device__ __forceinline__ float feq_dir(int i, float rho, float ux, float uy, float uz) {
  const float eu = float(dir_ex(i)) * ux + float(dir_ey(i)) * uy + float(dir_ez(i)) * uz;
  const float usq = (ux * ux + uy * uy) + uz * uz;
  return (dir_w(i) * rho) * (((1.0f + 3.0f * eu) + 4.5f * (eu * eu)) - 1.5f * usq);
}

// ------------------------------------------------------------ addressing
__device__ __forceinline__ int neighbour_block(const Params& P, int bx, int by, int bz, int dx, int dy, int dz) {
  int c[3] = {bx + dx, by + dy, bz + dz};
  const int n[3] = {P.nbx, P.nby, P.nbz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (c[d] < 0 || c[d] >= n[d]) {
      if (P.bc[2 * d] != kPeriodic) return -1;
      c[d] = (c[d] + n[d]) % n[d];
    }
  }
  return c[0] + P.nbx * (c[1] + P.nby * c[2]);
}

__device__ __forceinline__ int sgn_out(int s) { return s < 0 ? -1 : (s > 15 ? 1 : 0); }

// Element index (within a population buffer, component 0) of the value that
// streams into direction I of cell (x,y,z): f*_I(x - e_I), or f*_opp(I)(x)
// when the link bounces (mask bit I).  nb[d] is the first element of the
// slot of neighbour block d = 13 + ox + 3 oy + 9 oz.
template <int I>
__device__ __forceinline__ long long pull_index(int x, int y, int z, uint32_t m, const long long* nb) {
  constexpr int ex = dir_ex(I), ey = dir_ey(I), ez = dir_ez(I);
  if constexpr (I == 0) {
    return nb[13] + (x + 16 * y + 256 * z);
  } else {
    const int sx = x - ex, sy = y - ey, sz = z - ez;
    const int ox = ex ? sgn_out(sx) : 0, oy = ey ? sgn_out(sy) : 0, oz = ez ? sgn_out(sz) : 0;
    const int c = (sx & 15) + 16 * (sy & 15) + 256 * (sz & 15);
    const long long pulled = nb[13 + ox + 3 * oy + 9 * oz] + (long long)I * kCells + c;
    const long long bounced = nb[13] + (long long)dir_opp(I) * kCells + (x + 16 * y + 256 * z);
    return (m >> I) & 1u ? bounced : pulled;
  }
}

// Loads the 19 populations of component a arriving at (x,y,z).
template <bool PULL>
__device__ __forceinline__ void load_cell(const float* __restrict__ fb, long long comp_off, int x, int y, int z,
                                          uint32_t m, const long long* nb, float f[kQ]) {
  if constexpr (PULL) {
    unroll<kQ>([&](auto I) {
      constexpr int i = decltype(I)::value;
      f[i] = fb[pull_index<i>(x, y, z, m, nb) + comp_off];
    });
  } else {
    const long long base = nb[13] + comp_off + (x + 16 * y + 256 * z);
#pragma unroll
    for (int i = 0; i < kQ; ++i) f[i] = fb[base + (long long)i * kCells];
  }
}

// The 27 neighbour slots of a block (inactive and outside -> rest slot),
// their block ids (-1 outside) and the candidate mask: neighbours that are
// inside the domain, inactive and hold fluid.
struct BlockCtx {
  long long nb[27];
  int nslot[27];
  int nbk[27];
  unsigned cand;
  unsigned fired;
};

__device__ __forceinline__ void setup_block(const Params& P, const Buffers& D, int blk, long long slot_elems,
                                            BlockCtx& ctx) {
  const int t = threadIdx.x;
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  bool cand = false;
  if (t < 27) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int nbid = neighbour_block(P, bx, by, bz, dx, dy, dz);
    int sl = nbid < 0 ? -1 : D.block_slot[nbid];
    if (t != 13 && nbid >= 0 && sl < 0 && D.bfluid[nbid]) cand = true;
    if (sl < 0) sl = P.capacity;
    ctx.nb[t] = (long long)sl * slot_elems;
    ctx.nslot[t] = sl;
    ctx.nbk[t] = nbid;
  }
  // threads 0..26 are all in the first wave
  const unsigned long long bal = __ballot(cand);
  if (t == 0) {
    ctx.cand = (unsigned)bal;
    ctx.fired = 0u;
  }
}

// Directions d (bit d, d = 13 + dx + 3 dy + 9 dz) of the neighbour blocks
// whose distance from cell (x,y,z) is at most w cells.
__device__ __forceinline__ unsigned shell_dirs(int x, int y, int z, int w) {
  auto axis = [&](int v) -> unsigned {
    unsigned s = 2u;  // offset 0
    if (v <= w - 1) s |= 1u;
    if (v >= kB - w) s |= 4u;
    return s;
  };
  const unsigned ax = axis(x), ay = axis(y), az = axis(z);
  unsigned out = 0u;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
      if (((ay >> dy) & 1u) && ((az >> dz) & 1u)) out |= ax << (3 * dy + 9 * dz);
  return out & ~(1u << 13);
}

// ----------------------------------------------------------- rest state
// Iterates the update of a cell whose every neighbour is itself (uniform
// lattice at rest, density bg) until the populations stop changing; the same
// device functions as k_moments/k_collide, so the result is a fixed point of
// the real update.  Single thread; tiny.
__global__ void k_rest_state(Params P, const float* bg, float* out, int* iters) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // the rest state is defined without body force
  for (int a = 0; a < kMaxComp; ++a) P.body[a][0] = P.body[a][1] = P.body[a][2] = 0.0f;
  float f[kMaxComp][kQ];
  for (int a = 0; a < P.ncomp; ++a)
    for (int i = 0; i < kQ; ++i) f[a][i] = dir_w(i) * bg[a];
  int it = 0;
  for (; it < 100000; ++it) {
    float psi[kMaxComp] = {0.0f, 0.0f};
    Mom m[kMaxComp];
    for (int a = 0; a < P.ncomp; ++a) {
      m[a] = moments(f[a]);
      bool cl;
      psi[a] = pseudo_potential(P, a, m[a].rho, cl);
    }
    bool same = true;
    float nf[kMaxComp][kQ];
    for (int a = 0; a < P.ncomp; ++a) {
      float ns[kQ], no[kQ];
      for (int i = 0; i < kQ; ++i) {
        ns[i] = psi[a];
        no[i] = psi[P.ncomp == 2 ? 1 - a : a];
      }
      const Vec3 F = interaction_force(P, a, psi[a], ns, no, m[a].rho);
      collide(P.omega[a], f[a], m[a], F, nf[a]);
      for (int i = 0; i < kQ; ++i) same = same && (__float_as_uint(nf[a][i]) == __float_as_uint(f[a][i]));
    }
    for (int a = 0; a < P.ncomp; ++a)
      for (int i = 0; i < kQ; ++i) f[a][i] = nf[a][i];
    if (same) break;
  }
  for (int a = 0; a < P.ncomp; ++a) {
    const Mom m = moments(f[a]);
    bool cl;
    for (int i = 0; i < kQ; ++i) out[a * kQ + i] = f[a][i];
    out[kMaxComp * kQ + a] = m.rho;
    out[kMaxComp * kQ + kMaxComp + a] = pseudo_potential(P, a, m.rho, cl);
  }
  *iters = it;
}

// ----------------------------------------------------------- slot init
// Initialises slots [first, first+count): per-cell mask (links that bounce,
// cell kind), populations of buffer `buf`, psi and the criterion history.
// Slot `capacity` (the rest slot) is initialised the same way with the rest
// state everywhere and an all-fluid mask.
__global__ void __launch_bounds__(256) k_init(Params P, Buffers D, int buf, int first_h, int count_h, int from_dev,
                                              int use_init) {
  const int first = from_dev ? D.ctrl[kNewFirst] : first_h;
  const int count = from_dev ? D.ctrl[kNewCount] : count_h;
  const long long slot_elems = (long long)P.ncomp * kQ * kCells;
  float* fb = D.f[buf];
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const int slot = first + k;
    const bool rest_slot = slot == P.capacity;
    const int blk = rest_slot ? -1 : D.slot_block[slot];
    const int bx = rest_slot ? 0 : blk % P.nbx, by = rest_slot ? 0 : (blk / P.nbx) % P.nby,
              bz = rest_slot ? 0 : blk / (P.nbx * P.nby);
    for (int c = threadIdx.x; c < kCells; c += blockDim.x) {
      const int x = c & 15, y = (c >> 4) & 15, z = c >> 8;
      uint32_t m = 0u;
      long long n = -1;
      if (!rest_slot) {
        const int X = bx * kB + x, Y = by * kB + y, Z = bz * kB + z;
        n = X + (long long)P.nx * (Y + (long long)P.ny * Z);
        uint32_t kind = D.solid[n] ? kSolid : kFluid;
        if (kind == kFluid) {
          const bool on[6] = {X == 0, X == P.nx - 1, Y == 0, Y == P.ny - 1, Z == 0, Z == P.nz - 1};
          for (int fc = 0; fc < 6; ++fc)
            if (on[fc] && P.bc[fc] == kOutletFace) kind = kOutlet;
          for (int fc = 0; fc < 6; ++fc)
            if (on[fc] && P.bc[fc] == kInletFace) kind = kInlet;
        }
        m = kind << kKindShift;
        unroll<kQ>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (i > 0) {
            int s[3] = {X - dir_ex(i), Y - dir_ey(i), Z - dir_ez(i)};
            const int L[3] = {P.nx, P.ny, P.nz};
            bool bounce = false;
            for (int d = 0; d < 3; ++d) {
              if (s[d] < 0 || s[d] >= L[d]) {
                if (P.bc[2 * d] != kPeriodic) bounce = true;
                s[d] = (s[d] + L[d]) % L[d];
              }
            }
            if (!bounce) bounce = D.solid[s[0] + (long long)P.nx * (s[1] + (long long)P.ny * s[2])] != 0;
            if (bounce) m |= 1u << i;
          }
        });
      }
      D.mask[(long long)slot * kCells + c] = m;
      for (int a = 0; a < P.ncomp; ++a) {
        float r0 = __int_as_float(0x7fc00000);  // NaN: rest state
        float ux = 0.0f, uy = 0.0f, uz = 0.0f;
        if (use_init && n >= 0 && D.init_rho) {
          r0 = D.init_rho[(long long)a * P.nx * P.ny * P.nz + n];
          if (D.init_u) {
            const long long N = (long long)P.nx * P.ny * P.nz;
            ux = D.init_u[n];
            uy = D.init_u[N + n];
            uz = D.init_u[2 * N + n];
          }
        }
        const bool at_rest = !(r0 == r0);
        const long long base = (long long)slot * slot_elems + (long long)a * kQ * kCells + c;
        for (int i = 0; i < kQ; ++i) fb[base + (long long)i * kCells] = at_rest ? P.f_rest[a][i] : feq_dir(i, r0, ux, uy, uz);
        D.psi[((long long)slot * P.ncomp + a) * kCells + c] = P.psi_rest[a];
        if (!rest_slot && D.uprev)
          for (int d = 0; d < 3; ++d) D.uprev[(((long long)slot * P.ncomp + a) * 3 + d) * kCells + c] = 0.0f;
      }
    }
  }
}

// --------------------------------------------------------------- moments
// K1: per active block, pull f(t), compute rho_a, u_a (Eq 4-5) and psi_a
// (Eq 6-7) for every cell; store psi.  On frontier blocks (an inactive
// neighbour holding fluid), evaluate Eq 13: a fluid cell within `shell` cells
// of such a neighbour whose velocity differs from the previous step's, for
// any component, requests that neighbour (section 4.2).  crit_mode: 0 = no
// criterion, 1 = only record velocities (first step), 2 = evaluate and record.
template <bool PULL>
__global__ void __launch_bounds__(256) k_moments(Params P, Buffers D, int rbuf, int crit_mode) {
  const int s = blockIdx.x;
  if (s >= D.ctrl[kNActive]) return;
  __shared__ BlockCtx ctx;
  const long long slot_elems = (long long)P.ncomp * kQ * kCells;
  setup_block(P, D, D.slot_block[s], slot_elems, ctx);
  __syncthreads();
  const unsigned cand = crit_mode ? ctx.cand : 0u;
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  const float* __restrict__ fb = D.f[rbuf];
  unsigned fired = 0u;
  unsigned numeric = 0u, clamps = 0u;
  for (int z = 0; z < kB; ++z) {
    const int c = x + 16 * y + 256 * z;
    const uint32_t m = D.mask[(long long)s * kCells + c];
    const uint32_t kind = (m >> kKindShift) & 3u;
    const unsigned dirs = cand ? (shell_dirs(x, y, z, P.shell) & cand) : 0u;
    bool changed = false;
    for (int a = 0; a < P.ncomp; ++a) {
      float f[kQ];
      load_cell<PULL>(fb, (long long)a * kQ * kCells, x, y, z, m, ctx.nb, f);
      const Mom mo = moments(f);
      float psi = 0.0f;
      if (kind == kFluid) {
        bool cl;
        psi = pseudo_potential(P, a, mo.rho, cl);
        clamps += cl ? 1u : 0u;
        if (!(mo.rho > 0.0f && mo.rho < 3.0e38f)) numeric = 1u;
      } else if (kind == kInlet) {
        psi = P.psi_in[a];
      } else if (kind == kOutlet) {
        psi = P.psi_rest[a];
      }
      D.psi[((long long)s * P.ncomp + a) * kCells + c] = psi;
      if (dirs && kind != kSolid) {
        float inv = 0.0f;
        if (mo.rho > 0.0f) inv = 1.0f / mo.rho;
        const float u[3] = {mo.jx * inv, mo.jy * inv, mo.jz * inv};
        float* up = D.uprev + (((long long)s * P.ncomp + a) * 3) * kCells + c;
        if (crit_mode == 2) {
          float d2 = 0.0f;
          bool diff = false;
          for (int d = 0; d < 3; ++d) {
            const float dd = u[d] - up[(long long)d * kCells];
            diff = diff || (dd != 0.0f);
            d2 = d2 + dd * dd;
          }
          changed = changed || (P.s_zero ? diff : (sqrtf(d2) > P.S));
        }
        for (int d = 0; d < 3; ++d) up[(long long)d * kCells] = u[d];
      }
    }
    if (changed) fired |= dirs;
  }
  if (numeric) atomicOr(&D.ctrl[kNumeric], 1);
  if (clamps) atomicAdd(&D.counters[1], (unsigned long long)clamps);
  if (cand) {
    if (fired) atomicOr(&ctx.fired, fired);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 27 && ((ctx.fired >> t) & 1u)) D.request[ctx.nbk[t]] = 1;
  }
}

// -------------------------------------------------------------- activate
// K3: one workgroup of 1024 threads compacts the requested blocks (inactive,
// holding fluid) into new slots, in block order: slot = n_active + rank, with
// the rank from a wave ballot and a workgroup prefix sum.  Clears requests.
__global__ void __launch_bounds__(1024) k_activate(Params P, Buffers D, int step) {
  __shared__ int wave_count[16];
  __shared__ int wave_base[16];
  __shared__ int chunk_total;
  __shared__ int stop;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int n0 = D.ctrl[kNActive];
  const int tr0 = D.ctrl[kTraceLen];
  int base = n0;
  if (t == 0) stop = 0;
  __syncthreads();
  for (int b0 = 0; b0 < P.nb; b0 += 1024) {
    const int b = b0 + t;
    int flag = 0;
    if (b < P.nb && D.request[b]) flag = (D.block_slot[b] < 0 && D.bfluid[b]) ? 1 : 0;
    const unsigned long long bal = __ballot(flag);
    const int lane_rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_count[wave] = __popcll(bal);
    __syncthreads();
    if (t == 0) {
      int acc = 0;
      for (int w = 0; w < 16; ++w) {
        wave_base[w] = acc;
        acc += wave_count[w];
      }
      chunk_total = acc;
      if (base + acc > P.capacity) stop = 1;
    }
    __syncthreads();
    if (stop) break;  // pool full: keep the remaining requests, report
    if (flag) {
      const int rank = base - n0 + wave_base[wave] + lane_rank;
      const int slot = base + wave_base[wave] + lane_rank;
      D.block_slot[b] = slot;
      D.slot_block[slot] = b;
      if (tr0 + rank < P.trace_cap) {
        D.trace[2 * (tr0 + rank)] = step;
        D.trace[2 * (tr0 + rank) + 1] = b;
      }
    }
    if (b < P.nb) D.request[b] = 0;
    base += chunk_total;
    __syncthreads();
  }
  if (t == 0) {
    D.ctrl[kNewFirst] = n0;
    D.ctrl[kNewCount] = base - n0;
    D.ctrl[kNActive] = base;
    D.ctrl[kTraceLen] = tr0 + (base - n0);
    if (stop) D.ctrl[kPoolFull] = 1;
  }
}

// --------------------------------------------------------------- collide
// K2: per active block, stage psi of the 18^3 halo (block plus one cell) for
// every component in LDS, then per cell: pull f(t), moments, forces from the
// LDS psi stencil (Eq 8-9), collision with exact-difference forcing
// (Eq 10-12), boundary nodes impose their state, aligned store of f*(t) to
// the other buffer.  MODE 1 instead writes psi and the force to lattice-wide
// debug arrays.  Frontier blocks also count leaks: a non-rest population or
// potential handed to a cell of an inactive block.
constexpr int kH = kB + 2;            // halo edge
constexpr int kHalo = kH * kH * kH;   // 5832 cells

__device__ __forceinline__ int hidx(int x, int y, int z) { return (x + 1) + kH * ((y + 1) + kH * (z + 1)); }

template <bool PULL, int MODE>
__global__ void __launch_bounds__(256) k_collide(Params P, Buffers D, int rbuf, float* dbg_psi, float* dbg_force) {
  const int s = blockIdx.x;
  if (s >= D.ctrl[kNActive]) return;
  __shared__ BlockCtx ctx;
  __shared__ float psi_s[kMaxComp * kHalo];
  const long long slot_elems = (long long)P.ncomp * kQ * kCells;
  const int blk = D.slot_block[s];
  setup_block(P, D, blk, slot_elems, ctx);
  __syncthreads();
  // psi halo
  for (int h = threadIdx.x; h < kHalo; h += blockDim.x) {
    const int hx = h % kH - 1, hy = (h / kH) % kH - 1, hz = h / (kH * kH) - 1;
    const int d = 13 + sgn_out(hx) + 3 * sgn_out(hy) + 9 * sgn_out(hz);
    const long long slot = ctx.nslot[d];
    const int c = (hx & 15) + 16 * (hy & 15) + 256 * (hz & 15);
    for (int a = 0; a < P.ncomp; ++a) psi_s[a * kHalo + h] = D.psi[(slot * P.ncomp + a) * kCells + c];
  }
  __syncthreads();
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  const float* __restrict__ fb = D.f[rbuf];
  float* __restrict__ fw = D.f[rbuf ^ 1];
  const bool frontier = ctx.cand != 0u;
  unsigned long long leak = 0ull;
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  for (int z = 0; z < kB; ++z) {
    const int c = x + 16 * y + 256 * z;
    const uint32_t m = D.mask[(long long)s * kCells + c];
    const uint32_t kind = (m >> kKindShift) & 3u;
    if (kind == kSolid) continue;
    const int h0 = hidx(x, y, z);
    bool bad_psi = false;
    for (int a = 0; a < P.ncomp; ++a) bad_psi = bad_psi || (psi_s[a * kHalo + h0] != P.psi_rest[a]);
    uint32_t bad_dirs = 0u;
    for (int a = 0; a < P.ncomp; ++a) {
      const int o = P.ncomp == 2 ? 1 - a : a;
      const float pc = psi_s[a * kHalo + h0], po = psi_s[o * kHalo + h0];
      float f[kQ];
      load_cell<PULL>(fb, (long long)a * kQ * kCells, x, y, z, m, ctx.nb, f);
      const Mom mo = moments(f);
      float out[kQ];
      Vec3 F = {0.0f, 0.0f, 0.0f};
      if (kind == kFluid) {
        float ns[kQ], no[kQ];
        ns[0] = pc;
        no[0] = po;
        unroll<kQ>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (i > 0) {
            const int hn = hidx(x + dir_ex(i), y + dir_ey(i), z + dir_ez(i));
            const bool solid_nb = (m >> dir_opp(i)) & 1u;  // x + e_i is solid or outside
            ns[i] = solid_nb ? pc : psi_s[a * kHalo + hn];
            no[i] = solid_nb ? po : psi_s[o * kHalo + hn];
          }
        });
        F = interaction_force(P, a, pc, ns, no, mo.rho);
        if constexpr (MODE == 0) collide(P.omega[a], f, mo, F, out);
      } else {
        const float* src = kind == kInlet ? P.f_in[a] : P.f_rest[a];
#pragma unroll
        for (int i = 0; i < kQ; ++i) out[i] = src[i];
      }
      if constexpr (MODE == 0) {
        const long long wb = (long long)s * slot_elems + (long long)a * kQ * kCells + c;
#pragma unroll
        for (int i = 0; i < kQ; ++i) fw[wb + (long long)i * kCells] = out[i];
        if (frontier) {
          // leak check toward cells of inactive blocks
          unroll<kQ>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
              const int tx = x + dir_ex(i), ty = y + dir_ey(i), tz = z + dir_ez(i);
              const int d = 13 + sgn_out(tx) + 3 * sgn_out(ty) + 9 * sgn_out(tz);
              const bool outside_or_solid = (m >> dir_opp(i)) & 1u;
              const bool inactive = ctx.nslot[d] == P.capacity && d != 13;
              if (!outside_or_solid && inactive && (out[i] != P.f_rest[a][i] || bad_psi)) bad_dirs |= 1u << i;
            }
          });
        }
      } else {
        const int X = bx * kB + x, Y = by * kB + y, Z = bz * kB + z;
        const long long N = (long long)P.nx * P.ny * P.nz;
        const long long n = X + (long long)P.nx * (Y + (long long)P.ny * Z);
        dbg_psi[a * N + n] = pc;
        dbg_force[(a * 3 + 0) * N + n] = F.x;
        dbg_force[(a * 3 + 1) * N + n] = F.y;
        dbg_force[(a * 3 + 2) * N + n] = F.z;
      }
    }
    leak += (unsigned long long)__popc(bad_dirs);
  }
  if constexpr (MODE == 0) {
    if (frontier && leak) atomicAdd(&D.counters[0], leak);
  }
}

// ---------------------------------------------------------------- export
// Lattice-wide default: rest state for fluid cells, zeros for solid cells.
__global__ void k_fill_default(Params P, Buffers D, float* rho, float* u, float* umix) {
  const long long N = (long long)P.nx * P.ny * P.nz;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const bool sol = D.solid[n] != 0;
    for (int a = 0; a < P.ncomp; ++a) {
      if (rho) rho[a * N + n] = sol ? 0.0f : P.rho_rest[a];
      if (u)
        for (int d = 0; d < 3; ++d) u[(a * 3 + d) * N + n] = 0.0f;
    }
    if (umix)
      for (int d = 0; d < 3; ++d) umix[d * N + n] = 0.0f;
  }
}

// Moments (Eq 4-5) of the active blocks into lattice-wide arrays.
template <bool PULL>
__global__ void __launch_bounds__(256) k_export(Params P, Buffers D, int rbuf, float* rho, float* u, float* umix) {
  const int s = blockIdx.x;
  if (s >= D.ctrl[kNActive]) return;
  __shared__ BlockCtx ctx;
  const long long slot_elems = (long long)P.ncomp * kQ * kCells;
  const int blk = D.slot_block[s];
  setup_block(P, D, blk, slot_elems, ctx);
  __syncthreads();
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  const long long N = (long long)P.nx * P.ny * P.nz;
  for (int z = 0; z < kB; ++z) {
    const int c = x + 16 * y + 256 * z;
    const uint32_t m = D.mask[(long long)s * kCells + c];
    const bool sol = ((m >> kKindShift) & 3u) == kSolid;
    const long long n = (bx * kB + x) + (long long)P.nx * ((by * kB + y) + (long long)P.ny * (bz * kB + z));
    float mr = 0.0f, mx = 0.0f, my = 0.0f, mz = 0.0f;
    for (int a = 0; a < P.ncomp; ++a) {
      Mom mo = {0.0f, 0.0f, 0.0f, 0.0f};
      if (!sol) {
        float f[kQ];
        load_cell<PULL>(D.f[rbuf], (long long)a * kQ * kCells, x, y, z, m, ctx.nb, f);
        mo = moments(f);
      }
      float inv = 0.0f;
      if (mo.rho > 0.0f) inv = 1.0f / mo.rho;
      if (rho) rho[a * N + n] = mo.rho;
      if (u) {
        u[(a * 3 + 0) * N + n] = mo.jx * inv;
        u[(a * 3 + 1) * N + n] = mo.jy * inv;
        u[(a * 3 + 2) * N + n] = mo.jz * inv;
      }
      mr = mr + mo.rho;
      mx = mx + mo.jx;
      my = my + mo.jy;
      mz = mz + mo.jz;
    }
    if (umix) {
      float inv = 0.0f;
      if (mr > 0.0f) inv = 1.0f / mr;
      umix[n] = mx * inv;
      umix[N + n] = my * inv;
      umix[2 * N + n] = mz * inv;
    }
  }
}

// Sum of rho_a over the fluid cells of the active blocks, FP64; out[2 + a]
// counts those cells.
template <bool PULL>
__global__ void __launch_bounds__(256) k_mass(Params P, Buffers D, int rbuf, double* out) {
  const int s = blockIdx.x;
  if (s >= D.ctrl[kNActive]) return;
  __shared__ BlockCtx ctx;
  __shared__ double red[kMaxComp][256];
  __shared__ int cnt[256];
  const long long slot_elems = (long long)P.ncomp * kQ * kCells;
  setup_block(P, D, D.slot_block[s], slot_elems, ctx);
  __syncthreads();
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  double acc[kMaxComp] = {0.0, 0.0};
  int nf = 0;
  for (int z = 0; z < kB; ++z) {
    const int c = x + 16 * y + 256 * z;
    const uint32_t m = D.mask[(long long)s * kCells + c];
    if (((m >> kKindShift) & 3u) == kSolid) continue;
    ++nf;
    for (int a = 0; a < P.ncomp; ++a) {
      float f[kQ];
      load_cell<PULL>(D.f[rbuf], (long long)a * kQ * kCells, x, y, z, m, ctx.nb, f);
      acc[a] += (double)moments(f).rho;
    }
  }
  for (int a = 0; a < kMaxComp; ++a) red[a][threadIdx.x] = acc[a];
  cnt[threadIdx.x] = nf;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int a = 0; a < kMaxComp; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
      cnt[threadIdx.x] += cnt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int a = 0; a < P.ncomp; ++a) atomicAdd(&out[a], red[a][0]);
    atomicAdd(&out[2], (double)cnt[0]);
  }
}

}  // namespace

// --------------------------------------------------------------- launchers
hipError_t launch_rest_state(const Params& P, const float* bg, float* out, int* iters, hipStream_t stream) {
  hipLaunchKernelGGL(k_rest_state, dim3(1), dim3(64), 0, stream, P, bg, out, iters);
  return hipGetLastError();
}

hipError_t launch_init_slots(const Params& P, const Buffers& D, int buf, int first, int count, bool from_dev,
                             bool use_init, hipStream_t stream) {
  const int grid = from_dev ? 512 : (count > 0 ? (count < 4096 ? count : 4096) : 1);
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, stream, P, D, buf, first, count, from_dev ? 1 : 0,
                     use_init ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_moments(const Params& P, const Buffers& D, int rbuf, bool pull, int crit_mode, hipStream_t stream) {
  if (pull)
    hipLaunchKernelGGL(k_moments<true>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, crit_mode);
  else
    hipLaunchKernelGGL(k_moments<false>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, crit_mode);
  return hipGetLastError();
}

hipError_t launch_activate(const Params& P, const Buffers& D, int step, hipStream_t stream) {
  hipLaunchKernelGGL(k_activate, dim3(1), dim3(1024), 0, stream, P, D, step);
  return hipGetLastError();
}

hipError_t launch_collide(const Params& P, const Buffers& D, int rbuf, bool pull, hipStream_t stream) {
  if (pull)
    hipLaunchKernelGGL((k_collide<true, 0>), dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_collide<false, 0>), dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_export(const Params& P, const Buffers& D, int rbuf, bool pull, float* rho, float* u, float* umix,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_fill_default, dim3(2048), dim3(256), 0, stream, P, D, rho, u, umix);
  if (pull)
    hipLaunchKernelGGL(k_export<true>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, rho, u, umix);
  else
    hipLaunchKernelGGL(k_export<false>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, rho, u, umix);
  return hipGetLastError();
}

hipError_t launch_mass(const Params& P, const Buffers& D, int rbuf, bool pull, double* out, hipStream_t stream) {
  if (pull)
    hipLaunchKernelGGL(k_mass<true>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, out);
  else
    hipLaunchKernelGGL(k_mass<false>, dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, out);
  return hipGetLastError();
}

hipError_t launch_debug_fields(const Params& P, const Buffers& D, int rbuf, bool pull, float* psi, float* force,
                               hipStream_t stream) {
  if (pull)
    hipLaunchKernelGGL((k_collide<true, 1>), dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, psi, force);
  else
    hipLaunchKernelGGL((k_collide<false, 1>), dim3(P.capacity), dim3(256), 0, stream, P, D, rbuf, psi, force);
  return hipGetLastError();
}

}  // namespace lbm
