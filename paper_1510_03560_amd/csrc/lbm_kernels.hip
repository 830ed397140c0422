// HIP kernels for gfx950 (CDNA4, wave64) of the progressive-mesh two-component
// pseudo-potential lattice Boltzmann update (Duchateau et al., arXiv
// 1510.03560, sections 2 and 4).
//
// Data layout.  The lattice is cut into 16^3 blocks; an active block owns a
// slot of the pool.  Populations are structure-of-arrays (section 3) by
// direction plane over the whole pool, the components of a cell side by side:
//     f[buf][dir][slot * slot_cells + cell][comp],
//     cell = (x mod 8) + 8 (y mod 4) + 32 (x div 8) + 64 (y div 4) + 256 z
// (8 x 4 tiles of x and y, see cell_of), so the 64 lanes of a wave read or
// write two whole tiles of one plane.  slot_cells is 4096, or 4160 when the
// block grid has a multiple of 16 blocks along x (the host's choice: the
// padding keeps y and z neighbours from sitting a power-of-two number of
// bytes apart, which made such meshes 7 % slower).  Every pull is a 32-bit
// byte offset from a wave-uniform base (the first plane of the
// opposite-direction pair), which keeps address arithmetic in single VGPRs.
// The extra slot `capacity` holds the rest state and stands in for every
// inactive block and for the outside of the domain.
//
// One time step (section 4.3) runs
//   k_criterion : frontier blocks only: pull the shell cells, Eq 13 ->
//                 activation requests; leak checks
//   k_activate  : compact requests into new slots (wave ballot + scan)
//   k_init      : new slots take the rest state
//   k_fused     : per active block, a z-sweep that pulls f(t) with half-way
//                 bounce-back, takes rho, psi (Eq 4-7) into LDS, the forces
//                 (Eq 8-9) from the LDS psi stencil, BGK collision with
//                 exact-difference forcing (Eq 10-12), and stores f*(t)
// (a static mesh runs k_fused only).  The state between steps is the
// post-collision f*; the first step of a run reads the initial populations
// in place instead of pulling.

// Storage formats: FP32, or FP16 deviations h = s (f - w_i rho_ref) with
// rho_ref the writing cell's own density of that step (kept, double-buffered,
// in `rho`), s = 2^12; arithmetic is FP32 in both.
//
// Every floating-point expression is written out explicitly and the library
// is compiled without floating-point contraction, so the same inputs give the
// same bits in every kernel.  That makes the rest state computed by
// k_rest_state an exact fixed point of k_fused, which is what
// lets a progressive run reproduce the static run bit for bit.

#include <hip/hip_fp16.h>

#include <mutex>
#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kThreads = 512;            // workgroup of the per-block kernels
constexpr int kZStep = kThreads / 256;   // z-planes handled together

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

// e_i . (x, y, z) for a constant direction: the sum of the nonzero terms in
// x, y, z order (the terms with a zero component are exactly zero, so this is
// the full dot product without its multiplications by 0 and 1).
template <int ex, int ey, int ez>
__device__ __forceinline__ float edot(float x, float y, float z) {
  static_assert(ex != 0 || ey != 0 || ez != 0, "rest direction");
  const float tx = ex > 0 ? x : -x, ty = ey > 0 ? y : -y, tz = ez > 0 ? z : -z;
  if constexpr (ex != 0 && ey != 0 && ez != 0) return (tx + ty) + tz;
  if constexpr (ex != 0 && ey != 0) return tx + ty;
  if constexpr (ex != 0 && ez != 0) return tx + tz;
  if constexpr (ey != 0 && ez != 0) return ty + tz;
  if constexpr (ex != 0) return tx;
  if constexpr (ey != 0) return ty;
  return tz;
}

template <int N, typename F>
__host__ __device__ __forceinline__ void unroll(F&& fn) {
  if constexpr (N > 0) {
    unroll<N - 1>(fn);
    fn(std::integral_constant<int, N - 1>{});
  }
}

// Loads and stores at a 32-bit byte offset from a wave-uniform base: the
// form that keeps the base in SGPRs and the offset in one VGPR.  Offsets are
// computed in 32-bit arithmetic by the callers (every population pair spans
// less than 4 GiB).
template <typename T>
__device__ __forceinline__ T ld(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Streaming store: the populations written by a step are read back only in
// the next step, so they should not displace the lines the current step
// still reads from the L2 (the non-temporal hint).
__device__ __forceinline__ void st_stream(float* base, uint32_t off, float v) {
  __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off));
}
__device__ __forceinline__ void st_stream(__half* base, uint32_t off, __half v) {
  __builtin_nontemporal_store(__half_as_ushort(v),
                              reinterpret_cast<unsigned short*>(reinterpret_cast<char*>(base) + off));
}

// ------------------------------------------------- reference densities
// FP16 store: the reference densities of a cell (its density of the step
// that wrote its populations), the components side by side: element
// cell * ncomp + a of D.rho[b]; one load or store per cell.
template <int NC>
__device__ __forceinline__ void ld_refs(const float* base, uint32_t cell, float (&r)[NC]) {
  if constexpr (NC == 1) {
    r[0] = ld(base, cell * 4u);
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 w = ld(reinterpret_cast<const f2*>(base), cell * 8u);
    r[0] = w.x;
    r[1] = w.y;
  }
}
template <int NC>
__device__ __forceinline__ void st_refs(float* base, uint32_t cell, const float (&r)[NC]) {
  if constexpr (NC == 1) {
    st(base, cell * 4u, r[0]);
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 w;
    w.x = r[0];
    w.y = r[1];
    st(reinterpret_cast<f2*>(base), cell * 8u, w);
  }
}

// ------------------------------------------------------ population layout
// Plane i of a population buffer holds direction i of every cell of every
// slot, with the components of a cell side by side: component a of cell c
// (slot * slot_cells + in-block index) is element (i * plane + c) * ncomp + a.  A
// link's values for every component then travel in one load and one store,
// which halves the memory instructions of the two-component step (the step
// kernels are bound by how many they issue, not by the bytes).  Opposite
// directions are adjacent planes (2p - 1, 2p): a pull reaches either plane
// of a pair from the pair's base with a 32-bit byte offset, and the host
// keeps 2 * plane * ncomp * sizeof(value) within 2^32.
__host__ __device__ __forceinline__ size_t pop_index(int i, uint32_t c, int a, int ncomp, uint32_t plane) {
  return ((size_t)i * plane + c) * (size_t)ncomp + (size_t)a;
}

typedef float float2v __attribute__((ext_vector_type(2)));

// The NC stored values of one link, loaded with one instruction at byte
// offset off from base.
template <typename T, int NC>
__device__ __forceinline__ void ld_link(const T* base, uint32_t off, T (&v)[NC]) {
  static_assert(NC == 1 || NC == 2, "one or two components");
  if constexpr (NC == 1) {
    v[0] = ld(base, off);
  } else if constexpr (std::is_same<T, float>::value) {
    const float2v w = ld(reinterpret_cast<const float2v*>(base), off);
    v[0] = w.x;
    v[1] = w.y;
  } else {
    const uint32_t w = ld(reinterpret_cast<const uint32_t*>(base), off);
    v[0] = __ushort_as_half((unsigned short)(w & 0xFFFFu));
    v[1] = __ushort_as_half((unsigned short)(w >> 16));
  }
}

// Stores the NC values of one link with one instruction; STREAM: with the
// non-temporal hint.
template <bool STREAM, typename T, int NC>
__device__ __forceinline__ void st_link(T* base, uint32_t off, const T (&v)[NC]) {
  static_assert(NC == 1 || NC == 2, "one or two components");
  if constexpr (NC == 1) {
    if constexpr (STREAM)
      st_stream(base, off, v[0]);
    else
      st(base, off, v[0]);
  } else if constexpr (std::is_same<T, float>::value) {
    float2v w;
    w.x = v[0];
    w.y = v[1];
    float2v* p = reinterpret_cast<float2v*>(reinterpret_cast<char*>(base) + off);
    if constexpr (STREAM)
      __builtin_nontemporal_store(w, p);
    else
      *p = w;
  } else {
    const uint32_t w = (uint32_t)__half_as_ushort(v[0]) | ((uint32_t)__half_as_ushort(v[1]) << 16);
    uint32_t* p = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + off);
    if constexpr (STREAM)
      __builtin_nontemporal_store(w, p);
    else
      *p = w;
  }
}

// --------------------------------------------------------- storage codecs
struct StoreF32 {
  using T = float;
  static constexpr bool kRef = false;
  __device__ static __forceinline__ float decode(T v, float) { return v; }
  __device__ static __forceinline__ T encode(float f, float) { return f; }
  static constexpr float kScale = 1.0f;
  __device__ static __forceinline__ T encode_scaled(float f, float) { return f; }
  __device__ static __forceinline__ uint32_t bits(T v) { return __float_as_uint(v); }
};

// FP16 deviation from w_i rho_ref, scaled by 2^12 (wr = w_i * rho_ref).
struct StoreF16 {
  using T = __half;
  static constexpr bool kRef = true;
  static constexpr float kScale = 4096.0f;
  static constexpr float kInvScale = 1.0f / 4096.0f;
  // wr + h 2^-12 as one fused multiply-add: the product is exact (a power-of-two
  // scaling of a half value, never below the FP32 normal range), so the one
  // rounding is that of the addition, the same bits as the separate operations
  __device__ static __forceinline__ float decode(T v, float wr) { return __builtin_fmaf(__half2float(v), kInvScale, wr); }
  __device__ static __forceinline__ T encode(float f, float wr) { return __float2half_rn((f - wr) * kScale); }
  // encode with the reference given already scaled, wrs = wr 2^12 (exact):
  // f 2^12 - wrs is (f - wr) 2^12 before its one rounding, so the fused form
  // gives the bits of encode(f, wr)
  __device__ static __forceinline__ T encode_scaled(float f, float wrs) {
    return __float2half_rn(__builtin_fmaf(f, kScale, -wrs));
  }
  __device__ static __forceinline__ uint32_t bits(T v) { return (uint32_t)__half_as_ushort(v); }
};

// --------------------------------------------------------------- moments
// Eq 4-5.  Momentum is accumulated over opposite pairs so that a population
// set symmetric under reflection gives exactly zero.
struct Mom {
  float rho, jx, jy, jz;
};

// Momentum of f, with its density already summed (by moments() on the same
// values, so the bits are those moments() would give).
__device__ __forceinline__ Mom moments_with_rho(const float f[kQ], float rho) {
  Mom m;
  const float d1 = f[1] - f[2], d3 = f[3] - f[4], d5 = f[5] - f[6];
  const float d7 = f[7] - f[8], d9 = f[9] - f[10], d11 = f[11] - f[12];
  const float d13 = f[13] - f[14], d15 = f[15] - f[16], d17 = f[17] - f[18];
  m.rho = rho;
  m.jx = (((d1 + d7) + d9) + d11) + d13;
  m.jy = (((d3 + d7) - d9) + d15) + d17;
  m.jz = (((d5 + d11) - d13) + d15) - d17;
  return m;
}

__device__ __forceinline__ Mom moments(const float f[kQ]) {
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
  return moments_with_rho(f, r);
}

// ------------------------------------------------------------------- EOS
// Eq 7 (Peng-Robinson, denominator 1 + 2 b rho - b^2 rho^2) and Eq 6.  A
// negative radicand gives psi = 0 and is reported through `clamped`.
// The two terms of Eq 7 are put over their common denominator, divided by
// with the hardware reciprocal (1 ulp), and the square root is the hardware
// one (1 ulp).
__device__ __forceinline__ float pseudo_potential(const Params& P, int a, float rho, bool& clamped) {
  const float g = P.g_self[a];
  clamped = false;
  if (g == 0.0f) return 0.0f;
  const float brho = P.b * rho;
  const float d1 = 1.0f - brho, d2 = (1.0f + 2.0f * brho) - brho * brho;
  const float p = ((rho * P.RT) * d2 - (P.a_theta * rho * rho) * d1) * __builtin_amdgcn_rcpf(d1 * d2);
  const float rad = (p - kThird * rho) * (6.0f / g);  // 2 (p - c_s^2 rho) / (c_s^2 g)
  if (!(rad >= 0.0f)) {
    clamped = true;
    return 0.0f;
  }
  return __builtin_amdgcn_sqrtf(rad);
}

// -------------------------------------------------------------- forcing
struct Vec3 {
  float x, y, z;
};

// Eq 8-9 read with lattice weights (the paper's weights being 6 w_i):
//   F_a = -beta g_aa psi_a(x) sum w_i psi_a(x+e_i) e_i
//         - (1-beta)/2 g_aa sum w_i psi_a(x+e_i)^2 e_i
//         - g_ab psi_a(x) sum w_i psi_b(x+e_i) e_i
// for every component at once (add_body adds rho_a body_a).  nb(a, i) returns psi of component a at x+e_i,
// already replaced by the centre value where x + e_i is solid or outside.
// Stencil sums run over opposite pairs, so a uniform psi gives exactly zero.
template <int NC, typename NB>
__device__ __forceinline__ void interaction_forces(const Params& P, const float psi_c[NC], NB&& nb, Vec3 F[NC]) {
  Vec3 s1[NC], s2[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) s1[a] = s2[a] = Vec3{0.0f, 0.0f, 0.0f};
  unroll<9>([&](auto K) {
    constexpr int i = 2 * decltype(K)::value + 1;  // pair (i, i+1), e_{i+1} = -e_i
    constexpr int ex = dir_ex(i), ey = dir_ey(i), ez = dir_ez(i);
    constexpr float w = dir_w(i);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const float p = nb(a, i), q = nb(a, i + 1);
      const float d1 = w * (p - q);
      const float d2 = d1 * (p + q);  // w (p^2 - q^2)
      if constexpr (ex != 0) {
        s1[a].x = ex > 0 ? s1[a].x + d1 : s1[a].x - d1;
        s2[a].x = ex > 0 ? s2[a].x + d2 : s2[a].x - d2;
      }
      if constexpr (ey != 0) {
        s1[a].y = ey > 0 ? s1[a].y + d1 : s1[a].y - d1;
        s2[a].y = ey > 0 ? s2[a].y + d2 : s2[a].y - d2;
      }
      if constexpr (ez != 0) {
        s1[a].z = ez > 0 ? s1[a].z + d1 : s1[a].z - d1;
        s2[a].z = ez > 0 ? s2[a].z + d2 : s2[a].z - d2;
      }
    }
  });
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const float c1 = -P.beta * P.g_self[a] * psi_c[a];
    const float c2 = -0.5f * (1.0f - P.beta) * P.g_self[a];
    F[a].x = c1 * s1[a].x + c2 * s2[a].x;
    F[a].y = c1 * s1[a].y + c2 * s2[a].y;
    F[a].z = c1 * s1[a].z + c2 * s2[a].z;
    if constexpr (NC == 2) {
      const int b = 1 - a;
      const float c3 = -P.g_cross * psi_c[a];
      F[a].x = F[a].x + c3 * s1[b].x;
      F[a].y = F[a].y + c3 * s1[b].y;
      F[a].z = F[a].z + c3 * s1[b].z;
    }
  }
}

// Extra body force per unit density (gravity, section 2.2), added last.
__device__ __forceinline__ Vec3 add_body(const Params& P, int a, Vec3 F, float rho) {
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
// Both are split over each opposite pair (e_j = -e_i) into a part even in e
// (shared) and a part odd in e (sign flipped), which halves the work.
// The collision conserves the cell's mass exactly, so the rest population is
// taken as the remainder rho - sum_{i>0} f*_i: with FP32 weights (whose sum
// exceeds 1 by 1.5e-8) the direct formula would add that much mass per step.
template <typename Emit>
__device__ __forceinline__ void collide_emit(float omega, const float f[kQ], const Mom& m, const Vec3& F,
                                             Emit&& emit) {
  float inv = 0.0f;
  if (m.rho > 0.0f) inv = __builtin_amdgcn_rcpf(m.rho);  // 1 ulp
  const float ux = m.jx * inv, uy = m.jy * inv, uz = m.jz * inv;
  const float dx = F.x * inv, dy = F.y * inv, dz = F.z * inv;
  const float sx = (ux + ux) + dx, sy = (uy + uy) + dy, sz = (uz + uz) + dz;  // u + v
  const float usq = (ux * ux + uy * uy) + uz * uz;
  const float dus = (dx * sx + dy * sy) + dz * sz;
  const float e0 = 1.0f - 1.5f * usq;  // even part of feq / (w rho), without (e.u)^2
  const float d0 = -1.5f * dus;        // even part of the forcing bracket, without (e.du)(e.s)
  // per weight class: w rho, 3 w rho, 4.5 w rho
  const float wa = (1.0f / 18.0f) * m.rho, wd = (1.0f / 36.0f) * m.rho;
  const float wa3 = 3.0f * wa, wd3 = 3.0f * wd, wa45 = 4.5f * wa, wd45 = 4.5f * wd;
  const float wae = wa * e0, wde = wd * e0, wad = wa * d0, wdd = wd * d0;
  float rest = 0.0f;
  unroll<9>([&](auto K) {
    constexpr int i = 2 * decltype(K)::value + 1, j = i + 1;
    constexpr int ex = dir_ex(i), ey = dir_ey(i), ez = dir_ez(i);
    constexpr bool axis = i <= 6;
    const float w3 = axis ? wa3 : wd3, w45 = axis ? wa45 : wd45, we = axis ? wae : wde, wdv = axis ? wad : wdd;
    const float eu = edot<ex, ey, ez>(ux, uy, uz);
    const float ed = edot<ex, ey, ez>(dx, dy, dz);
    const float es = edot<ex, ey, ez>(sx, sy, sz);
    // explicit fused multiply-adds: the same rounding in every kernel that
    // inlines this function (no contraction is left to the compiler)
    const float even = __builtin_fmaf(w45, eu * eu, we);
    const float odd = w3 * eu;
    const float deven = __builtin_fmaf(w45, ed * es, wdv);
    const float dodd = w3 * ed;
    const float oi = __builtin_fmaf(omega, (even + odd) - f[i], f[i]) + (deven + dodd);
    const float oj = __builtin_fmaf(omega, (even - odd) - f[j], f[j]) + (deven - dodd);
    emit(std::integral_constant<int, i>{}, oi);
    emit(std::integral_constant<int, j>{}, oj);
    rest = i == 1 ? (oi + oj) : rest + (oi + oj);
  });
  emit(std::integral_constant<int, 0>{}, m.rho - rest);
}

__device__ __forceinline__ void collide(float omega, const float f[kQ], const Mom& m, const Vec3& F,
                                        float out[kQ]) {
  collide_emit(omega, f, m, F, [&](auto I, float v) { out[decltype(I)::value] = v; });
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

__host__ __device__ __forceinline__ int sgn_out(int s) { return s < 0 ? -1 : (s > 15 ? 1 : 0); }

// Index of cell (x, y, z) within a block: x and y in tiles of 8 x 4 (one
// 128-byte line of an FP32 population plane per tile), z planes outermost.
// A face of the block then spans 4 (x faces) or 2 (y faces) lines of a plane
// instead of 8 or 1, so the halo a neighbouring block reads touches fewer lines.
__host__ __device__ constexpr uint32_t cell_x(int x) { return (uint32_t)((x & 7) + 32 * ((x >> 3) & 1)); }
__host__ __device__ constexpr uint32_t cell_y(int y) { return (uint32_t)(8 * (y & 3) + 64 * ((y >> 2) & 3)); }
__host__ __device__ constexpr uint32_t cell_of(int x, int y, int z) { return cell_x(x) + cell_y(y) + 256u * (uint32_t)z; }
__host__ __device__ __forceinline__ void cell_xyz(int c, int& x, int& y, int& z) {
  x = (c & 7) + 8 * ((c >> 5) & 1);
  y = ((c >> 3) & 3) + 4 * ((c >> 6) & 3);
  z = c >> 8;
}

// Sources of the 19 populations arriving at a cell.  fidx[i] is the element
// index of the value within the two planes of direction i's opposite pair
// (plane offset included); for the FP16 store ridx[i] is the source cell's
// index, where its reference density lives.  A bounced link (mask bit i:
// x - e_i is solid or outside) reads the cell's own opposite population.
template <bool REF>
struct Sources {
  uint32_t fidx[kQ];
  uint32_t ridx[REF ? kQ : 1];
};

// Per-thread precomputation for the pulls.  For a shift s in {-1, 0, +1}
// along an axis, the word (offset of the neighbour block along that axis,
// scaled by 1, 3 or 9, in the high half) << 16 + (in-block coordinate of the
// source, scaled by 1, 16 or 256) is stored, so that the sum of the three
// words for a direction gives (neighbour index d << 16) + source cell in one
// add: the low halves sum to at most 4095 and d lies in [0, 26].
struct PullAxes {
  uint32_t ax[3], ay[3], az[3];
};

__host__ __device__ __forceinline__ uint32_t pack_axis(int v, int shift, int scale_d, int axis, int bias) {
  const int sv = v + shift;
  const int o = sv < 0 ? -1 : (sv > 15 ? 1 : 0);
  const uint32_t c = axis == 0 ? cell_x(sv & 15) : (axis == 1 ? cell_y(sv & 15) : 256u * (uint32_t)(sv & 15));
  return ((uint32_t)(bias + scale_d * o) << 16) + c;
}

__host__ __device__ __forceinline__ void pull_axes_xy(int x, int y, PullAxes& a) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.ax[k] = pack_axis(x, k - 1, 1, 0, 0);
    a.ay[k] = pack_axis(y, k - 1, 3, 1, 0);
  }
}
__host__ __device__ __forceinline__ void pull_axes_z(int z, PullAxes& a) {
#pragma unroll
  for (int k = 0; k < 3; ++k) a.az[k] = pack_axis(z, k - 1, 9, 2, 13);
}

template <int RD, bool REF>
__host__ __device__ __forceinline__ void sources(const PullAxes& pa, uint32_t own, uint32_t m, uint32_t plane,
                                        const int* nslot, int rest, uint32_t slot_cells, Sources<REF>& s) {
  s.fidx[0] = own;
  if constexpr (REF) s.ridx[0] = own;
  const uint32_t own_second = own + plane;
  if constexpr (RD == kRdOwn) {
    unroll<kQ - 1>([&](auto K) {
      constexpr int i = decltype(K)::value + 1;
      constexpr bool second = !(i & 1);  // plane i is the second of its pair
      s.fidx[i] = second ? own_second : own;
      if constexpr (REF) s.ridx[i] = own;
    });
  } else {
    // all slot lookups first (independent table reads), then the addresses
    uint32_t w[kQ];
    int slot[kQ];
    unroll<kQ - 1>([&](auto K) {
      constexpr int i = decltype(K)::value + 1;
      w[i] = pa.ax[1 - dir_ex(i)] + pa.ay[1 - dir_ey(i)] + pa.az[1 - dir_ez(i)];  // source = x - e_i
    });
    unroll<kQ - 1>([&](auto K) {
      constexpr int i = decltype(K)::value + 1;
      slot[i] = nslot[w[i] >> 16];
    });
    unroll<kQ - 1>([&](auto K) {
      constexpr int i = decltype(K)::value + 1;
      constexpr bool second = !(i & 1);  // plane i is the second of its pair
      const uint32_t src_cell = (uint32_t)slot[i] * slot_cells + (w[i] & 0xFFFFu);
      const bool bounce = (m >> i) & 1u;
      const uint32_t own_i = second ? own_second : own;   // (x, plane i)
      const uint32_t own_o = second ? own : own_second;   // (x, plane of the opposite direction)
      const uint32_t src_i = second ? src_cell + plane : src_cell;
      const uint32_t src_o = second ? src_cell : src_cell + plane;
      if constexpr (RD == kRdPull) {
        // bounced: the cell's own population of the opposite direction, which
        // is the other plane of the pair
        s.fidx[i] = bounce ? own_o : src_i;
      } else if constexpr (RD == kRdAAOdd) {
        // f*_i(x - e_i) sits at (x - e_i, opposite plane); a bounced link's
        // value at (x, plane i)
        s.fidx[i] = bounce ? own_i : src_o;
      } else {
        // streamed in place to (x, plane i); a link from a block that did
        // not take part in the last step carries the rest state, read from
        // the rest slot (which stores it swapped, like a post-collision cell)
        s.fidx[i] = (bounce || slot[i] != rest) ? own_i : src_o;
      }
      // reference density (FP16 store): that of the cell that wrote the
      // value, which is the source cell, or the cell itself for a bounced link
      if constexpr (REF) s.ridx[i] = bounce ? own : src_cell;
    });
  }
}

// Populations of every component arriving at the cell (decoded to FP32),
// one load per link.  refs(I, r): the FP16 store's reference densities of
// every component for direction I, into r[NC] (not called with the FP32
// store).
template <typename S, int NC, typename Refs>
__device__ __forceinline__ void gather_links(const typename S::T* __restrict__ fb, uint32_t plane,
                                             const Sources<S::kRef>& s, Refs&& refs, float f[NC][kQ]) {
  using T = typename S::T;
  constexpr uint32_t stride = NC * sizeof(T);
  unroll<kQ>([&](auto K) {
    constexpr int i = decltype(K)::value;
    constexpr int first = i == 0 ? 0 : ((i & 1) ? i : i - 1);  // first plane of the pair
    T v[NC];
    ld_link<T, NC>(fb + (size_t)first * plane * NC, s.fidx[i] * stride, v);
    if constexpr (S::kRef) {
      float r[NC];
      refs(K, r);
#pragma unroll
      for (int a = 0; a < NC; ++a) f[a][i] = S::decode(v[a], dir_w(i) * r[a]);
    } else {
#pragma unroll
      for (int a = 0; a < NC; ++a) f[a][i] = S::decode(v[a], 0.0f);
    }
  });
}

// Populations of component a (of NC) arriving at the cell (decoded to FP32).
//   fb: buffer base; plane: cells per plane; rref: densities of the previous
//   step (FP16 store only).
template <typename S, int NC>
__device__ __forceinline__ void gather(const typename S::T* __restrict__ fb, uint32_t plane, int a,
                                       const Sources<S::kRef>& s, const float* __restrict__ rref, float f[kQ]) {
  using T = typename S::T;
  constexpr uint32_t stride = NC * sizeof(T);
  const T* base0 = fb + a;  // component a of every link
  const float* rbase = S::kRef ? rref + a : nullptr;  // component a of each cell's references
  unroll<kQ>([&](auto K) {
    constexpr int i = decltype(K)::value;
    constexpr int first = i == 0 ? 0 : ((i & 1) ? i : i - 1);  // first plane of the pair
    const T v = ld(base0 + (size_t)first * plane * NC, s.fidx[i] * stride);
    float wr = 0.0f;
    if constexpr (S::kRef) wr = dir_w(i) * ld(rbase, s.ridx[i] * (uint32_t)(4 * NC));
    f[i] = S::decode(v, wr);
  });
}

// The 27 neighbour slots of a block (inactive and outside -> rest slot),
// their block ids (-1 outside) and the candidate mask: neighbours that are
// inside the domain, inactive and hold fluid.
struct BlockCtx {
  int nslot[27];
  int nbk[27];
  unsigned cand;
  unsigned fired;
};

__device__ __forceinline__ void setup_block(const Params& P, const Buffers& D, int blk, BlockCtx& ctx) {
  const int t = threadIdx.x;
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  bool cand = false;
  if (t < 27) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int nbid = neighbour_block(P, bx, by, bz, dx, dy, dz);
    int sl = nbid < 0 ? -1 : D.block_slot[nbid];
    if (t != 13 && nbid >= 0 && sl < 0 && D.bfluid[nbid]) cand = true;
    if (sl < 0) sl = P.capacity;
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

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup g runs on
// XCD g mod 8), and each XCD has its own L2.  Give XCD k the contiguous run of
// slots [k*chunk, (k+1)*chunk): blocks next to each other in slot order (x
// neighbours on the static mesh) then run together on one L2, and the cache
// lines they share (the row that x-shifted pulls read from both sides) are
// fetched once.  Grids are launched with a multiple of 8 workgroups.
constexpr int kXcds = 8;
// Returns n_active (no slot) for workgroups beyond the active range.
__device__ __forceinline__ int slot_of_workgroup(int g, int n_active) {
  const int chunk = (n_active + kXcds - 1) / kXcds;
  const int q = g / kXcds;
  if (q >= chunk) return n_active;
  const int s = (g % kXcds) * chunk + q;
  return s < n_active ? s : n_active;
}
__host__ __device__ constexpr int grid_for(int capacity) { return (capacity + kXcds - 1) / kXcds * kXcds; }

// Simulation of position gi of a batch's merged active list: the last i with
// off[i] <= gi (members without active blocks have off[i] == off[i + 1]).
__device__ __forceinline__ int batch_sim(const Batch& B, int gi) {
  int lo = 0, hi = B.nsims - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (B.off[mid] <= gi)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename S>
__device__ __forceinline__ typename S::T* fplane(const Buffers& D, int buf) {
  return reinterpret_cast<typename S::T*>(D.f[buf]);
}

// Stored form of the rest population of (a, i), from the bits the host
// copied into Params.
template <typename S>
__device__ __forceinline__ typename S::T rest_stored(const Params& P, int a, int i) {
  if constexpr (std::is_same<typename S::T, float>::value)
    return __uint_as_float(P.f_rest_bits[a][i]);
  else
    return __ushort_as_half((unsigned short)P.f_rest_bits[a][i]);
}

// Batched kernels copy their member's Params and Buffers into LDS once per
// workgroup: read through a reference into global memory, every field would
// be loaded again after each global store, which the compiler must assume
// could overwrite it.
template <typename T>
__device__ __forceinline__ void stage_struct(T& dst, const T& src) {
  static_assert(sizeof(T) % 4 == 0, "word copy");
  const uint32_t* s = reinterpret_cast<const uint32_t*>(&src);
  uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
  for (int k = threadIdx.x; k < (int)(sizeof(T) / 4); k += blockDim.x) d[k] = s[k];
}

// ----------------------------------------------------------- rest state
// Iterates the update of a cell whose every neighbour is itself (uniform
// lattice at rest, density bg) until the stored populations (and, for the
// FP16 store, the reference density) stop changing; the same device
// functions as k_fused, so the result is a fixed point of the real update.  Single thread; tiny.
//   out: [2*19] stored bits, then decoded populations [2*19], then
//   reference density [2], density [2], psi [2] (as floats).
template <typename S, int NC>
__global__ void k_rest_state(Params P, const float* bg, float* out, int* iters) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int a = 0; a < kMaxComp; ++a) P.body[a][0] = P.body[a][1] = P.body[a][2] = 0.0f;
  typename S::T h[NC][kQ];
  float r[NC];
  for (int a = 0; a < NC; ++a) {
    r[a] = bg[a];
    for (int i = 0; i < kQ; ++i) h[a][i] = S::encode(dir_w(i) * bg[a], dir_w(i) * r[a]);
  }
  int it = 0;
  for (; it < 100000; ++it) {
    float f[NC][kQ], psi[NC], rho[NC];
    Mom m[NC];
    for (int a = 0; a < NC; ++a) {
      for (int i = 0; i < kQ; ++i) f[a][i] = S::decode(h[a][i], dir_w(i) * r[a]);
      m[a] = moments(f[a]);
      bool cl;
      psi[a] = pseudo_potential(P, a, m[a].rho, cl);
      rho[a] = m[a].rho;
    }
    Vec3 F[NC];
    interaction_forces<NC>(P, psi, [&](int a, int) { return psi[a]; }, F);
    bool same = true;
    typename S::T nh[NC][kQ];
    for (int a = 0; a < NC; ++a) {
      float o[kQ];
      collide(P.omega[a], f[a], m[a], add_body(P, a, F[a], rho[a]), o);
      for (int i = 0; i < kQ; ++i) {
        nh[a][i] = S::encode(o[i], dir_w(i) * m[a].rho);
        same = same && (S::bits(nh[a][i]) == S::bits(h[a][i]));
      }
      same = same && (__float_as_uint(m[a].rho) == __float_as_uint(r[a]));
    }
    for (int a = 0; a < NC; ++a) {
      r[a] = m[a].rho;
      for (int i = 0; i < kQ; ++i) h[a][i] = nh[a][i];
    }
    if (same) break;
  }
  for (int a = 0; a < NC; ++a) {
    float f[kQ];
    for (int i = 0; i < kQ; ++i) {
      f[i] = S::decode(h[a][i], dir_w(i) * r[a]);
      out[a * kQ + i] = __uint_as_float(S::bits(h[a][i]));
      out[kMaxComp * kQ + a * kQ + i] = f[i];
    }
    const Mom m = moments(f);
    bool cl;
    out[4 * kQ + a] = r[a];
    out[4 * kQ + kMaxComp + a] = m.rho;
    out[4 * kQ + 2 * kMaxComp + a] = pseudo_potential(P, a, m.rho, cl);
  }
  *iters = it;
}

// ----------------------------------------------------------- slot init
// Initialises slots [first, first+count): per-cell mask (links that bounce,
// cell kind), populations of buffer `buf` (placed as `mode` says), psi,
// reference densities and the criterion history.  Slot `capacity` (the rest
// slot) is initialised the same way with the rest state everywhere and an
// all-fluid mask.  A workgroup takes a sixteenth of a slot (256 cells, one
// per thread) at a time, so that a handful of new blocks still spreads over
// many compute units and no thread waits for the loads of a second cell
// (a quarter, four cells per thread, took 1.7x as long per growth step); the
// stored rest populations come from LDS.
constexpr int kInitParts = 16;

template <typename S, bool BATCH>
__global__ void __launch_bounds__(256) k_init(Params Pv, Buffers Dv, int buf, int first_h, int count_h, int from_dev,
                                              int use_init, Batch Bt, int mode, int born) {
  // batched: blockIdx.y selects the simulation
  constexpr bool batched = BATCH;
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  if constexpr (BATCH) {
    stage_struct(P_s, Bt.P[blockIdx.y]);
    stage_struct(D_s, Bt.D[blockIdx.y]);
    __syncthreads();
  }
  const Params& P = BATCH ? P_s : Pv;
  const Buffers& D = BATCH ? D_s : Dv;
  const int first = from_dev ? D.ctrl[kNewFirst] : first_h;
  const int count = from_dev ? D.ctrl[kNewCount] : count_h;
  if (count <= 0) return;  // the same value for the whole workgroup
  if (batched) born = D.ctrl[kStepCount];  // the members' step, kept on the device
  __shared__ uint32_t rest_bits[kMaxComp][kQ];
  if (threadIdx.x < kMaxComp * kQ) {
    const int a = threadIdx.x / kQ, i = threadIdx.x % kQ;
    rest_bits[a][i] = P.f_rest_bits[a][i];
  }
  __syncthreads();
  const uint32_t plane = P.plane;
  const int ncomp = P.ncomp;
  typename S::T* fb = fplane<S>(D, buf);
  const long long N = (long long)P.nx * P.ny * P.nz;
  auto stored_rest = [&](int a, int i) -> typename S::T {
    const uint32_t bits = rest_bits[a][i];
    if constexpr (std::is_same<typename S::T, float>::value)
      return __uint_as_float(bits);
    else
      return __ushort_as_half((unsigned short)bits);
  };
  for (int u = blockIdx.x; u < count * kInitParts; u += gridDim.x) {
    const int slot = first + u / kInitParts;
    const int part = u % kInitParts;
    const bool rest_slot = slot == P.capacity;
    const int blk = rest_slot ? -1 : D.slot_block[slot];
    const int bx = rest_slot ? 0 : blk % P.nbx, by = rest_slot ? 0 : (blk / P.nbx) % P.nby,
              bz = rest_slot ? 0 : blk / (P.nbx * P.nby);
#pragma unroll 1
    for (int c = part * (kCells / kInitParts) + (int)threadIdx.x; c < (part + 1) * (kCells / kInitParts);
         c += (int)blockDim.x) {
      int x, y, z;
      cell_xyz(c, x, y, z);
      const uint32_t cid = (uint32_t)slot * P.slot_cells + c;
      uint32_t m = 0u;
      long long n = -1;
      const int X = bx * kB + x, Y = by * kB + y, Z = bz * kB + z;
      // cells beyond the lattice (padding of a block that a non-periodic
      // face cuts) are solid
      const bool pad = !rest_slot && (X >= P.nx || Y >= P.ny || Z >= P.nz);
      if (pad) m = (uint32_t)kSolid << kKindShift;
      if (!rest_slot && !pad) {
        n = X + (long long)P.nx * (Y + (long long)P.ny * Z);
        uint32_t kind = D.solid[n] ? kSolid : kFluid;
        if (kind == kFluid) {
          const bool on[6] = {X == 0, X == P.nx - 1, Y == 0, Y == P.ny - 1, Z == 0, Z == P.nz - 1};
#pragma unroll
          for (int fc = 0; fc < 6; ++fc)
            if (on[fc] && P.bc[fc] == kOutletFace) kind = kOutlet;
#pragma unroll
          for (int fc = 0; fc < 6; ++fc)
            if (on[fc] && P.bc[fc] == kInletFace) kind = kInlet;
        }
        m = kind << kKindShift;
        unroll<kQ - 1>([&](auto I) {
          constexpr int i = decltype(I)::value + 1;
          int sx = X - dir_ex(i), sy = Y - dir_ey(i), sz = Z - dir_ez(i);
          bool bounce = false;
          if (dir_ex(i) != 0 && (sx < 0 || sx >= P.nx)) {
            if (P.bc[0] != kPeriodic) bounce = true;
            sx = (sx + P.nx) % P.nx;
          }
          if (dir_ey(i) != 0 && (sy < 0 || sy >= P.ny)) {
            if (P.bc[2] != kPeriodic) bounce = true;
            sy = (sy + P.ny) % P.ny;
          }
          if (dir_ez(i) != 0 && (sz < 0 || sz >= P.nz)) {
            if (P.bc[4] != kPeriodic) bounce = true;
            sz = (sz + P.nz) % P.nz;
          }
          if (!bounce) bounce = D.solid[sx + (long long)P.nx * (sy + (long long)P.ny * sz)] != 0;
          if (bounce) m |= 1u << i;
        });
      }
      D.mask[cid] = m;
      if (c == 0 && !rest_slot) D.frontier[slot] = 1;
      // in place, before an even step: the links whose source cell lies in a
      // block that took part in the last step (active, not joining now)
      // take what that cell streamed towards this one (each such value has
      // one receiving link, so one thread moves it)
      uint32_t stash[kQ];
#pragma unroll
      for (int i = 0; i < kQ; ++i) stash[i] = ~0u;
      if (mode == kInitStash && !rest_slot && ((m >> kKindShift) & 3u) != kSolid) {
        unroll<kQ - 1>([&](auto I) {
          constexpr int i = decltype(I)::value + 1;
          if (!((m >> i) & 1u)) {  // bounced: rest, like every link from a solid cell
            const int sx = (X - dir_ex(i) + P.nx) % P.nx, sy = (Y - dir_ey(i) + P.ny) % P.ny,
                      sz = (Z - dir_ez(i) + P.nz) % P.nz;
            const int nbk = sx / kB + P.nbx * (sy / kB + P.nby * (sz / kB));
            const int sl = D.block_slot[nbk];
            if (sl >= 0 && D.act_step[nbk] != born)
              stash[i] = (uint32_t)sl * P.slot_cells + cell_of(sx & 15, sy & 15, sz & 15);
          }
        });
      }
      if (D.psi)
        for (int a = 0; a < ncomp; ++a) D.psi[(size_t)a * plane + cid] = P.psi_rest[a];
      for (int a = 0; a < ncomp; ++a) {
        float r0 = __int_as_float(0x7fc00000);  // NaN: rest state
        float ux = 0.0f, uy = 0.0f, uz = 0.0f;
        if (use_init && n >= 0 && D.init_rho) {
          r0 = D.init_rho[(long long)a * N + n];
          if (D.init_u) {
            ux = D.init_u[n];
            uy = D.init_u[N + n];
            uz = D.init_u[2 * N + n];
          }
        }
        const bool at_rest = !(r0 == r0);
        float fe[kQ];
        unroll<kQ>([&](auto I) {
          constexpr int i = decltype(I)::value;
          fe[i] = at_rest ? 0.0f : feq_dir(i, r0, ux, uy, uz);
        });
        // reference density of the FP16 store: the cell's own density
        const float rref = at_rest ? P.rho_ref_rest[a] : moments(fe).rho;
        unroll<kQ>([&](auto I) {
          constexpr int i = decltype(I)::value;
          typename S::T v = at_rest ? stored_rest(a, mode == kInitSwapped ? dir_opp(i) : i)
                                    : S::encode(fe[i], dir_w(i) * rref);
          if (stash[i] != ~0u) {
            // moved here; the sender's address reads as the rest state again
            typename S::T* sp = fb + pop_index(dir_opp(i), stash[i], a, ncomp, plane);
            v = *sp;
            *sp = stored_rest(a, dir_opp(i));
          }
          fb[pop_index(i, cid, a, ncomp, plane)] = v;
        });
        if constexpr (S::kRef) {
          D.rho[0][(size_t)cid * ncomp + a] = rref;
          D.rho[1][(size_t)cid * ncomp + a] = rref;
        }
        if (!rest_slot && D.uprev)
          for (int d = 0; d < 3; ++d) D.uprev[((size_t)(a * 3 + d)) * plane + cid] = 0.0f;
      }
    }
  }
}

// ------------------------------------------------------------ debug psi
// Test dump, first pass: psi (Eq 6-7) of every non-solid cell of the active
// blocks into a slot-indexed buffer, exactly as the step computes it (pulled
// densities; inlet nodes psi(inlet density), outlet nodes the rest value).
template <typename S, int NC, int RD>
__global__ void __launch_bounds__(kThreads) k_debug_psi(Params P, Buffers D, int rbuf, float* psi_out) {
  const int n_active = D.ctrl[kNActive];
  const int s = slot_of_workgroup(blockIdx.x, n_active);
  if (s >= n_active) return;
  __shared__ BlockCtx ctx;
  setup_block(P, D, D.slot_block[s], ctx);
  __syncthreads();
  int x, y, z0;
  cell_xyz((int)threadIdx.x, x, y, z0);
  PullAxes pa;
  pull_axes_xy(x, y, pa);
  const uint32_t plane = P.plane;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
#pragma unroll 1
  for (int z = z0; z < kB; z += kZStep) {
    const uint32_t cid = own_base + cell_of(x, y, z);
    const uint32_t m = ld(D.mask, cid * 4u);
    const uint32_t kind = (m >> kKindShift) & 3u;
    if (kind == kSolid) continue;
    Sources<S::kRef> src;
    pull_axes_z(z, pa);
    sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      float f[kQ];
      gather<S, NC>(fb, plane, a, src, rref, f);
      float psi = P.psi_rest[a];
      if (kind == kFluid) {
        bool cl;
        psi = pseudo_potential(P, a, moments(f).rho, cl);
      } else if (kind == kInlet) {
        psi = P.psi_in[a];
      }
      st(psi_out + (size_t)a * plane, cid * 4u, psi);
    }
  }
}

// -------------------------------------------------------------- activate
// K3: one workgroup of 1024 threads compacts the requested blocks (inactive,
// holding fluid) into new slots, in block order: slot = n_active + rank, with
// the rank from a wave ballot and a workgroup prefix sum.  Clears requests.
// When the criterion (or the proposal) recorded nothing since the last pass,
// the active set is unchanged and the pass only reports that no block is new.
template <bool BATCH>
__global__ void __launch_bounds__(1024) k_activate(Params Pv, Buffers Dv, int step_arg, Batch Bt) {
  // batched: one workgroup per simulation, whose step count is on the device
  const Params& P = BATCH ? Bt.P[blockIdx.x] : Pv;
  const Buffers& D = BATCH ? Bt.D[blockIdx.x] : Dv;
  const int step = BATCH ? D.ctrl[kStepCount] : step_arg;
  __shared__ int wave_count[16];
  __shared__ int wave_base[16];
  __shared__ int order_count[2][16];  // active blocks per wave: before and after this pass's new slots
  __shared__ int order_base[2][16];
  __shared__ int order_total[2];
  __shared__ int chunk_total;
  __shared__ int stop, chunk_stop;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int n0 = D.ctrl[kNActive];
  const int tr0 = D.ctrl[kTraceLen];
  if (D.ctrl[kPending] == 0) {  // the same value for the whole workgroup
    if (t == 0) {
      D.ctrl[kNewFirst] = n0;
      D.ctrl[kNewCount] = 0;
    }
    return;
  }
  // one pass over the blocks, 1024 at a time: every array a block needs is
  // loaded together, then two prefix sums (new slots, and the active list in
  // block order, which is the order the step kernel schedules them in, so
  // that neighbouring blocks run together and share one L2) take one round
  // of barriers
  int base = n0, obase = 0;
  unsigned long long leak = 0ull;  // failing links recorded by the criterion into blocks still inactive
  if (t == 0) stop = 0;
  for (int b0 = 0; b0 < P.nb; b0 += 1024) {
    const int b = b0 + t;
    int req = 0, sl = -1, fl = 0, e = 0;
    if (b < P.nb) {
      req = D.request[b];
      sl = D.block_slot[b];
      fl = D.bfluid[b];
      e = D.expose[b];
    }
    const int flag = (req && sl < 0 && fl) ? 1 : 0;
    const unsigned long long bal = __ballot(flag);
    const unsigned long long bal_old = __ballot(sl >= 0);
    const unsigned long long bal_new = bal | bal_old;
    const unsigned long long below = (1ull << lane) - 1ull;
    if (lane == 0) {
      wave_count[wave] = __popcll(bal);
      order_count[0][wave] = __popcll(bal_old);
      order_count[1][wave] = __popcll(bal_new);
    }
    // (the sums of the previous chunk are read by every thread before this
    // barrier, and written again only after it)
    __syncthreads();
    if (t == 0) {
      int acc = 0, acc_o[2] = {0, 0};
      for (int w = 0; w < 16; ++w) {
        wave_base[w] = acc;
        acc += wave_count[w];
        for (int k = 0; k < 2; ++k) {
          order_base[k][w] = acc_o[k];
          acc_o[k] += order_count[k][w];
        }
      }
      chunk_total = acc;
      order_total[0] = acc_o[0];
      order_total[1] = acc_o[1];
      // pool full: no slot in this chunk or after; their requests stay
      if (!stop && base + acc > P.capacity) stop = 1;
      chunk_stop = stop;
    }
    __syncthreads();
    const bool assign = !chunk_stop;  // the same value for the whole workgroup
    if (assign && flag) {
      const int rank = base - n0 + wave_base[wave] + __popcll(bal & below);
      sl = n0 + rank;
      D.block_slot[b] = sl;
      D.slot_block[sl] = b;
      D.act_step[b] = step;
      if (tr0 + rank < P.trace_cap) {
        D.trace[2 * (tr0 + rank)] = step;
        D.trace[2 * (tr0 + rank) + 1] = b;
      }
    }
    const int k = assign ? 1 : 0;
    if (sl >= 0) D.order[obase + order_base[k][wave] + __popcll((assign ? bal_new : bal_old) & below)] = sl;
    // a leak if the target block is still inactive now that this step's
    // activations are done
    if (e) {
      if (sl < 0) leak += (unsigned long long)e;
      D.expose[b] = 0;
    }
    if (assign && b < P.nb) D.request[b] = 0;
    if (assign) base += chunk_total;
    obase += order_total[k];
  }
  if (leak) atomicAdd(&D.counters[0], leak);
  if (t == 0) {
    D.ctrl[kNewFirst] = n0;
    D.ctrl[kNewCount] = base - n0;
    D.ctrl[kNActive] = base;
    D.ctrl[kTraceLen] = tr0 + (base - n0);
    if (stop) D.ctrl[kPoolFull] = 1;
    D.ctrl[kPending] = stop;  // requests that did not fit stay pending
  }
}

// ----------------------------------------------------------- debug force
// Test dump, second pass: psi and the total force (Eq 8-9 plus body force)
// of every non-solid cell of the active blocks, written to lattice-wide
// arrays.  Psi of the 18^3 halo is staged in LDS from the first pass;
// inactive and outside blocks show the rest value.
constexpr int kH = kB + 2;            // halo edge
constexpr int kRW = kB + 4;           // edge of the FP16 reference footprint
constexpr int kHalo = kH * kH * kH;   // 5832 cells

__device__ __forceinline__ int hidx(int x, int y, int z) { return (x + 1) + kH * ((y + 1) + kH * (z + 1)); }

template <typename S, int NC, int RD>
__global__ void __launch_bounds__(kThreads) k_debug_force(Params P, Buffers D, int rbuf, const float* psi_slots,
                                                          float* dbg_psi, float* dbg_force) {
  const int n_active = D.ctrl[kNActive];
  const int s = slot_of_workgroup(blockIdx.x, n_active);
  if (s >= n_active) return;
  __shared__ BlockCtx ctx;
  __shared__ float psi_s[NC * kHalo];
  const int blk = D.slot_block[s];
  setup_block(P, D, blk, ctx);
  __syncthreads();
  const uint32_t plane = P.plane;
  for (int h = threadIdx.x; h < kHalo; h += blockDim.x) {
    const int hx = h % kH - 1, hy = (h / kH) % kH - 1, hz = h / (kH * kH) - 1;
    const int d = 13 + sgn_out(hx) + 3 * sgn_out(hy) + 9 * sgn_out(hz);
    const int slot = ctx.nslot[d];
    const uint32_t cid = (uint32_t)slot * P.slot_cells + cell_of(hx & 15, hy & 15, hz & 15);
#pragma unroll
    for (int a = 0; a < NC; ++a)
      psi_s[a * kHalo + h] = slot == P.capacity ? P.psi_rest[a] : ld(psi_slots + (size_t)a * plane, cid * 4u);
  }
  __syncthreads();
  int x, y, z0;
  cell_xyz((int)threadIdx.x, x, y, z0);
  PullAxes pa;
  pull_axes_xy(x, y, pa);
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  const long long N = (long long)P.nx * P.ny * P.nz;
#pragma unroll 1
  for (int z = z0; z < kB; z += kZStep) {
    const uint32_t cid = own_base + cell_of(x, y, z);
    const uint32_t m = ld(D.mask, cid * 4u);
    const uint32_t kind = (m >> kKindShift) & 3u;
    if (kind == kSolid) continue;
    const int h0 = hidx(x, y, z);
    float psi_c[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) psi_c[a] = psi_s[a * kHalo + h0];
    Vec3 F[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) F[a] = Vec3{0.0f, 0.0f, 0.0f};
    if (kind == kFluid)
      interaction_forces<NC>(P, psi_c,
                             [&](int a, int i) {
                               const int hn = h0 + dir_ex(i) + kH * (dir_ey(i) + kH * dir_ez(i));
                               const bool solid_nb = (m >> dir_opp(i)) & 1u;  // x + e_i solid or outside
                               return solid_nb ? psi_c[a] : psi_s[a * kHalo + hn];
                             },
                             F);
    Sources<S::kRef> src;
    pull_axes_z(z, pa);
    sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
    const long long n = (bx * kB + x) + (long long)P.nx * ((by * kB + y) + (long long)P.ny * (bz * kB + z));
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      float f[kQ];
      gather<S, NC>(fb, plane, a, src, rref, f);
      const Vec3 Fa = kind == kFluid ? add_body(P, a, F[a], moments(f).rho) : F[a];
      dbg_psi[a * N + n] = psi_c[a];
      dbg_force[(a * 3 + 0) * N + n] = Fa.x;
      dbg_force[(a * 3 + 1) * N + n] = Fa.y;
      dbg_force[(a * 3 + 2) * N + n] = Fa.z;
    }
  }
}

// ------------------------------------------------------------ fused step
// The production step kernel: moments, pseudo-potential, forces, collision
// and streaming in one pass over the populations.  One workgroup per active
// block.  Thread t owns a column of the block's 18 x 18 footprint (the block
// plus a one-cell ring): t < 256 the 16 x 16 interior (four full waves, each
// on two whole tiles), 256 <= t < 324 the ring.  The workgroup sweeps the planes
// z = -1 .. 16.  At plane z every column pulls its cell's populations,
// computes rho and psi (Eq 4-7) and puts psi in a ring of four LDS planes;
// after one barrier the interior threads collide their cell of plane z - 1
// (forces from the three LDS planes z-2 .. z, Eq 8-12) with the populations
// they pulled one plane earlier and still hold in registers, and store f*.
// Cells of inactive blocks (and outside the domain) are frozen at the rest
// state: they contribute psi_rest without being pulled.  Psi never goes to
// memory; the populations are read once (plus the ring and the two halo
// planes, which neighbouring blocks also read) and written once.
constexpr int kFusedThreads = 384;
constexpr int kPsiRing = 4;
constexpr int kFoot = kH * kH;  // 324 columns

// The work of one workgroup: planes [z0, z0 + 16/parts) of the block in
// position g of the active list (with the halo planes on either side).
template <typename S, int NC, bool PULL>
__device__ __forceinline__ void fused_block(const Params& P, const Buffers& D, int rbuf, int g, int part,
                                            int parts) {
  const int zlen = kB / parts, z0 = part * zlen;
  const int s = D.order[g];  // active slots in block order
  __shared__ BlockCtx ctx;
  __shared__ float psi_s[kPsiRing][NC][kFoot];
  __shared__ uint32_t mask_s[2][kFusedThreads];
  __shared__ float f_in_s[NC][kQ], f_rest_s[NC][kQ];
  // FP16 store: the previous step's densities (the references of the stored
  // deviations) of a 20 x 20 footprint, x and y in [-2, 17], four planes in a
  // ring (plane p in slot p & 3), so that a pull decodes its 19 values with
  // LDS reads instead of 19 more loads per component
  __shared__ float rref_s[S::kRef ? kPsiRing : 1][NC][S::kRef ? kRW * kRW : 1];
  setup_block(P, D, D.slot_block[s], ctx);
  if (threadIdx.x >= 64 && threadIdx.x < 64 + NC * kQ) {
    const int k = threadIdx.x - 64, a = k / kQ, i = k % kQ;
    f_in_s[a][i] = P.f_in[a][i];
    f_rest_s[a][i] = P.f_rest[a][i];
  }
  __syncthreads();
  const int t = threadIdx.x;
  const bool col = t < kFoot;
  const bool interior = t < 256;
  int cx, cy;
  if (interior) {
    int cz;
    cell_xyz(t, cx, cy, cz);  // consecutive threads take consecutive cells of a plane
  } else {
    const int r = col ? t - 256 : 0;  // ring: rows y = -1, 16 (18 each), then columns x = -1, 16
    if (r < 18) {
      cx = r - 1;
      cy = -1;
    } else if (r < 36) {
      cx = r - 19;
      cy = 16;
    } else if (r < 52) {
      cx = -1;
      cy = r - 36;
    } else {
      cx = 16;
      cy = r - 52;
    }
  }
  const int hp = (cy + 1) * kH + (cx + 1);  // index in an LDS psi plane
  PullAxes pa;
  pull_axes_xy(cx, cy, pa);
  const int dxy = 13 + sgn_out(cx) + 3 * sgn_out(cy);
  const uint32_t cxy = cell_x(cx & 15) + cell_y(cy & 15);
  const uint32_t plane = P.plane;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  typename S::T* __restrict__ fw = fplane<S>(D, rbuf ^ 1);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;   // references of f(t)
  float* __restrict__ rnew = S::kRef ? D.rho[rbuf ^ 1] : nullptr;     // this step's densities
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  float fp[NC][kQ];   // populations of this column's cell one plane back
  float rp[NC];       // and its densities
  uint32_t mp = 0u;   // and its mask
  bool store_next = false;
  unsigned numeric = 0u, clamps = 0u;
  // Masks are loaded one plane ahead and handed to the next plane through
  // LDS: the load completes while the plane's pulls are waited for, so the
  // pull addresses of a plane never wait for a memory round trip of their
  // own.  Cells outside the active blocks read as solid (no pulls, rest psi).
  // Every thread loads and hands over a mask at every plane (addresses in
  // bounds also past the last plane and in the rest slot), so that no load
  // is pending on one path and not on another.
  auto mask_load = [&](int z) -> uint32_t {
    const int slot = ctx.nslot[dxy + 9 * sgn_out(z)];
    return ld(D.mask, ((uint32_t)slot * P.slot_cells + cxy + 256u * (uint32_t)(z & 15)) * 4u);
  };
  // (threads without a column hand over a mask too, which they never read:
  // the select then needs no branch, and the load is consumed on every path)
  auto in_mesh = [&](int z) { return ctx.nslot[dxy + 9 * sgn_out(z)] != P.capacity; };
  constexpr uint32_t kNoCell = (uint32_t)kSolid << kKindShift;
  {
    const uint32_t raw = mask_load(z0 - 1);
    mask_s[0][t] = in_mesh(z0 - 1) ? raw : kNoCell;
  }
  // references of plane zp: entries t, t + 384, ... of the 400 x NC values
  // (entry e: column e / NC, component e % NC, as they lie in memory)
  constexpr int kRefPer = (NC * kRW * kRW + kFusedThreads - 1) / kFusedThreads;
  auto rref_fetch = [&](int zp, float (&v)[kRefPer]) {
#pragma unroll
    for (int j = 0; j < kRefPer; ++j) {
      const int e = t + j * kFusedThreads;
      v[j] = 0.0f;
      if (e < NC * kRW * kRW) {
        const int aa = e % NC, col = e / NC;
        const int rx = col % kRW - 2, ry = col / kRW - 2;
        const int slot = ctx.nslot[13 + sgn_out(rx) + 3 * sgn_out(ry) + 9 * sgn_out(zp)];
        const uint32_t cell = (uint32_t)slot * P.slot_cells + cell_of(rx & 15, ry & 15, zp & 15);
        v[j] = ld(rref, (cell * NC + (uint32_t)aa) * 4u);
      }
    }
  };
  auto rref_put = [&](int ring, const float (&v)[kRefPer]) {
#pragma unroll
    for (int j = 0; j < kRefPer; ++j) {
      const int e = t + j * kFusedThreads;
      if (e < NC * kRW * kRW) rref_s[ring & 3][e % NC][e / NC] = v[j];
    }
  };
  const int rcol = (cy + 2) * kRW + (cx + 2);  // this column in the reference footprint
  if constexpr (S::kRef) {
    for (int zp = z0 - 2; zp <= z0; ++zp) {
      float v[kRefPer];
      rref_fetch(zp, v);
      rref_put(zp, v);
    }
    __syncthreads();
  }
#pragma unroll 1
  for (int k = 0; k < zlen + 2; ++k) {
    const int z = z0 + k - 1;
    // FP32 store: the wave's pulls and psi run at raised priority, so that
    // its loads go out ahead of the arithmetic of waves in their collision
    // (0.659 -> 0.654 ms per 192^3 full-mesh launch)
    if constexpr (!S::kRef) __builtin_amdgcn_s_setprio(1);
    const bool own = interior && z >= z0 && z < z0 + zlen;
    const uint32_t m = mask_s[k & 1][t];
    const uint32_t m_ahead = mask_load(z + 1);
    float rref_ahead[kRefPer];  // FP16: references of plane z + 2, handed over like the masks
    if constexpr (S::kRef) rref_fetch(min(z + 2, z0 + zlen + 1), rref_ahead);
    // ---- plane z: pull, moments, psi
    float f[NC][kQ];
    float rho[NC];
    if (col) {
      float psi[NC];
      const int slot = ctx.nslot[dxy + 9 * sgn_out(z)];
      const uint32_t cell = (uint32_t)slot * P.slot_cells + cxy + 256u * (uint32_t)(z & 15);
#pragma unroll
      for (int a = 0; a < NC; ++a) psi[a] = P.psi_rest[a];
      if (slot != P.capacity) {
        const uint32_t kind = (m >> kKindShift) & 3u;
        // fluid cells, and (FP16 store) the block's own boundary nodes, whose
        // density is the reference of what they store
        const bool pull = kind == kFluid || (S::kRef && own && kind != kSolid);
        if (pull) {
          Sources<S::kRef> src;
          pull_axes_z(z, pa);
          sources<PULL ? kRdPull : kRdOwn, S::kRef>(pa, cell, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
          // FP16 store: references from the LDS ring, the source cell's, or
          // the cell's own for a bounced link (and on the first step, which
          // does not stream)
          gather_links<S, NC>(fb, plane, src,
                              [&](auto I, float (&r)[NC]) {
                                constexpr int i = decltype(I)::value;
                                const bool self = !PULL || i == 0 || ((m >> i) & 1u);
#pragma unroll
                                for (int a = 0; a < NC; ++a)
                                  r[a] = self ? rref_s[z & 3][a][rcol]
                                              : rref_s[(z - dir_ez(i)) & 3][a][rcol - dir_ex(i) - kRW * dir_ey(i)];
                              },
                              f);
#pragma unroll
          for (int a = 0; a < NC; ++a) rho[a] = moments(f[a]).rho;
        }
        if (kind == kFluid) {
#pragma unroll
          for (int a = 0; a < NC; ++a) {
            bool cl;
            psi[a] = pseudo_potential(P, a, rho[a], cl);
            if (own) {
              clamps += cl ? 1u : 0u;
              if (!(rho[a] > 0.0f && rho[a] < 3.0e38f)) numeric = 1u;
            }
          }
        } else if (kind == kInlet) {
#pragma unroll
          for (int a = 0; a < NC; ++a) psi[a] = P.psi_in[a];
        }
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) psi_s[k % kPsiRing][a][hp] = psi[a];
    }
    mask_s[(k + 1) & 1][t] = in_mesh(z + 1) ? m_ahead : kNoCell;
    // (past the last plane the values land in a slot no later pull reads)
    if constexpr (S::kRef) rref_put(z + 2, rref_ahead);
    if constexpr (!S::kRef) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    // ---- plane z - 1: every cell of the block is stored, so that each
    // written cache line is complete (a partial line costs the memory a
    // read-modify-write).  Fluid cells collide; inlet and outlet nodes impose
    // their state; solid cells take the rest state, which nothing reads.
    if (store_next) {
      const int zc = z - 1;
      const uint32_t cid = own_base + cell_of(cx, cy, zc);
      const uint32_t kind = (mp >> kKindShift) & 3u;
      float rr[NC];  // FP16 reference: the cell's density of this step
      if (kind == kFluid) {
        const int sl[3] = {(k + 2) % kPsiRing, (k + 3) % kPsiRing, k % kPsiRing};  // planes zc-1, zc, zc+1
        float psi_c[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) psi_c[a] = psi_s[sl[1]][a][hp];
        Vec3 F[NC];
        interaction_forces<NC>(P, psi_c,
                               [&](int a, int i) {
                                 const int hn = hp + dir_ex(i) + kH * dir_ey(i);
                                 const bool solid_nb = (mp >> dir_opp(i)) & 1u;  // x + e_i solid or outside
                                 return solid_nb ? psi_c[a] : psi_s[sl[1 + dir_ez(i)]][a][hn];
                               },
                               F);
        // post-collision populations replace the pulled ones (each opposite
        // pair is read before it is written)
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          const Mom mo = moments_with_rho(fp[a], rp[a]);  // rp: the density the pull summed
          rr[a] = rp[a];
          collide_emit(P.omega[a], fp[a], mo, add_body(P, a, F[a], mo.rho),
                       [&](auto I, float v) { fp[a][decltype(I)::value] = v; });
        }
      } else {
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          // FP16 reference: a boundary node's own density of this step
          rr[a] = kind == kSolid ? P.rho_ref_rest[a] : rp[a];
#pragma unroll
          for (int i = 0; i < kQ; ++i) fp[a][i] = kind == kInlet ? f_in_s[a][i] : f_rest_s[a][i];
        }
      }
      // one store per population for the whole wave, fluid and boundary
      // lanes alike, so that each written line is complete in one request
      if constexpr (S::kRef) st_refs<NC>(rnew, cid, rr);
      float rrs[NC];  // the references scaled by the store's 2^12 (exact): w_i rrs = (w_i rr) 2^12
#pragma unroll
      for (int a = 0; a < NC; ++a) rrs[a] = rr[a] * S::kScale;
      unroll<kQ>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int first = i == 0 ? 0 : ((i & 1) ? i : i - 1);
        constexpr bool second = i != 0 && !(i & 1);
        typename S::T enc[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) enc[a] = S::encode_scaled(fp[a][i], dir_w(i) * rrs[a]);
        st_link<true>(fw + (size_t)first * plane * NC, (cid + (second ? plane : 0u)) * (uint32_t)sizeof(enc), enc);
      });
    }
    // ---- keep plane z for its store at the next iteration
    store_next = own;
    if (own) {
      mp = m;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        rp[a] = rho[a];
#pragma unroll
        for (int i = 0; i < kQ; ++i) fp[a][i] = f[a][i];
      }
    }
  }
  if (numeric) atomicOr(&D.ctrl[kNumeric], 1);
  if (clamps) atomicAdd(&D.counters[1], (unsigned long long)clamps);
}

template <typename S, int NC, bool PULL, bool BATCH>
__device__ __forceinline__ void fused_entry(const Params& Pv, const Buffers& Dv, int rbuf, const Batch& Bt,
                                            int parts) {
  // parts workgroups share a block, each sweeping kB / parts of its planes
  // (plus the two halo planes): more workgroups for a small mesh; the parts
  // of a block are adjacent in the XCD mapping, so they share one L2
  int sim = 0, g, part;
  if constexpr (BATCH) {
    const int total = Bt.off[Bt.nsims];
    const int gi = slot_of_workgroup(blockIdx.x, total * parts);
    if (gi >= total * parts) return;
    part = gi % parts;
    sim = batch_sim(Bt, gi / parts);
    g = gi / parts - Bt.off[sim];
  }
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  if constexpr (BATCH) {
    stage_struct(P_s, Bt.P[sim]);
    stage_struct(D_s, Bt.D[sim]);
    __syncthreads();
  }
  const Params& P = BATCH ? P_s : Pv;
  const Buffers& D = BATCH ? D_s : Dv;
  if constexpr (!BATCH) {
    const int n_active = D.ctrl[kNActive];
    const int gi = slot_of_workgroup(blockIdx.x, n_active * parts);
    if (gi >= n_active * parts) return;
    g = gi / parts;
    part = gi % parts;
  }
  fused_block<S, NC, PULL>(P, D, rbuf, g, part, parts);
}

template <typename S, int NC, bool PULL, bool BATCH>
__global__ void __launch_bounds__(kFusedThreads) k_fused(Params Pv, Buffers Dv, int rbuf, Batch Bt, int parts) {
  fused_entry<S, NC, PULL, BATCH>(Pv, Dv, rbuf, Bt, parts);
}

// The step kernel with the FP16 store: left to itself the compiler gives it
// 173 registers per lane (both planes decoded plus the decode temporaries),
// which fits one workgroup per compute unit; bounded to three waves per SIMD
// (168 registers, no spills) two fit, and a launch takes 1.7 % less time.
// The FP32 kernel fits two with 143 registers and keeps the unbounded form
// (the bound would cut its scalar registers and spill them).
template <int NC, bool PULL, bool BATCH>
__global__ void __launch_bounds__(kFusedThreads, 3) k_fused_f16(Params Pv, Buffers Dv, int rbuf, Batch Bt,
                                                                int parts) {
  fused_entry<StoreF16, NC, PULL, BATCH>(Pv, Dv, rbuf, Bt, parts);
}

// The step kernel of a storage format.
template <typename S, int NC, bool PULL, bool BATCH>
constexpr auto fused_kernel() {
  if constexpr (std::is_same<S, StoreF16>::value)
    return &k_fused_f16<NC, PULL, BATCH>;
  else
    return &k_fused<S, NC, PULL, BATCH>;
}

// Persistent form of the batched step kernel: a resident grid whose
// workgroups take (block, part) items from the merged active list of all
// members until none is left.  The list is cut into one contiguous queue per
// XCD (neighbouring blocks share its L2); a workgroup drains the queue of its
// own XCD first, then steals from the others.  The queue heads are counters
// in device memory, reset by the step's closing k_batch_tick; a workgroup
// stops once every queue is empty, so the grid drains without any
// workgroup waiting on another.
__device__ __forceinline__ int take_item(int32_t* heads, int xcd, int total) {
  const int chunk = (total + kXcds - 1) / kXcds;
  for (int j = 0; j < kXcds; ++j) {
    const int q = (xcd + j) % kXcds;
    const int lo = q * chunk, hi = min(total, lo + chunk);
    if (lo >= hi) continue;
    if (atomicAdd(&heads[q], 0) >= hi - lo) continue;  // empty: no increment
    const int v = atomicAdd(&heads[q], 1);
    if (lo + v < hi) return lo + v;
  }
  return -1;
}

template <typename S, int NC, bool PULL>
__global__ void __launch_bounds__(kFusedThreads) k_fused_persistent(Batch Bt, int rbuf, int parts) {
  __shared__ int item_s;
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  const int total = Bt.off[Bt.nsims] * parts;
  const int xcd = blockIdx.x % kXcds;
  for (;;) {
    if (threadIdx.x == 0) item_s = take_item(Bt.heads, xcd, total);
    __syncthreads();
    const int gi = item_s;
    if (gi < 0) break;  // uniform: every queue is empty
    const int sim = batch_sim(Bt, gi / parts);
    stage_struct(P_s, Bt.P[sim]);
    stage_struct(D_s, Bt.D[sim]);
    __syncthreads();
    fused_block<S, NC, PULL>(P_s, D_s, rbuf, gi / parts - Bt.off[sim], gi % parts, parts);
    __syncthreads();  // the next item overwrites item_s, P_s, D_s and the block's LDS
  }
}

// ------------------------------------------------------- in-place step
// The A-A access pattern (section 3): one population buffer, updated in
// place.  A step of even index reads f(t) at each cell's own address and
// writes f* back to the same cell with each opposite pair swapped; a step of
// odd index reads f*_i(x - e_i) at the neighbour's swapped address and writes
// f*_i(x) into the neighbour x + e_i at its natural address, so that after
// every second step the populations are in natural order again.  Each
// address a step reads is written by the thread that read it, after the
// read, so no second buffer is needed; the pseudo-potential of the
// neighbours (Eq 8-9), however, has to be taken before any of them is
// overwritten, so the step runs as two passes: k_inplace_psi stores psi of
// every cell of the active blocks, k_inplace_collide takes the forces from
// it, collides and streams.  The arithmetic of each cell is that of k_fused,
// in the same order, so both patterns give the same bits.  With the
// FP16-deviation store a value decodes with the density of the cell that
// wrote it, which is the link's source in both parities (the cell itself for
// a bounced link); those densities stay double-buffered by step parity.
//
// Progressive mesh: a link from a cell of an inactive block carries the rest
// state.  At a step of odd index a population streamed towards a block that
// is inactive stays at the sender's own swapped address (nothing else writes
// there), which the next step reads as the rest state (kRdAAEven: the link's
// source is inactive).  If that block joins the next step, its
// initialisation moves the value to the receiving cell and leaves the rest
// state in its place (kInitStash).

constexpr int kInplaceThreads = 256;

// The block of this workgroup: (simulation, position g in its active list in
// block order); false for workgroups past the end of the list.
template <bool BATCH>
__device__ __forceinline__ bool workgroup_block(const Buffers& Dv, const Batch& Bt, int& sim, int& g) {
  sim = 0;
  if constexpr (BATCH) {
    const int total = Bt.off[Bt.nsims];
    const int gi = slot_of_workgroup(blockIdx.x, total);
    if (gi >= total) return false;
    sim = batch_sim(Bt, gi);
    g = gi - Bt.off[sim];
  } else {
    const int n_active = Dv.ctrl[kNActive];
    g = slot_of_workgroup(blockIdx.x, n_active);
    if (g >= n_active) return false;
  }
  return true;
}

// Pass 1: psi (Eq 6-7) of every cell of the active blocks (fluid cells from
// their densities, inlet nodes psi(inlet density), outlet and solid cells the
// rest value) into D.psi.
template <typename S, int NC, int RD, bool BATCH>
__global__ void __launch_bounds__(kThreads) k_inplace_psi(Params Pv, Buffers Dv, int rbuf, Batch Bt) {
  int sim, g;
  if (!workgroup_block<BATCH>(Dv, Bt, sim, g)) return;
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  if constexpr (BATCH) {
    stage_struct(P_s, Bt.P[sim]);
    stage_struct(D_s, Bt.D[sim]);
    __syncthreads();
  }
  const Params& P = BATCH ? P_s : Pv;
  const Buffers& D = BATCH ? D_s : Dv;
  const int s = D.order[g];
  __shared__ BlockCtx ctx;
  setup_block(P, D, D.slot_block[s], ctx);
  __syncthreads();
  int x, y, z0;
  cell_xyz((int)threadIdx.x, x, y, z0);
  PullAxes pa;
  pull_axes_xy(x, y, pa);
  const uint32_t plane = P.plane;
  const typename S::T* __restrict__ fb = fplane<S>(D, 0);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;  // references of f(t)
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  unsigned numeric = 0u, clamps = 0u;
#pragma unroll 1
  for (int z = z0; z < kB; z += kZStep) {
    const uint32_t cid = own_base + cell_of(x, y, z);
    const uint32_t m = ld(D.mask, cid * 4u);
    const uint32_t kind = (m >> kKindShift) & 3u;
    float psi[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) psi[a] = kind == kInlet ? P.psi_in[a] : P.psi_rest[a];
    if (kind == kFluid) {
      Sources<S::kRef> src;
      pull_axes_z(z, pa);
      sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
      float f[NC][kQ];
      gather_links<S, NC>(fb, plane, src,
                          [&](auto I, float (&r)[NC]) { ld_refs<NC>(rref, src.ridx[decltype(I)::value], r); }, f);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const float rho = moments(f[a]).rho;
        bool cl;
        psi[a] = pseudo_potential(P, a, rho, cl);
        clamps += cl ? 1u : 0u;
        if (!(rho > 0.0f && rho < 3.0e38f)) numeric = 1u;
      }
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) st(D.psi + (size_t)a * plane, cid * 4u, psi[a]);
  }
  if (numeric) atomicOr(&D.ctrl[kNumeric], 1);
  if (clamps) atomicAdd(&D.counters[1], (unsigned long long)clamps);
}

// Pass 2: forces (Eq 8-9, psi of an 18 x 18 footprint in an LDS ring of four
// planes), collision (Eq 10-12) and in-place streaming.  One workgroup per
// active block; thread t owns column t of the block and sweeps z = 0 .. 15.
// Inlet and outlet nodes stream their imposed state and solid cells write the
// rest state to their own address, which nothing reads.
template <typename S, int NC, int RD, bool BATCH>
__global__ void __launch_bounds__(kInplaceThreads) k_inplace_collide(Params Pv, Buffers Dv, int rbuf, Batch Bt) {
  static_assert(RD != kRdPull, "the in-place step reads in place");
  constexpr bool kOdd = RD == kRdAAOdd;
  int sim, g;
  if (!workgroup_block<BATCH>(Dv, Bt, sim, g)) return;
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  if constexpr (BATCH) {
    stage_struct(P_s, Bt.P[sim]);
    stage_struct(D_s, Bt.D[sim]);
    __syncthreads();
  }
  const Params& P = BATCH ? P_s : Pv;
  const Buffers& D = BATCH ? D_s : Dv;
  const int s = D.order[g];
  __shared__ BlockCtx ctx;
  __shared__ float psi_s[kPsiRing][NC][kFoot];
  __shared__ float f_in_s[NC][kQ], f_rest_s[NC][kQ];
  setup_block(P, D, D.slot_block[s], ctx);
  if (threadIdx.x >= 64 && threadIdx.x < 64 + NC * kQ) {
    const int k = threadIdx.x - 64, a = k / kQ, i = k % kQ;
    f_in_s[a][i] = P.f_in[a][i];
    f_rest_s[a][i] = P.f_rest[a][i];
  }
  __syncthreads();
  const int t = threadIdx.x;
  int cx, cy, cz0;
  cell_xyz(t, cx, cy, cz0);
  const int hp = (cy + 1) * kH + (cx + 1);
  const uint32_t plane = P.plane;
  using T = typename S::T;
  T* __restrict__ fb = fplane<S>(D, 0);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;  // references of f(t)
  float* __restrict__ rnew = S::kRef ? D.rho[rbuf ^ 1] : nullptr;    // this step's densities
  const float* __restrict__ psi_g = D.psi;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  // FP16 store: the references of f(t) over the same footprint (a link's
  // value decodes with its source cell's), in a ring of their own
  __shared__ float rref_s[S::kRef ? kPsiRing : 1][NC][S::kRef ? kFoot : 1];
  // psi (and references) of footprint plane zp (x, y in [-1, 16]) into ring
  // slot zp & 3; inactive neighbours read the rest slot, which holds psi_rest
  // and the rest state's reference
  auto psi_load = [&](int zp) {
    for (int e = t; e < NC * kFoot; e += kInplaceThreads) {
      const int a = e / kFoot, col = e % kFoot;
      const int hx = col % kH - 1, hy = col / kH - 1;
      const int slot = ctx.nslot[13 + sgn_out(hx) + 3 * sgn_out(hy) + 9 * sgn_out(zp)];
      const uint32_t off = ((uint32_t)slot * P.slot_cells + cell_of(hx & 15, hy & 15, zp & 15)) * 4u;
      psi_s[zp & 3][a][col] = ld(psi_g + (size_t)a * plane, off);
      if constexpr (S::kRef) rref_s[zp & 3][a][col] = ld(rref, off * NC + (uint32_t)(4 * a));
    }
  };
  psi_load(-1);
  psi_load(0);
  PullAxes pa;
  pull_axes_xy(cx, cy, pa);
#pragma unroll 1
  for (int z = 0; z < kB; ++z) {
    // (ring slot (z + 1) & 3 was last read two planes ago, before the
    // previous barrier)
    psi_load(z + 1);
    __syncthreads();
    const uint32_t cid = own_base + cell_of(cx, cy, z);
    const uint32_t m = ld(D.mask, cid * 4u);
    const uint32_t kind = (m >> kKindShift) & 3u;
    pull_axes_z(z, pa);
    float fp[NC][kQ];
    float rr[NC];  // FP16 store: the reference of what the cell writes, its density of this step
#pragma unroll
    for (int a = 0; a < NC; ++a) rr[a] = P.rho_ref_rest[a];
    // fluid cells, and (FP16 store) boundary nodes, whose density is the
    // reference of what they write
    if (kind == kFluid || (S::kRef && kind != kSolid)) {
      Sources<S::kRef> src;
      sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
      // FP16 store: the source cell's reference, or the cell's own for a
      // bounced link (and on the first step, which reads in place)
      gather_links<S, NC>(fb, plane, src,
                          [&](auto I, float (&r)[NC]) {
                            constexpr int i = decltype(I)::value;
                            const bool self = RD == kRdOwn || i == 0 || ((m >> i) & 1u);
#pragma unroll
                            for (int a = 0; a < NC; ++a)
                              r[a] = self ? rref_s[z & 3][a][hp]
                                          : rref_s[(z - dir_ez(i)) & 3][a][hp - dir_ex(i) - kH * dir_ey(i)];
                          },
                          fp);
#pragma unroll
      for (int a = 0; a < NC; ++a) rr[a] = moments(fp[a]).rho;
    }
    if (kind == kFluid) {
      float psi_c[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) psi_c[a] = psi_s[z & 3][a][hp];
      Vec3 F[NC];
      interaction_forces<NC>(P, psi_c,
                             [&](int a, int i) {
                               const int hn = hp + dir_ex(i) + kH * dir_ey(i);
                               const bool solid_nb = (m >> dir_opp(i)) & 1u;  // x + e_i solid or outside
                               return solid_nb ? psi_c[a] : psi_s[(z + dir_ez(i)) & 3][a][hn];
                             },
                             F);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const Mom mo = moments_with_rho(fp[a], rr[a]);  // rr: the density summed after the pull
        collide_emit(P.omega[a], fp[a], mo, add_body(P, a, F[a], mo.rho),
                     [&](auto I, float v) { fp[a][decltype(I)::value] = v; });
      }
    } else {
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int i = 0; i < kQ; ++i) fp[a][i] = kind == kInlet ? f_in_s[a][i] : f_rest_s[a][i];
    }
    // destination of f*_i: even index, the cell's own swapped address; odd
    // index, x + e_i at its natural address, or the own swapped address when
    // x + e_i is solid, outside or in an inactive block, or x is solid
    uint32_t dst[kQ];
    dst[0] = cid;
    unroll<kQ - 1>([&](auto K) {
      constexpr int i = decltype(K)::value + 1;
      constexpr bool second = !(i & 1);
      const uint32_t own_o = second ? cid : cid + plane;
      if constexpr (!kOdd) {
        dst[i] = own_o;
      } else {
        const uint32_t w = pa.ax[1 + dir_ex(i)] + pa.ay[1 + dir_ey(i)] + pa.az[1 + dir_ez(i)];  // x + e_i
        const int tslot = ctx.nslot[w >> 16];
        const bool keep = kind == kSolid || ((m >> dir_opp(i)) & 1u) || tslot == P.capacity;
        const uint32_t tcell = (uint32_t)tslot * P.slot_cells + (w & 0xFFFFu);
        dst[i] = keep ? own_o : (second ? tcell + plane : tcell);
      }
    });
    // even index: every line is written whole by one store of the wave,
    // non-temporal; odd index: the shifted stores write parts of lines that
    // other waves complete, which the L2 merges while it holds them
    if constexpr (S::kRef) st_refs<NC>(rnew, cid, rr);
    float rrs[NC];  // the references scaled by the store's 2^12 (exact): w_i rrs = (w_i rr) 2^12
#pragma unroll
    for (int a = 0; a < NC; ++a) rrs[a] = rr[a] * S::kScale;
    unroll<kQ>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int first = i == 0 ? 0 : ((i & 1) ? i : i - 1);
      T enc[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) enc[a] = S::encode_scaled(fp[a][i], dir_w(i) * rrs[a]);
      st_link<!kOdd>(fb + (size_t)first * plane * NC, dst[i] * (uint32_t)sizeof(enc), enc);
    });
  }
}

// ------------------------------------------------------------- criterion
// Eq 13 on frontier blocks only (section 4.2): a fluid cell within `shell`
// cells of an inactive neighbour block that holds fluid, whose velocity
// differs from the previous step's for any component, requests that block.
// Only the shell cells of frontier blocks are read, so once the mesh covers
// the domain this kernel does no work.
//
// The same pass checks that the progressive mesh hides nothing (the leak
// counter).  For a link from an active cell x into a non-solid cell of an
// inactive block N:
//  - kCritEmission: the populations the previous step stored at x for the
//    link (and, for the FP16 store, their reference density) must have the
//    rest state's bits if N is still inactive now: N's cells would have
//    pulled them this step;
//  - kCritExposure: psi(x) of this step must be the rest value if N is still
//    inactive when this step's forces are taken.
// Both depend on this step's activation, so the failing links are counted
// per target block in D.expose and settled by k_activate.
// The shell cells of a block are first compacted into an LDS list (in any
// order: every result is a per-cell store, an integer atomic or a bit OR), so
// that all threads work on them together.
template <typename S, int NC, int RD, bool BATCH>
__global__ void __launch_bounds__(kThreads) k_criterion(Params Pv, Buffers Dv, int rbuf, int flags, Batch Bt) {
  int sim = 0, s;
  if constexpr (BATCH) {
    const int total = Bt.off[Bt.nsims];
    const int gi = slot_of_workgroup(blockIdx.x, total);
    if (gi >= total) return;
    sim = batch_sim(Bt, gi);
    s = gi - Bt.off[sim];
  }
  __shared__ Params P_s;
  __shared__ Buffers D_s;
  if constexpr (BATCH) {
    stage_struct(P_s, Bt.P[sim]);
    stage_struct(D_s, Bt.D[sim]);
    __syncthreads();
  }
  const Params& P = BATCH ? P_s : Pv;
  const Buffers& D = BATCH ? D_s : Dv;
  bool live = true;
  if constexpr (!BATCH) {
    // workgroup g takes slot g, so that the active count, the block id and
    // the frontier flag are loaded together (through the active count, as
    // the step kernel maps them, the criterion took 1.35x as long); the grid
    // may exceed the pool, hence the clamp
    s = min((int)blockIdx.x, P.capacity - 1);
    live = (int)blockIdx.x < D.ctrl[kNActive];
  }
  const int blk = D.slot_block[s];
  const int front = D.frontier[s];
  // a block none of whose neighbours is an inactive block holding fluid
  // stays so (blocks are never deactivated): such slots skip the pass
  if (!live || !front) return;  // uniform
  __shared__ BlockCtx ctx;
  __shared__ int expo[27];
  __shared__ uint16_t list[kCells];
  __shared__ int count;
  setup_block(P, D, blk, ctx);
  if (threadIdx.x < 27) expo[threadIdx.x] = 0;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  const unsigned cand = ctx.cand;
  if (!cand) {  // uniform
    if (threadIdx.x == 0) D.frontier[s] = 0;
    return;
  }
  for (int c = threadIdx.x; c < kCells; c += kThreads) {
    int cxx, cyy, czz;
    cell_xyz(c, cxx, cyy, czz);
    const bool in_shell = (shell_dirs(cxx, cyy, czz, P.shell) & cand) != 0u;
    const unsigned long long bal = __ballot(in_shell);
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(&count, __popcll(bal));
    base = __shfl(base, 0);
    if (in_shell) list[base + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)c;
  }
  __syncthreads();
  const int n_shell = count;
  const uint32_t plane = P.plane;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  const bool pull_cells = (flags & (kCritRecord | kCritEval | kCritExposure)) != 0;
  unsigned fired = 0u;
  // each cell's mask is loaded one iteration ahead, so that an iteration
  // waits for one round trip (its pulls), not two (the mask, then the pulls
  // whose addresses depend on it)
  uint32_t m_next = 0u;
  if ((int)threadIdx.x < n_shell) m_next = ld(D.mask, (own_base + (uint32_t)list[threadIdx.x]) * 4u);
#pragma unroll 1
  for (int j = threadIdx.x; j < n_shell; j += kThreads) {
    const int c = list[j];
    int x, y, z;
    cell_xyz(c, x, y, z);
    const unsigned dirs = shell_dirs(x, y, z, P.shell) & cand;
    const uint32_t cid = own_base + (uint32_t)c;
    const uint32_t m = m_next;
    if (j + kThreads < n_shell) m_next = ld(D.mask, (own_base + (uint32_t)list[j + kThreads]) * 4u);
    const uint32_t kind = (m >> kKindShift) & 3u;
    if (kind == kSolid) continue;
    // the previous velocities, loaded before the pulls so that both are in
    // flight together
    float u_old[NC][3];
    if (flags & kCritEval) {
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) u_old[a][d] = D.uprev[(size_t)(a * 3 + d) * plane + cid];
    }
    // links x -> x + e_i into a non-solid cell of a candidate block
    uint32_t out_links = 0u;
    unroll<kQ - 1>([&](auto I) {
      constexpr int i = decltype(I)::value + 1;
      const int d = 13 + sgn_out(x + dir_ex(i)) + 3 * sgn_out(y + dir_ey(i)) + 9 * sgn_out(z + dir_ez(i));
      const bool target_solid = (m >> dir_opp(i)) & 1u;  // x + e_i solid or outside
      if (d != 13 && ((cand >> d) & 1u) && !target_solid) out_links |= 1u << i;
    });
    // every load of the cell is issued before any is used: the pulled
    // populations, then (for the leak check) the populations this cell
    // stored last step, all of its 18 links, so that no load waits behind
    // a branch of its own
    float f[NC][kQ];
    if (pull_cells) {
      PullAxes pa;
      pull_axes_xy(x, y, pa);
      pull_axes_z(z, pa);
      Sources<S::kRef> src;
      sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
      gather_links<S, NC>(fb, plane, src,
                          [&](auto I, float (&r)[NC]) { ld_refs<NC>(rref, src.ridx[decltype(I)::value], r); }, f);
    }
    uint32_t bad = 0u;  // failing links
    if ((flags & kCritEmission) && out_links) {
      uint32_t em[NC][kQ] = {};
      unroll<kQ - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        constexpr int first = (i & 1) ? i : i - 1;
        // f*_i(x) is stored at (x, plane i), or with the in-place pattern
        // at (x, opposite plane) after either parity of step.  FP32 store:
        // only the links into a candidate block are loaded (five of the
        // eighteen for a cell on a face; 8 % less time at 384^3).  FP16
        // store: all eighteen (the same choice took 12 % more time there)
        constexpr bool upper = (RD == kRdAAEven || RD == kRdAAOdd) ? (i & 1) : !(i & 1);
        if (S::kRef || ((out_links >> i) & 1u)) {
          typename S::T v[NC];
          ld_link<typename S::T, NC>(fb + (size_t)first * plane * NC, (cid + (upper ? plane : 0u)) * (uint32_t)sizeof(v),
                                     v);
#pragma unroll
          for (int a = 0; a < NC; ++a) em[a][i] = S::bits(v[a]);
        }
      });
      if constexpr (S::kRef) {
        float r[NC];
        ld_refs<NC>(rref, cid, r);
#pragma unroll
        for (int a = 0; a < NC; ++a) em[a][0] = __float_as_uint(r[a]);
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        unroll<kQ - 1>([&](auto I) {
          constexpr int i = decltype(I)::value + 1;
          if (((out_links >> i) & 1u) && em[a][i] != P.f_rest_bits[a][i]) bad |= 1u << i;
        });
        if constexpr (S::kRef) {
          if (em[a][0] != __float_as_uint(P.rho_ref_rest[a])) bad = out_links;
        }
      }
    }
    if (pull_cells) {
      bool changed = false, psi_differs = false;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const Mom mo = moments(f[a]);
        float psi = P.psi_rest[a];
        if (kind == kFluid) {
          bool cl;
          psi = pseudo_potential(P, a, mo.rho, cl);
        } else if (kind == kInlet) {
          psi = P.psi_in[a];
        }
        psi_differs = psi_differs || (psi != P.psi_rest[a]);
        if (flags & (kCritRecord | kCritEval)) {
          float inv = 0.0f;
          if (mo.rho > 0.0f) inv = 1.0f / mo.rho;
          const float u[3] = {mo.jx * inv, mo.jy * inv, mo.jz * inv};
          float* up = D.uprev + (size_t)(a * 3) * plane + cid;
          if (flags & kCritEval) {
            float d2 = 0.0f;
            bool diff = false;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float dd = u[d] - u_old[a][d];
              diff = diff || (dd != 0.0f);
              d2 = d2 + dd * dd;
            }
            changed = changed || (P.s_zero ? diff : (sqrtf(d2) > P.S));
          }
          if (flags & kCritRecord)
            for (int d = 0; d < 3; ++d) up[(size_t)d * plane] = u[d];
        }
      }
      if (changed) fired |= dirs;
      if ((flags & kCritExposure) && psi_differs) bad = out_links;
    }
    if (bad) {
      unroll<kQ - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        if ((bad >> i) & 1u) {
          const int d = 13 + sgn_out(x + dir_ex(i)) + 3 * sgn_out(y + dir_ey(i)) + 9 * sgn_out(z + dir_ez(i));
          atomicAdd(&expo[d], 1);
        }
      });
    }
  }
  if (fired) atomicOr(&ctx.fired, fired);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 27) {
    if ((ctx.fired >> t) & 1u) D.request[ctx.nbk[t]] = 1;
    if (expo[t]) atomicAdd(&D.expose[ctx.nbk[t]], expo[t]);
    if (((ctx.fired >> t) & 1u) || expo[t]) D.ctrl[kPending] = 1;
  }
}

// -------------------------------------------------------------- proposal
// The learned activation proposal.  k_candidates lists, in block order, the
// inactive blocks holding fluid that have an active neighbour (one
// workgroup, wave ballot + scan as in k_activate).
__global__ void __launch_bounds__(1024) k_candidates(Params P, Buffers D) {
  __shared__ int wave_count[16];
  __shared__ int wave_base[16];
  __shared__ int chunk_total;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int base = 0;
  for (int b0 = 0; b0 < P.nb; b0 += 1024) {
    const int b = b0 + t;
    int flag = 0;
    if (b < P.nb && D.block_slot[b] < 0 && D.bfluid[b]) {
      const int bx = b % P.nbx, by = (b / P.nbx) % P.nby, bz = b / (P.nbx * P.nby);
      for (int d = 0; d < 27 && !flag; ++d) {
        if (d == 13) continue;
        const int nb = neighbour_block(P, bx, by, bz, d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1);
        if (nb >= 0 && D.block_slot[nb] >= 0) flag = 1;
      }
    }
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
    }
    __syncthreads();
    if (flag) D.cand[base + wave_base[wave] + lane_rank] = b;
    base += chunk_total;
    __syncthreads();
  }
  if (t == 0) D.ctrl[kCandCount] = base;
}

// One workgroup per candidate N.  For every active neighbour B of N it
// visits the cells of B within `shell` cells of N (a slab of B), pulls them
// as the criterion does and adds up rho_a, |u_a| and |psi_a - psi_rest,a|;
// the sums are reduced over the threads in a fixed order.  Features (in this
// order): the six means, the steps since a neighbour of N was activated,
// N's fluid fraction, N's number of active neighbours, and the mean over the
// active neighbours of the unit vector from B to N.  With mlp set the
// workgroup then evaluates the network (the same arithmetic as
// lbm_mlp_forward) and requests N when sigma(z) > thr.
constexpr int kFeat = 12;
constexpr int kPropThreads = 256;

template <typename S, int NC, int RD>
__global__ void __launch_bounds__(kPropThreads) k_propose(Params P, Buffers D, int rbuf, int step,
                                                          const float* __restrict__ mlp, float thr,
                                                          float* __restrict__ feat_out,
                                                          int32_t* __restrict__ block_out, int cap) {
  const int ci = blockIdx.x;
  if (ci >= D.ctrl[kCandCount]) return;
  const int N = D.cand[ci];
  const int t = threadIdx.x;
  __shared__ int slot5[125];     // slots of N's neighbourhood, offsets -2..2 (-1: inactive or outside)
  __shared__ int nslotB[27];     // the 27 neighbour slots of the block being visited
  __shared__ float red[8][kPropThreads];
  __shared__ float fe[kFeat];
  __shared__ float h1s[64];
  __shared__ float h2s[64];
  const int bx = N % P.nbx, by = (N / P.nbx) % P.nby, bz = N / (P.nbx * P.nby);
  if (t < 125) {
    const int nb = neighbour_block(P, bx, by, bz, t % 5 - 2, (t / 5) % 5 - 2, t / 25 - 2);
    slot5[t] = nb < 0 ? -1 : D.block_slot[nb];
  }
  __syncthreads();
  const uint32_t plane = P.plane;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
  const int w = P.shell;
  float acc[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q] = 0.0f;
  int n_act = 0, last_act = -1;
  float dirx = 0.0f, diry = 0.0f, dirz = 0.0f;
#pragma unroll 1
  for (int d = 0; d < 27; ++d) {
    const int ox = d % 3 - 1, oy = (d / 3) % 3 - 1, oz = d / 9 - 1;  // offset of B from N
    if (d == 13) continue;
    const int sB = slot5[(ox + 2) + 5 * ((oy + 2) + 5 * (oz + 2))];
    if (sB < 0) continue;  // uniform
    {
      const int nbid = neighbour_block(P, bx, by, bz, ox, oy, oz);
      n_act += 1;
      last_act = max(last_act, D.act_step[nbid]);
      const float inv = 1.0f / sqrtf((float)(ox * ox + oy * oy + oz * oz));
      dirx = dirx - ox * inv;
      diry = diry - oy * inv;
      dirz = dirz - oz * inv;
    }
    __syncthreads();  // nslotB of the previous neighbour no longer in use
    if (t < 27) {
      const int ex = t % 3 - 1, ey = (t / 3) % 3 - 1, ez = t / 9 - 1;
      const int sl = slot5[(ox + ex + 2) + 5 * ((oy + ey + 2) + 5 * (oz + ez + 2))];
      nslotB[t] = sl < 0 ? P.capacity : sl;
    }
    __syncthreads();
    // the slab of B within w cells of N
    const int x0 = ox > 0 ? 0 : (ox < 0 ? kB - w : 0), lx = ox != 0 ? w : kB;
    const int y0 = oy > 0 ? 0 : (oy < 0 ? kB - w : 0), ly = oy != 0 ? w : kB;
    const int z0 = oz > 0 ? 0 : (oz < 0 ? kB - w : 0), lz = oz != 0 ? w : kB;
    const int total = lx * ly * lz;
#pragma unroll 1
    for (int c = t; c < total; c += kPropThreads) {
      const int x = x0 + c % lx, y = y0 + (c / lx) % ly, z = z0 + c / (lx * ly);
      const uint32_t cid = (uint32_t)sB * P.slot_cells + cell_of(x, y, z);
      const uint32_t m = ld(D.mask, cid * 4u);
      const uint32_t kind = (m >> kKindShift) & 3u;
      if (kind == kSolid) continue;
      PullAxes pa;
      pull_axes_xy(x, y, pa);
      pull_axes_z(z, pa);
      Sources<S::kRef> src;
      sources<RD, S::kRef>(pa, cid, m, plane, nslotB, P.capacity, P.slot_cells, src);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        float f[kQ];
        gather<S, NC>(fb, plane, a, src, rref, f);
        const Mom mo = moments(f);
        float inv = 0.0f;
        if (mo.rho > 0.0f) inv = 1.0f / mo.rho;
        const float ux = mo.jx * inv, uy = mo.jy * inv, uz = mo.jz * inv;
        float psi = P.psi_rest[a];
        if (kind == kFluid) {
          bool cl;
          psi = pseudo_potential(P, a, mo.rho, cl);
        } else if (kind == kInlet) {
          psi = P.psi_in[a];
        }
        acc[a] = acc[a] + mo.rho;
        acc[2 + a] = acc[2 + a] + sqrtf((ux * ux + uy * uy) + uz * uz);
        acc[4 + a] = acc[4 + a] + fabsf(psi - P.psi_rest[a]);
      }
      acc[6] = acc[6] + 1.0f;
    }
  }
  // fixed-order reduction over the threads
#pragma unroll
  for (int q = 0; q < 7; ++q) red[q][t] = acc[q];
  __syncthreads();
  for (int h = kPropThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int q = 0; q < 7; ++q) red[q][t] = red[q][t] + red[q][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const float cnt = red[6][0];
    const float icnt = cnt > 0.0f ? 1.0f / cnt : 0.0f;
    for (int q = 0; q < 6; ++q) fe[q] = red[q][0] * icnt;
    fe[6] = (float)(step - last_act);
    fe[7] = D.bfrac[N];
    fe[8] = (float)n_act;
    const float ia = n_act > 0 ? 1.0f / (float)n_act : 0.0f;
    fe[9] = dirx * ia;
    fe[10] = diry * ia;
    fe[11] = dirz * ia;
    if (!mlp && ci < cap) {
      for (int q = 0; q < kFeat; ++q) feat_out[(size_t)ci * kFeat + q] = fe[q];
      block_out[ci] = N;
    }
  }
  if (!mlp) return;  // uniform
  __syncthreads();
  // the network, with the arithmetic of lbm_mlp_forward
  constexpr int kW1 = 2 * kFeat, kB1 = kW1 + 64 * kFeat, kW2 = kB1 + 64, kB2 = kW2 + 64 * 64, kW3 = kB2 + 64,
                kB3 = kW3 + 64;
  if (t < 64) {
    float xn[kFeat];
#pragma unroll
    for (int i = 0; i < kFeat; ++i) xn[i] = (fe[i] - mlp[i]) * mlp[kFeat + i];
    float a1 = mlp[kB1 + t];
#pragma unroll
    for (int i = 0; i < kFeat; ++i) a1 = a1 + mlp[kW1 + t * kFeat + i] * xn[i];
    h1s[t] = a1 > 0.0f ? a1 : 0.0f;
  }
  __syncthreads();
  if (t < 64) {
    float a2 = mlp[kB2 + t];
    for (int k = 0; k < 64; ++k) a2 = a2 + mlp[kW2 + t * 64 + k] * h1s[k];
    h2s[t] = a2 > 0.0f ? a2 : 0.0f;
  }
  __syncthreads();
  if (t == 0) {
    float z = mlp[kB3];
    for (int j = 0; j < 64; ++j) z = z + mlp[kW3 + j] * h2s[j];
    const float p = 1.0f / (1.0f + expf(-z));
    if (p > thr) {
      D.request[N] = 1;
      D.ctrl[kPending] = 1;
    }
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

// Per lattice cell: 1 if its block is active.
__global__ void k_active_cells(Params P, Buffers D, uint8_t* out) {
  const long long N = (long long)P.nx * P.ny * P.nz;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    out[n] = D.block_slot[x / kB + P.nbx * (y / kB + P.nby * (z / kB))] >= 0 ? 1 : 0;
  }
}

// ---------------------------------------------------------------- repack
// Once every block holding fluid is active, the slots are put in block order:
// slot j takes the block of D.order[j], the j-th active slot in block order.
// The progressive mesh then lays its blocks out as the static mesh does
// (neighbours along x in adjacent slots), and its steps run as fast.  Each
// slot-indexed plane is gathered into a scratch region and copied back, one
// plane at a time; the slot tables follow last.  Only slots below n_active
// move (the rest slot stays where it is).
//   slot_vec: 16-byte words per slot in the plane; gather: read slot order[j]
//   (else slot j) into slot j.
__global__ void k_repack_plane(const uint4* __restrict__ src, uint4* __restrict__ dst,
                               const int32_t* __restrict__ order, const int32_t* __restrict__ ctrl,
                               uint32_t slot_vec, int gather) {
  const long long total = (long long)ctrl[kNActive] * slot_vec;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e / slot_vec);
    const uint32_t w = (uint32_t)(e % slot_vec);
    const int from = gather ? order[j] : j;
    dst[(size_t)j * slot_vec + w] = src[(size_t)from * slot_vec + w];
  }
}

// Slot tables: tmp[j] = block of slot order[j], tmp[cap + j] = its frontier flag.
__global__ void k_repack_tables_gather(Buffers D, int32_t* tmp, int cap) {
  const int n = D.ctrl[kNActive];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int from = D.order[j];
    tmp[j] = D.slot_block[from];
    tmp[cap + j] = D.frontier[from];
  }
}
__global__ void k_repack_tables_apply(Buffers D, const int32_t* tmp, int cap) {
  const int n = D.ctrl[kNActive];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int b = tmp[j];
    D.slot_block[j] = b;
    D.frontier[j] = tmp[cap + j];
    D.block_slot[b] = j;
    D.order[j] = j;
  }
}

// Moments (Eq 4-5) of the active blocks into lattice-wide arrays.
template <typename S, int NC, int RD>
__global__ void __launch_bounds__(kThreads) k_export(Params P, Buffers D, int rbuf, float* rho, float* u,
                                                      float* umix) {
  const int n_active = D.ctrl[kNActive];
  const int s = slot_of_workgroup(blockIdx.x, n_active);
  if (s >= n_active) return;
  __shared__ BlockCtx ctx;
  const int blk = D.slot_block[s];
  setup_block(P, D, blk, ctx);
  __syncthreads();
  int x, y, z0;
  cell_xyz((int)threadIdx.x, x, y, z0);
  PullAxes pa;
  pull_axes_xy(x, y, pa);
  const int bx = blk % P.nbx, by = (blk / P.nbx) % P.nby, bz = blk / (P.nbx * P.nby);
  const long long N = (long long)P.nx * P.ny * P.nz;
  const uint32_t plane = P.plane;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
#pragma unroll 1
  for (int z = z0; z < kB; z += kZStep) {
    const uint32_t cid = own_base + cell_of(x, y, z);
    const uint32_t m = D.mask[cid];
    const bool sol = ((m >> kKindShift) & 3u) == kSolid;
    const int X = bx * kB + x, Y = by * kB + y, Z = bz * kB + z;
    if (X >= P.nx || Y >= P.ny || Z >= P.nz) continue;  // padding: not part of the lattice
    const long long n = X + (long long)P.nx * (Y + (long long)P.ny * (long long)Z);
    float mr = 0.0f, mx = 0.0f, my = 0.0f, mz = 0.0f;
    Sources<S::kRef> src;
    pull_axes_z(z, pa);
    sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      Mom mo = {0.0f, 0.0f, 0.0f, 0.0f};
      if (!sol) {
        float f[kQ];
        gather<S, NC>(fb, plane, a, src, rref, f);
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

// Sum of rho_a over the fluid cells of the active blocks, FP64; out[2]
// counts those cells.
template <typename S, int NC, int RD>
__global__ void __launch_bounds__(kThreads) k_mass(Params P, Buffers D, int rbuf, double* out) {
  const int n_active = D.ctrl[kNActive];
  const int s = slot_of_workgroup(blockIdx.x, n_active);
  if (s >= n_active) return;
  __shared__ BlockCtx ctx;
  __shared__ double red[kMaxComp][kThreads];
  __shared__ int cnt[kThreads];
  setup_block(P, D, D.slot_block[s], ctx);
  __syncthreads();
  int x, y, z0;
  cell_xyz((int)threadIdx.x, x, y, z0);
  PullAxes pa;
  pull_axes_xy(x, y, pa);
  const uint32_t plane = P.plane;
  const uint32_t own_base = (uint32_t)s * P.slot_cells;
  const typename S::T* __restrict__ fb = fplane<S>(D, rbuf);
  const float* __restrict__ rref = S::kRef ? D.rho[rbuf] : nullptr;
  double acc[kMaxComp] = {0.0, 0.0};
  int nf = 0;
#pragma unroll 1
  for (int z = z0; z < kB; z += kZStep) {
    const uint32_t cid = own_base + cell_of(x, y, z);
    const uint32_t m = D.mask[cid];
    if (((m >> kKindShift) & 3u) == kSolid) continue;
    ++nf;
    Sources<S::kRef> src;
    pull_axes_z(z, pa);
    sources<RD, S::kRef>(pa, cid, m, plane, ctx.nslot, P.capacity, P.slot_cells, src);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      float f[kQ];
      gather<S, NC>(fb, plane, a, src, rref, f);
      acc[a] += (double)moments(f).rho;
    }
  }
  for (int a = 0; a < kMaxComp; ++a) red[a][threadIdx.x] = acc[a];
  cnt[threadIdx.x] = nf;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int a = 0; a < kMaxComp; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
      cnt[threadIdx.x] += cnt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int a = 0; a < NC; ++a) atomicAdd(&out[a], red[a][0]);
    atomicAdd(&out[2], (double)cnt[0]);
  }
}

// Calls fn with the read mode rd as a compile-time constant (the in-place
// modes exist for the FP32 store only).
template <typename S, typename Fn>
hipError_t with_rd(int rd, Fn&& fn) {
  if (rd == kRdOwn) return fn(std::integral_constant<int, kRdOwn>{});
  if (rd == kRdPull) return fn(std::integral_constant<int, kRdPull>{});
  if (rd == kRdAAEven) return fn(std::integral_constant<int, kRdAAEven>{});
  if (rd == kRdAAOdd) return fn(std::integral_constant<int, kRdAAOdd>{});
  return hipErrorInvalidValue;
}

// Dispatch on storage format and component count.
template <template <typename, int> class K, typename... A>
hipError_t dispatch(const Params& P, A&&... args) {
  if (P.store == 0) {
    if (P.ncomp == 2) return K<StoreF32, 2>::launch(P, args...);
    return K<StoreF32, 1>::launch(P, args...);
  }
  if (P.ncomp == 2) return K<StoreF16, 2>::launch(P, args...);
  return K<StoreF16, 1>::launch(P, args...);
}

template <typename S, int NC>
struct RestL {
  static hipError_t launch(const Params& P, const float* bg, float* out, int* it, hipStream_t st) {
    hipLaunchKernelGGL((k_rest_state<S, NC>), dim3(1), dim3(64), 0, st, P, bg, out, it);
    return hipGetLastError();
  }
};
template <typename S, int NC>
struct InitL {
  static hipError_t launch(const Params& P, const Buffers& D, int buf, int first, int count, bool from_dev,
                           bool use_init, int mode, int born, hipStream_t st) {
    const int grid = from_dev ? 2048 : (count > 0 ? (count * kInitParts < 8192 ? count * kInitParts : 8192) : 1);
    hipLaunchKernelGGL((k_init<S, false>), dim3(grid), dim3(256), 0, st, P, D, buf, first, count, from_dev ? 1 : 0,
                       use_init ? 1 : 0, Batch{}, mode, born);
    return hipGetLastError();
  }
};
template <typename S, int NC>
struct DebugL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, float* psi_slots, float* dp,
                           float* df, hipStream_t st) {
    const dim3 g(grid_for(P.capacity)), b(kThreads);
    return with_rd<S>(rd, [&](auto R) {
      constexpr int M = decltype(R)::value;
      hipLaunchKernelGGL((k_debug_psi<S, NC, M>), g, b, 0, st, P, D, rbuf, psi_slots);
      hipLaunchKernelGGL((k_debug_force<S, NC, M>), g, b, 0, st, P, D, rbuf, psi_slots, dp, df);
      return hipGetLastError();
    });
  }
};
template <typename S, int NC>
struct FusedL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, bool pull, int parts, hipStream_t st) {
    const dim3 g(grid_for(P.capacity * parts)), b(kFusedThreads);
    const auto kpull = fused_kernel<S, NC, true, false>();
    const auto kfirst = fused_kernel<S, NC, false, false>();
    if (pull)
      hipLaunchKernelGGL(kpull, g, b, 0, st, P, D, rbuf, Batch{}, parts);
    else
      hipLaunchKernelGGL(kfirst, g, b, 0, st, P, D, rbuf, Batch{}, parts);
    return hipGetLastError();
  }
};
template <typename S, int NC>
struct CriterionL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, int flags, hipStream_t st) {
    const dim3 g(grid_for(P.capacity)), b(kThreads);
    return with_rd<S>(rd, [&](auto R) {
      hipLaunchKernelGGL((k_criterion<S, NC, decltype(R)::value, false>), g, b, 0, st, P, D, rbuf, flags, Batch{});
      return hipGetLastError();
    });
  }
};
template <typename S, int NC>
struct InplaceL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, bool collide_pass, hipStream_t st) {
    const dim3 g(grid_for(P.capacity));
    return with_rd<S>(rd, [&](auto R) {
      constexpr int M = decltype(R)::value;
      if constexpr (M == kRdPull) {
        return hipErrorInvalidValue;
      } else {
        if (collide_pass)
          hipLaunchKernelGGL((k_inplace_collide<S, NC, M, false>), g, dim3(kInplaceThreads), 0, st, P, D, rbuf,
                             Batch{});
        else
          hipLaunchKernelGGL((k_inplace_psi<S, NC, M, false>), g, dim3(kThreads), 0, st, P, D, rbuf, Batch{});
        return hipGetLastError();
      }
    });
  }
};
template <typename S, int NC>
struct ProposeL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, int step, const float* mlp,
                           float thr, float* feat, int32_t* block, int cap, hipStream_t st) {
    const dim3 g(P.nb > 0 ? P.nb : 1), b(kPropThreads);
    return with_rd<S>(rd, [&](auto R) {
      hipLaunchKernelGGL((k_propose<S, NC, decltype(R)::value>), g, b, 0, st, P, D, rbuf, step, mlp, thr, feat,
                         block, cap);
      return hipGetLastError();
    });
  }
};
// Batched stepping: prefix sums of the members' active counts (the merged
// active list), and the members' step counters.
__global__ void k_batch_offsets(Batch B) {
  if (threadIdx.x != 0) return;
  int acc = 0;
  B.off[0] = 0;
  for (int i = 0; i < B.nsims; ++i) {
    acc += B.D[i].ctrl[kNActive];
    B.off[i + 1] = acc;
  }
}
__global__ void k_batch_tick(Batch B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B.nsims) B.D[i].ctrl[kStepCount] += 1;
  if (i < kXcds) B.heads[i] = 0;  // the persistent step kernel's queues, for the next step
}

// Resident workgroups of the persistent step kernel on the current device.
template <typename S, int NC, bool PULL>
int persistent_grid() {
  static const int grid = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_persistent<S, NC, PULL>, kFusedThreads, 0) !=
        hipSuccess)
      return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
  }();
  return grid;
}
template <typename S, int NC>
struct BatchL {
  static hipError_t launch(const Params& P0, const Batch& B, int rbuf, bool first, bool progressive,
                           bool in_place, int parts, bool persistent, hipStream_t st) {
    const dim3 gc(grid_for(B.total_capacity)), bc(kThreads), gf(grid_for(B.total_capacity * parts)),
        bf(kFusedThreads);
    if (in_place) {
      // the step's index has the parity of rbuf (both flip every step)
      const int rd = first ? kRdOwn : (rbuf ? kRdAAOdd : kRdAAEven);
      const int mode = first ? kInitNatural : (rbuf ? kInitSwapped : kInitStash);
      return with_rd<S>(rd, [&](auto R) {
        constexpr int M = decltype(R)::value;
        if constexpr (M == kRdPull) {
          return hipErrorInvalidValue;
        } else {
          if (progressive) {
            const int flags = first ? (kCritRecord | kCritExposure)
                                    : (kCritRecord | kCritEval | kCritExposure | kCritEmission);
            hipLaunchKernelGGL((k_criterion<S, NC, M, true>), gc, bc, 0, st, P0, Buffers{}, rbuf, flags, B);
            hipLaunchKernelGGL((k_activate<true>), dim3(B.nsims), dim3(1024), 0, st, P0, Buffers{}, 0, B);
            hipLaunchKernelGGL((k_init<S, true>), dim3(64, B.nsims), dim3(256), 0, st, P0, Buffers{}, rbuf, 0, 0, 1, 0, B,
                               mode, -1);
            hipLaunchKernelGGL(k_batch_offsets, dim3(1), dim3(64), 0, st, B);
          }
          hipLaunchKernelGGL((k_inplace_psi<S, NC, M, true>), gc, bc, 0, st, P0, Buffers{}, rbuf, B);
          hipLaunchKernelGGL((k_inplace_collide<S, NC, M, true>), gc, dim3(kInplaceThreads), 0, st, P0, Buffers{},
                             rbuf, B);
          hipLaunchKernelGGL(k_batch_tick, dim3((B.nsims + 63) / 64), dim3(64), 0, st, B);
          return hipGetLastError();
        }
      });
    }
    if (progressive) {
      const int flags = first ? (kCritRecord | kCritExposure)
                              : (kCritRecord | kCritEval | kCritExposure | kCritEmission);
      if (first)
        hipLaunchKernelGGL((k_criterion<S, NC, kRdOwn, true>), gc, bc, 0, st, P0, Buffers{}, rbuf, flags, B);
      else
        hipLaunchKernelGGL((k_criterion<S, NC, kRdPull, true>), gc, bc, 0, st, P0, Buffers{}, rbuf, flags, B);
      hipLaunchKernelGGL((k_activate<true>), dim3(B.nsims), dim3(1024), 0, st, P0, Buffers{}, 0, B);
      hipLaunchKernelGGL((k_init<S, true>), dim3(64, B.nsims), dim3(256), 0, st, P0, Buffers{}, rbuf, 0, 0, 1, 0, B,
                         (int)kInitNatural, -1);
      hipLaunchKernelGGL(k_batch_offsets, dim3(1), dim3(64), 0, st, B);
    }
    if (persistent) {
      // resident grid, no more workgroups than items
      const int items = grid_for(B.total_capacity * parts);
      const int res = first ? persistent_grid<S, NC, false>() : persistent_grid<S, NC, true>();
      if (res <= 0) return hipErrorInvalidValue;
      const dim3 gp(res < items ? res : items);
      if (first)
        hipLaunchKernelGGL((k_fused_persistent<S, NC, false>), gp, bf, 0, st, B, rbuf, parts);
      else
        hipLaunchKernelGGL((k_fused_persistent<S, NC, true>), gp, bf, 0, st, B, rbuf, parts);
    } else if (first) {
      const auto k = fused_kernel<S, NC, false, true>();
      hipLaunchKernelGGL(k, gf, bf, 0, st, P0, Buffers{}, rbuf, B, parts);
    } else {
      const auto k = fused_kernel<S, NC, true, true>();
      hipLaunchKernelGGL(k, gf, bf, 0, st, P0, Buffers{}, rbuf, B, parts);
    }
    hipLaunchKernelGGL(k_batch_tick, dim3((B.nsims + 63) / 64), dim3(64), 0, st, B);
    return hipGetLastError();
  }
};
template <typename S, int NC>
struct ExportL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, float* r, float* u, float* m,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_fill_default, dim3(2048), dim3(256), 0, st, P, D, r, u, m);
    return with_rd<S>(rd, [&](auto R) {
      hipLaunchKernelGGL((k_export<S, NC, decltype(R)::value>), dim3(grid_for(P.capacity)), dim3(kThreads), 0, st, P,
                         D, rbuf, r, u, m);
      return hipGetLastError();
    });
  }
};
template <typename S, int NC>
struct MassL {
  static hipError_t launch(const Params& P, const Buffers& D, int rbuf, int rd, double* out, hipStream_t st) {
    return with_rd<S>(rd, [&](auto R) {
      hipLaunchKernelGGL((k_mass<S, NC, decltype(R)::value>), dim3(grid_for(P.capacity)), dim3(kThreads), 0, st, P, D,
                         rbuf, out);
      return hipGetLastError();
    });
  }
};

}  // namespace

// ------------------------------------------------------ static staging
// Device staging of the allocation-free moments export: one copy of this
// array per GPU, held until the process ends.  Host code never uses the
// name itself (on the host it is not a device address): static_staging()
// looks up each device's copy with hipGetSymbolAddress.
static __device__ __align__(256) float scratch[kStaticStagingFloats];

hipError_t static_staging(float** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    float* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_active_cells(const Params& P, const Buffers& D, uint8_t* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_active_cells, dim3(2048), dim3(256), 0, stream, P, D, out);
  return hipGetLastError();
}

hipError_t launch_repack(const Params& P, const Buffers& D, int rbuf, bool in_place, hipStream_t stream) {
  // scratch: the population buffer the next step writes (two buffers), or
  // the psi planes, which the next step computes again (in place); either
  // holds at least one plane of any slot-indexed array
  char* scratch = reinterpret_cast<char*>(in_place ? static_cast<void*>(D.psi) : D.f[rbuf ^ 1]);
  if (!scratch) return hipErrorInvalidValue;
  const size_t plane = P.plane;
  const dim3 grid(1024), block(256);
  hipError_t e = hipSuccess;
  auto one = [&](void* base, size_t bytes_per_cell) {
    if (e != hipSuccess) return;
    const uint32_t slot_vec = (uint32_t)(P.slot_cells * bytes_per_cell / 16);
    hipLaunchKernelGGL(k_repack_plane, grid, block, 0, stream, reinterpret_cast<const uint4*>(base),
                       reinterpret_cast<uint4*>(scratch), D.order, D.ctrl, slot_vec, 1);
    hipLaunchKernelGGL(k_repack_plane, grid, block, 0, stream, reinterpret_cast<const uint4*>(scratch),
                       reinterpret_cast<uint4*>(base), D.order, D.ctrl, slot_vec, 0);
    e = hipGetLastError();
  };
  // the populations the next step reads: one plane per direction, every
  // component of a link side by side
  const size_t link = (size_t)P.ncomp * (P.store ? 2 : 4);
  char* f = reinterpret_cast<char*>(D.f[rbuf]);
  for (int i = 0; i < kQ; ++i) one(f + (size_t)i * plane * link, link);
  one(D.mask, 4);
  if (D.uprev)
    for (int k = 0; k < 3 * P.ncomp; ++k) one(D.uprev + (size_t)k * plane, 4);
  if (P.store)
    for (int b = 0; b < 2; ++b) one(D.rho[b], (size_t)4 * P.ncomp);
  if (e != hipSuccess) return e;
  int32_t* tmp = reinterpret_cast<int32_t*>(scratch);
  hipLaunchKernelGGL(k_repack_tables_gather, dim3(256), block, 0, stream, D, tmp, P.capacity);
  hipLaunchKernelGGL(k_repack_tables_apply, dim3(256), block, 0, stream, D, static_cast<const int32_t*>(tmp),
                     P.capacity);
  return hipGetLastError();
}

// --------------------------------------------------------------- launchers
hipError_t launch_rest_state(const Params& P, const float* bg, float* out, int* iters, hipStream_t stream) {
  return dispatch<RestL>(P, bg, out, iters, stream);
}

hipError_t launch_init_slots(const Params& P, const Buffers& D, int buf, int first, int count, bool from_dev,
                             bool use_init, hipStream_t stream, int mode, int born) {
  return dispatch<InitL>(P, D, buf, first, count, from_dev, use_init, mode, born, stream);
}

hipError_t launch_activate(const Params& P, const Buffers& D, int step, hipStream_t stream) {
  hipLaunchKernelGGL((k_activate<false>), dim3(1), dim3(1024), 0, stream, P, D, step, Batch{});
  return hipGetLastError();
}

hipError_t launch_fused(const Params& P, const Buffers& D, int rbuf, bool pull, int parts, hipStream_t stream) {
  if (parts != 1 && parts != 2 && parts != 4) return hipErrorInvalidValue;
  return dispatch<FusedL>(P, D, rbuf, pull, parts, stream);
}

hipError_t launch_criterion(const Params& P, const Buffers& D, int rbuf, int rd, int flags,
                            hipStream_t stream) {
  return dispatch<CriterionL>(P, D, rbuf, rd, flags, stream);
}

hipError_t launch_inplace_psi(const Params& P, const Buffers& D, int rbuf, int rd, hipStream_t stream) {
  return dispatch<InplaceL>(P, D, rbuf, rd, false, stream);
}

hipError_t launch_inplace_collide(const Params& P, const Buffers& D, int rbuf, int rd, hipStream_t stream) {
  return dispatch<InplaceL>(P, D, rbuf, rd, true, stream);
}

hipError_t launch_batch_offsets(const Batch& B, const Params& P0, hipStream_t stream) {
  (void)P0;
  hipLaunchKernelGGL(k_batch_offsets, dim3(1), dim3(64), 0, stream, B);
  return hipGetLastError();
}

hipError_t launch_batch_step(const Batch& B, const Params& P0, int rbuf, bool first, bool progressive,
                             bool in_place, int parts, bool persistent, hipStream_t stream) {
  if (parts != 1 && parts != 2 && parts != 4) return hipErrorInvalidValue;
  return dispatch<BatchL>(P0, B, rbuf, first, progressive, in_place, parts, persistent, stream);
}

hipError_t launch_candidates(const Params& P, const Buffers& D, hipStream_t stream) {
  hipLaunchKernelGGL(k_candidates, dim3(1), dim3(1024), 0, stream, P, D);
  return hipGetLastError();
}

hipError_t launch_propose(const Params& P, const Buffers& D, int rbuf, int rd, int step, const float* mlp,
                          float thr, float* feat, int32_t* block, int cap, hipStream_t stream) {
  return dispatch<ProposeL>(P, D, rbuf, rd, step, mlp, thr, feat, block, cap, stream);
}

hipError_t launch_export(const Params& P, const Buffers& D, int rbuf, int rd, float* rho, float* u, float* umix,
                         hipStream_t stream) {
  return dispatch<ExportL>(P, D, rbuf, rd, rho, u, umix, stream);
}

hipError_t launch_mass(const Params& P, const Buffers& D, int rbuf, int rd, double* out, hipStream_t stream) {
  return dispatch<MassL>(P, D, rbuf, rd, out, stream);
}

hipError_t launch_debug_fields(const Params& P, const Buffers& D, int rbuf, int rd, float* psi_slots, float* psi,
                               float* force, hipStream_t stream) {
  return dispatch<DebugL>(P, D, rbuf, rd, psi_slots, psi, force, stream);
}

}  // namespace lbm
