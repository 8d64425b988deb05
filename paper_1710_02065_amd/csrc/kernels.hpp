// Device code of the fused pull-stream + Hermite-regularized collision sweep
// and its companion kernels (initialisation, moments, probes, population
// import/export).
//
// One thread updates one cell.  Populations are structure-of-arrays,
// buf[i * P + c] with c = (z*ny + y)*nx + x, so a wavefront's 64 lanes read
// 64 consecutive cells of one population: every load and store is coalesced,
// and the pull offsets xi_i shift the addresses by whole rows/planes or by
// one element.  The step is bound by HBM bandwidth (read q, write q values
// per cell); there is no dense contraction, so no matrix cores are used.
//
// All non-FP64 formats compute in FP32 on deviations from the rest state
// h_i = f_i - w_i rho0, so the moments are sums of small numbers:
//   drho = sum h_i, j = sum h_i xi_i, P = sum h_i xi_i xi_i = Pi - rho0 cs^2 I.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice.hpp"

namespace hrlbm {

enum : int { kPeriodic = 0, kFreeSlip = 1, kOutflow = 2, kHalo = 3 };
// cell kinds: the public FLUID/SOLID/INLET, and the refinement roles
// COVERED (coarse node under the fine patch), IMPORT (coarse node rebuilt
// from fine data), RING (fine node rebuilt from coarse data); cells of the
// three internal kinds are not swept.
enum : uint8_t { kFluid = 0, kSolid = 1, kInlet = 2, kCovered = 3, kImport = 4, kRing = 5 };
// The mask byte holds the kind in its low three bits and flags: the cell
// has a SOLID neighbour, or it lies on a non-periodic face (both computed at
// initialisation; cells with neither pull like a periodic grid), or it lies
// in an absorbing layer given per cell.
// A tile of 64 consecutive cells (one wavefront) whose cells are all FLUID
// without flags is "plain": its sweep does not read the mask at all.
enum : uint8_t { kKindBits = 0x07, kFieldSponge = 0x08, kNearFace = 0x40, kNearSolid = 0x80 };

// ------------------------------------------------------------------------
// Division of 32-bit unsigned numbers below 2^31 by a run-time invariant
// divisor with one multiply-high, add and shift (Granlund & Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994).
// ------------------------------------------------------------------------
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{d, (uint32_t)m, l};
}

__host__ __device__ inline uint32_t fast_div(uint32_t n, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t t = __umulhi(n, f.m);
#else
  const uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
  return (t + n) >> f.s;
}

// ------------------------------------------------------------------------
// Storage formats
// ------------------------------------------------------------------------
struct StoreF64 {
  using T = double;
  using R = double;
  static constexpr bool kShifted = false;
};
struct StoreF32 {
  using T = float;
  using R = float;
  static constexpr bool kShifted = false;
};
struct StoreF32S {
  using T = float;
  using R = float;
  static constexpr bool kShifted = true;
};
struct StoreF16S {
  using T = _Float16;
  using R = float;
  static constexpr bool kShifted = true;
};

// stored value -> deviation h = f - w rho0
template <class S>
__device__ __forceinline__ typename S::R decode(typename S::T v,
                                                typename S::R wrho0) {
  using R = typename S::R;
  if constexpr (S::kShifted)
    return (R)v;
  else
    return (R)v - wrho0;
}
// deviation -> stored value (round to nearest even for narrowing formats)
template <class S>
__device__ __forceinline__ typename S::T encode(typename S::R h,
                                                typename S::R wrho0) {
  using T = typename S::T;
  if constexpr (S::kShifted)
    return (T)h;
  else
    return (T)(h + wrho0);
}

// Element idx of the population array starting at `base`, addressed as a
// uniform 64-bit base plus a 32-bit byte offset (every population array is
// smaller than 4 GiB; checked when a context is created), which maps onto
// the scalar-base global memory instructions.
template <class T>
__device__ __forceinline__ T load_pop(const T* base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     (uint32_t)(idx * (uint32_t)sizeof(T)));
}
// The same load with the non-temporal hint (streamed through the caches).
template <class T>
__device__ __forceinline__ T load_pop_nt(const T* base, uint32_t idx) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(
      reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T))));
}
// Non-temporal store of element idx of a population array through a raw
// buffer resource (scalar base, 32-bit offset, stores past `bytes` are
// dropped by the hardware).  The third resource word 0x00020000 is the
// gfx9-family untyped 32-bit data format.
template <class T>
__device__ __forceinline__ void store_pop_nt(T* base, uint32_t bytes, uint32_t idx, T v) {
  __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
  constexpr int kNonTemporal = 2;
  const uint32_t off = idx * (uint32_t)sizeof(T);
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0,
                                          kNonTemporal);
  }
  else if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0,
                                          kNonTemporal);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, off, 0,
                                          kNonTemporal);
}

// ------------------------------------------------------------------------
// Kernel arguments
// ------------------------------------------------------------------------
template <class S>
struct SweepArgs {
  using T = typename S::T;
  using R = typename S::R;
  const T* src;          // post-collision state at t
  T* dst;                // post-collision state at t + 1
  const uint8_t* mask;   // nullptr = all fluid
  const uint8_t* tiles;  // per 64-cell tile: 1 = plain (see the mask bits)
  int* status;           // sticky instability flag
  uint32_t nx, ny, nz, ncell;
  uint64_t pstride;      // population stride P >= ncell
  FastDiv div_nx, div_ny;
  R omega1;              // 1 - 1/tau
  R rho0;
  R chi_max, rho_ref, uref[3];
  R uin[3], noise;
  int32_t face[6];
  int32_t sponge[6];
  uint64_t seed;
  uint64_t t_new;        // time index of the state being produced
  int32_t level;
  uint32_t lstride;      // inlet-noise counter blocks per time index
  uint32_t ntiles;
  // workgroups per XCD run: runs of xcd_group consecutive tiles go to one
  // XCD (1: plain round-robin)
  uint32_t xcd_group;
  // refinement: pre-collision moments of the coarse nodes on the patch
  // boundary planes are recorded into rec (10 contiguous components per
  // node of the record box [rec_off, rec_off + rec_dim)); rec == nullptr
  // disables it
  R* rec;
  int32_t rec_off[3];
  uint32_t rec_dim[3];
  uint32_t rec_n;
  int32_t box_lo[3], box_hi[3];
  // refinement, child side: pre-collision moments of the nodes in the band
  // the parent's IMPORT nodes filter are recorded into recf (10 contiguous
  // components per node, indexed by the node over all ncell nodes of this
  // level); nullptr disables it
  R* recf;
  // refinement, child side: RING nodes rebuilt by this sweep from the
  // parent's records ring_wa * ring_Ma + ring_wb * ring_Mb (record box
  // [ring_off, ring_off + ring_dim) in parent coordinates, this level's box
  // at ring_lo, stress scaled by ring_alpha); ring_Ma == nullptr: RING nodes
  // are not written
  const R* ring_Ma;
  const R* ring_Mb;
  R ring_wa, ring_wb, ring_alpha;
  int32_t ring_lo[3], ring_off[3];
  uint32_t ring_dim[3];
  // absorbing layer given per cell: chi, rho_ref, u_ref (5 x ncell), read
  // for cells flagged kFieldSponge; nullptr: none
  const R* sp;
  // halo faces of the last axis (slab decomposition), side 0 = low, 1 =
  // high: populations entering through the face are read from hrecv[side],
  // those leaving are written to hsend[side] (nullptr: no pack), each
  // [rank][cell of the face plane] with hplane cells per plane; rank as in
  // halo_rank()
  const T* hrecv[2];
  T* hsend[2];
  uint32_t hplane;
};

// Component of a direction along the last axis (the slab-cut axis: z in
// 3D, y on D2Q9).
template <class L>
__host__ __device__ constexpr int last_component(const Dir& v) {
  return L::D == 3 ? v.z : v.y;
}
// Rank of direction i among the directions with the same last-axis
// component, in direction order: the row of the halo buffers holding it.
template <class L>
struct HaloRankTable {
  int v[27];
  constexpr HaloRankTable() : v() {
    for (int i = 0; i < L::Q; ++i) {
      int r = 0;
      for (int j = 0; j < i; ++j)
        if (last_component<L>(L::dir(j)) == last_component<L>(L::dir(i))) ++r;
      v[i] = r;
    }
  }
};
template <class L>
__host__ __device__ constexpr int halo_rank(int i) {
  return HaloRankTable<L>{}.v[i];
}
// directions crossing one halo face: 3 (D2Q9), 5 (D3Q19), 9 (D3Q27)
template <class L>
__host__ __device__ constexpr int halo_count() {
  int n = 0;
  for (int i = 0; i < L::Q; ++i)
    if (last_component<L>(L::dir(i)) == 1) ++n;
  return n;
}

// Band of a child level whose pre-collision moments its parent's IMPORT
// nodes filter: the parent's IMPORT shell [lo+1, hi-1] lies on child index 2
// and n - 3 of each axis, and the 3-point filter reaches one node further
// either way, so the band is every node inside [1, n - 2] on the active axes
// with index 1, 2, 3, n - 4, n - 3 or n - 2 on at least one of them.
template <int D>
__host__ __device__ inline bool in_import_band(uint32_t x, uint32_t y, uint32_t z, uint32_t nx,
                                               uint32_t ny, uint32_t nz) {
  const uint32_t p[3] = {x, y, z}, n[3] = {nx, ny, nz};
  bool edge = false;
  for (int a = 0; a < D; ++a) {
    if (p[a] < 1 || p[a] + 2 > n[a]) return false;
    if (p[a] <= 3 || p[a] + 4 >= n[a]) edge = true;
  }
  return edge;
}

// Index into the record box of a coarse node on a patch boundary plane, or
// -1 if the node is not recorded.  The record box spans [lo - 1, hi + 1] on
// the active axes; recorded nodes lie on a plane x_a = lo_a or x_a = hi_a.
template <int D>
__host__ __device__ inline int64_t record_index(const int32_t off[3],
                                                const uint32_t dim[3],
                                                const int32_t lo[3],
                                                const int32_t hi[3], uint32_t x,
                                                uint32_t y, uint32_t z) {
  const int32_t p[3] = {(int32_t)x, (int32_t)y, (int32_t)z};
  bool on_plane = false;
  int64_t idx = 0, stride = 1;
  for (int ax = 0; ax < 3; ++ax) {
    const int32_t r = p[ax] - off[ax];
    if (r < 0 || r >= (int32_t)dim[ax]) return -1;
    idx += (int64_t)r * stride;
    stride *= dim[ax];
    if (ax < D && (p[ax] == lo[ax] || p[ax] == hi[ax])) on_plane = true;
  }
  return on_plane ? idx : -1;
}

// ------------------------------------------------------------------------
// Regularized rebuild (eqs. eqH, neqH, optimizedLB) from Hermite
// coefficients.  With the combined coefficients
//   m0 (scalar), m1 (vector), m2 (symmetric), m3 (third-order set)
// the deviation from rest of every population is
//   h_i = w_i [ m0 + xi.m1 / cs^2 + H2(xi):m2 / (2 cs^4)
//              + sum_k H_k(xi) c_k(m3) / N_k ].
// ------------------------------------------------------------------------
template <class L, class R>
struct Coeffs {
  R m0;
  R m1[3];
  R m2[6];  // xx, yy, zz, xy, xz, yz
  R m3[7];  // xxy, xyy, xxz, xzz, yyz, yzz, xyz
  R mh[L::KH > 0 ? L::KH : 1];  // order >= 4 (full order only), divided by N_k
};

// Compile-time loop (the index is a constant in the body).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// All q populations from the coefficients.  Directions come in opposite
// pairs (2k-1, 2k) with xi_{2k} = -xi_{2k-1}: the zeroth- and second-order
// terms are even in xi, the first- and third-order terms odd, so each pair
// costs one even and one odd sum.  `base` is added to m0 (rho0 when the
// stored value is f itself, 0 when it is the deviation from rest).
template <class L, class R>
__device__ __forceinline__ void rebuild_all(const Coeffs<L, R>& c, const R bk[L::K], R base,
                                            R out[L::Q]) {
  const R tr = c.m2[0] + c.m2[1] + (L::D == 3 ? c.m2[2] : (R)0);
  // even part at xi = 0: m0 - cs^2 tr / (2 cs^4) = m0 - 1.5 tr
  const R e0 = base + c.m0 - (R)1.5 * tr;
  const R m1s[3] = {(R)3 * c.m1[0], (R)3 * c.m1[1], (R)3 * c.m1[2]};
  const R d2[3] = {(R)4.5 * c.m2[0], (R)4.5 * c.m2[1], (R)4.5 * c.m2[2]};
  const R o2[3] = {(R)9 * c.m2[3], (R)9 * c.m2[4], (R)9 * c.m2[5]};
  if constexpr (L::KH > 0) {
    R h0 = e0;
    static_for<0, L::KH>([&](auto KK) {
      constexpr double hk = high_h<L>(0, decltype(KK)::value);
      if constexpr (hk != 0.0) h0 += (R)hk * c.mh[decltype(KK)::value];
    });
    out[0] = (R)L::w(0) * h0;
  } else {
    out[0] = (R)L::w(0) * e0;
  }
  static_for<0, (L::Q - 1) / 2>([&](auto K) {
    constexpr int i = 1 + 2 * decltype(K)::value;
    constexpr Dir v = L::dir(i);
    R even = e0;
    if constexpr (v.x != 0) even += d2[0];
    if constexpr (v.y != 0) even += d2[1];
    if constexpr (v.z != 0) even += d2[2];
    if constexpr (v.x * v.y > 0) even += o2[0];
    if constexpr (v.x * v.y < 0) even -= o2[0];
    if constexpr (v.x * v.z > 0) even += o2[1];
    if constexpr (v.x * v.z < 0) even -= o2[1];
    if constexpr (v.y * v.z > 0) even += o2[2];
    if constexpr (v.y * v.z < 0) even -= o2[2];
    R odd = (R)0;
    if constexpr (v.x > 0) odd += m1s[0];
    if constexpr (v.x < 0) odd -= m1s[0];
    if constexpr (v.y > 0) odd += m1s[1];
    if constexpr (v.y < 0) odd -= m1s[1];
    if constexpr (v.z > 0) odd += m1s[2];
    if constexpr (v.z < 0) odd -= m1s[2];
    static_for<0, L::K>([&](auto KK) {
      constexpr double hk = basis_h<L>(i, decltype(KK)::value);
      if constexpr (hk != 0.0) odd += (R)hk * bk[decltype(KK)::value];
    });
    // orders 4 to 6: even orders join the even part, odd orders the odd
    static_for<0, L::KH>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      constexpr double hk = high_h<L>(i, k);
      if constexpr (hk != 0.0) {
        if constexpr (high_order(L::high(k)) % 2 == 0)
          even += (R)hk * c.mh[k];
        else
          odd += (R)hk * c.mh[k];
      }
    });
    constexpr R w = (R)L::w(i);
    out[i] = w * (even + odd);
    out[i + 1] = w * (even - odd);
  });
}

// third-order set -> basis coefficients c_k / N_k
template <class L, class R>
__device__ __forceinline__ void basis_coeffs(const R m3[7], R bk[L::K]) {
#pragma unroll
  for (int k = 0; k < L::K; ++k) {
    const Basis3 b = L::basis(k);
    R v = (R)b.sgn[0] * m3[b.idx[0]];
    if (b.n == 2) v += (R)b.sgn[1] * m3[b.idx[1]];
    bk[k] = v * (R)(1.0 / basis_norm<L>(k));
  }
}

// Third-order non-equilibrium coefficients from the recursion eq.
// (recursive2) at n = 3: t_abc = u_a A_bc + u_b A_ac + u_c A_ab for the seven
// packed components.  A in (xx, yy, zz, xy, xz, yz).
template <class R>
__device__ __forceinline__ void recursion3(const R u[3], const R A[6], R t[7]) {
  const R xx = A[0], yy = A[1], zz = A[2], xy = A[3], xz = A[4], yz = A[5];
  t[kXXY] = (R)2 * u[0] * xy + u[1] * xx;
  t[kXYY] = (R)2 * u[1] * xy + u[0] * yy;
  t[kXXZ] = (R)2 * u[0] * xz + u[2] * xx;
  t[kXZZ] = (R)2 * u[2] * xz + u[0] * zz;
  t[kYYZ] = (R)2 * u[1] * yz + u[2] * yy;
  t[kYZZ] = (R)2 * u[2] * yz + u[1] * zz;
  t[kXYZ] = u[0] * yz + u[1] * xz + u[2] * xy;
}

// u_a^n for n <= 2 (n is a constant after inlining)
template <class R>
__device__ __forceinline__ R upow(const R u[3], const R u2[3], int a, int n) {
  return n == 0 ? (R)1 : (n == 1 ? u[a] : u2[a]);
}

// packed index of a2_ab in (xx, yy, zz, xy, xz, yz)
constexpr int pack2(int a, int b) {
  return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

// Equilibrium and non-equilibrium Hermite coefficients of the high-order
// polynomial with multi-index m: eq = u^m (times rho by the caller), and the
// closed form of the recursion eq. (recursive2): a sum over every pair of
// positions in the index list of a2 on that pair times u over the rest,
// i.e. sum over a <= b of (n_a n_b, or n_a (n_a - 1) / 2 when a = b)
// a2_ab u^(m - e_a - e_b).
template <class R>
__device__ __forceinline__ void high_terms(const MultiIndex m, const R u[3], const R u2[3],
                                           const R a2[6], R& eq, R& neq) {
  eq = upow(u, u2, 0, m.n[0]) * upow(u, u2, 1, m.n[1]) * upow(u, u2, 2, m.n[2]);
  neq = (R)0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const int cnt = a == b ? m.n[a] * (m.n[a] - 1) / 2 : m.n[a] * m.n[b];
      if (cnt == 0) continue;
      int r[3] = {m.n[0], m.n[1], m.n[2]};
      r[a] -= 1;
      r[b] -= 1;
      neq += (R)cnt * a2[pack2(a, b)] * upow(u, u2, 0, r[0]) * upow(u, u2, 1, r[1]) *
             upow(u, u2, 2, r[2]);
    }
}

// High-order coefficients mh_k = (e rho u^m + chi rho_ref uref^m
// + omega1 a_neq) / N_k of the full-order rebuild.
template <class L, class R, bool kSponge>
__device__ __forceinline__ void high_coeffs(R rho, const R u[3], const R a2[6], R omega1,
                                            R chi, R rho_ref, const R uref[3],
                                            Coeffs<L, R>& c) {
  const R u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
  const R e = kSponge ? (R)1 - chi : (R)1;
  static_for<0, L::KH>([&](auto KK) {
    constexpr int k = decltype(KK)::value;
    constexpr MultiIndex m = L::high(k);
    R eq, neq;
    high_terms<R>(m, u, u2, a2, eq, neq);
    R v = e * rho * eq + omega1 * neq;
    if constexpr (kSponge) {
      const R r2[3] = {uref[0] * uref[0], uref[1] * uref[1], uref[2] * uref[2]};
      v += chi * rho_ref * upow(uref, r2, 0, m.n[0]) * upow(uref, r2, 1, m.n[1]) *
           upow(uref, r2, 2, m.n[2]);
    }
    c.mh[k] = v * (R)(1.0 / high_norm<L>(k));
  });
}

// rho u_a u_b u_c for the seven packed components
template <class R>
__device__ __forceinline__ void cube3(R rho, const R u[3], R t[7]) {
  const R ruu_x = rho * u[0], ruu_y = rho * u[1];
  t[kXXY] = ruu_x * u[0] * u[1];
  t[kXYY] = ruu_x * u[1] * u[1];
  t[kXXZ] = ruu_x * u[0] * u[2];
  t[kXZZ] = ruu_x * u[2] * u[2];
  t[kYYZ] = ruu_y * u[1] * u[2];
  t[kYZZ] = ruu_y * u[2] * u[2];
  t[kXYZ] = ruu_x * u[1] * u[2];
}

// Pre-collision moments of one cell from the pair sums s = h_i + h_{i+1} and
// differences d = h_i - h_{i+1} of its deviations h = f - w rho0:
// drho = sum h, j = sum h xi = sum d xi_i, P = sum h xi xi = sum s xi_i xi_i
// (P = Pi - rho0 cs^2 I).
template <class L, class R>
__device__ __forceinline__ void pair_moments(R h0, const R s[(L::Q - 1) / 2],
                                             const R d[(L::Q - 1) / 2], R& drho, R j[3],
                                             R P[6]) {
  drho = h0;
#pragma unroll
  for (int a = 0; a < 3; ++a) j[a] = (R)0;
#pragma unroll
  for (int a = 0; a < 6; ++a) P[a] = (R)0;
  static_for<0, (L::Q - 1) / 2>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr Dir v = L::dir(1 + 2 * k);
    drho += s[k];
    if constexpr (v.x > 0) j[0] += d[k];
    if constexpr (v.x < 0) j[0] -= d[k];
    if constexpr (v.y > 0) j[1] += d[k];
    if constexpr (v.y < 0) j[1] -= d[k];
    if constexpr (v.z > 0) j[2] += d[k];
    if constexpr (v.z < 0) j[2] -= d[k];
    if constexpr (v.x != 0) P[0] += s[k];
    if constexpr (v.y != 0) P[1] += s[k];
    if constexpr (v.z != 0) P[2] += s[k];
    if constexpr (v.x * v.y > 0) P[3] += s[k];
    if constexpr (v.x * v.y < 0) P[3] -= s[k];
    if constexpr (v.x * v.z > 0) P[4] += s[k];
    if constexpr (v.x * v.z < 0) P[4] -= s[k];
    if constexpr (v.y * v.z > 0) P[5] += s[k];
    if constexpr (v.y * v.z < 0) P[5] -= s[k];
  });
}

// Moments from the deviations h_i.
template <class L, class R>
__device__ __forceinline__ void raw_moments(const R h[L::Q], R& drho, R j[3], R P[6]) {
  constexpr int H = (L::Q - 1) / 2;
  R s[H], d[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    s[k] = h[1 + 2 * k] + h[2 + 2 * k];
    d[k] = h[1 + 2 * k] - h[2 + 2 * k];
  }
  pair_moments<L, R>(h[0], s, d, drho, j, P);
}

// Moments from stored values: shifted formats store h; the plain formats
// store f, and a pair's shift 2 w rho0 is removed from its sum only.
template <class L, class S>
__device__ __forceinline__ void stored_moments(const typename S::T raw[L::Q],
                                               typename S::R rho0, typename S::R& drho,
                                               typename S::R j[3], typename S::R P[6]) {
  using R = typename S::R;
  constexpr int H = (L::Q - 1) / 2;
  R s[H], d[H];
  static_for<0, H>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const R a = (R)raw[1 + 2 * k], b = (R)raw[2 + 2 * k];
    if constexpr (S::kShifted)
      s[k] = a + b;
    else
      s[k] = (a + b) - (R)(2.0 * L::w(1 + 2 * k)) * rho0;
    d[k] = a - b;
  });
  const R h0 = S::kShifted ? (R)raw[0] : (R)raw[0] - (R)L::w(0) * rho0;
  pair_moments<L, R>(h0, s, d, drho, j, P);
}

// 1 / x: hardware reciprocal in FP32 (one ulp), exact division in FP64
template <class R>
__device__ __forceinline__ R recip(R x) {
  if constexpr (sizeof(R) == 4)
    return __builtin_amdgcn_rcpf(x);
  else
    return (R)1 / x;
}

// a2_neq = Pi - rho cs^2 I - rho u u from the deviation moments
template <class L, class R>
__device__ __forceinline__ void noneq_stress(R drho, const R j[3], const R u[3],
                                             const R P[6], R a2[6]) {
  a2[0] = P[0] - (R)kCs2 * drho - j[0] * u[0];
  a2[1] = P[1] - (R)kCs2 * drho - j[1] * u[1];
  a2[2] = L::D == 3 ? P[2] - (R)kCs2 * drho - j[2] * u[2] : (R)0;
  a2[3] = P[3] - j[0] * u[1];
  a2[4] = L::D == 3 ? P[4] - j[0] * u[2] : (R)0;
  a2[5] = L::D == 3 ? P[5] - j[1] * u[2] : (R)0;
}

// Moments a collision used: rho* - rho0, u, a2_neq (all pre-collision).
template <class R>
struct CellMoments {
  R drho, u[3], a2[6];
};

// Hermite coefficients of one cell's collision (eq. optimizedLB, with eqs.
// spongeLB/dampingLBM and the modified moments at n = m = 1/2 where
// chi > 0): post = (1 - chi) E(rho*, u) + chi E(rho_ref, u_ref) + omega1 N.
// kSponge = false assumes chi = 0.  Returns rho* for the stability
// watchdog; fills *mo (pre-collision rho* - rho0, u, a2_neq) when given.
template <class L, class R, bool kSponge>
__device__ __forceinline__ R collide_coeffs(R drho, R j[3], const R P[6], R omega1, R rho0,
                                            R chi, R rho_ref, const R uref[3],
                                            Coeffs<L, R>& c, CellMoments<R>* mo = nullptr) {
  if constexpr (kSponge) {
    if (chi != (R)0) {
      const R k = recip((R)1 + (R)0.5 * chi);
      drho = (drho + (R)0.5 * chi * (rho_ref - rho0)) * k;
#pragma unroll
      for (int a = 0; a < 3; ++a) j[a] = (j[a] + (R)0.5 * chi * rho_ref * uref[a]) * k;
    }
  }
  const R rho = rho0 + drho;
  const R irho = recip(rho);
  R u[3] = {j[0] * irho, j[1] * irho, L::D == 3 ? j[2] * irho : (R)0};
  // a2_neq = Pi - rho cs^2 I - rho u u  (Pi - rho0 cs^2 I = P)
  R a2[6];
  noneq_stress<L, R>(drho, j, u, P, a2);
  if (mo) {
    mo->drho = drho;
#pragma unroll
    for (int a = 0; a < 3; ++a) mo->u[a] = u[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) mo->a2[a] = a2[a];
  }
  R a3n[7];
  recursion3<R>(u, a2, a3n);
  cube3<R>(rho, u, c.m3);
  c.m0 = drho;
#pragma unroll
  for (int a = 0; a < 3; ++a) c.m1[a] = j[a];
  c.m2[0] = j[0] * u[0];
  c.m2[1] = j[1] * u[1];
  c.m2[2] = j[2] * u[2];
  c.m2[3] = j[0] * u[1];
  c.m2[4] = j[0] * u[2];
  c.m2[5] = j[1] * u[2];
  if constexpr (kSponge) {
    if (chi != (R)0) {
      // (1 - chi) E(rho*, u) + chi E(rho_ref, u_ref)
      const R e = (R)1 - chi;
      const R ru[3] = {rho_ref * uref[0], rho_ref * uref[1], rho_ref * uref[2]};
      R a3r[7];
      cube3<R>(rho_ref, uref, a3r);
      c.m0 = e * c.m0 + chi * (rho_ref - rho0);
#pragma unroll
      for (int a = 0; a < 3; ++a) c.m1[a] = e * c.m1[a] + chi * ru[a];
      c.m2[0] = e * c.m2[0] + chi * ru[0] * uref[0];
      c.m2[1] = e * c.m2[1] + chi * ru[1] * uref[1];
      c.m2[2] = e * c.m2[2] + chi * ru[2] * uref[2];
      c.m2[3] = e * c.m2[3] + chi * ru[0] * uref[1];
      c.m2[4] = e * c.m2[4] + chi * ru[0] * uref[2];
      c.m2[5] = e * c.m2[5] + chi * ru[1] * uref[2];
#pragma unroll
      for (int k = 0; k < 7; ++k) c.m3[k] = e * c.m3[k] + chi * a3r[k];
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) c.m2[a] += omega1 * a2[a];
#pragma unroll
  for (int k = 0; k < 7; ++k) c.m3[k] += omega1 * a3n[k];
  if constexpr (L::KH > 0)
    high_coeffs<L, R, kSponge>(rho, u, a2, omega1, chi, rho_ref, uref, c);
  return rho;
}

// Populations from the Hermite coefficients (`base` added to m0: rho0 when
// the stored value is f itself, 0 when it is the deviation from rest).
template <class L, class R>
__device__ __forceinline__ void rebuild_from(const Coeffs<L, R>& c, R base, R out[L::Q]) {
  R bk[L::K];
  basis_coeffs<L, R>(c.m3, bk);
  rebuild_all<L, R>(c, bk, base, out);
}

// Collision of one cell: coefficients and rebuild.
template <class L, class R, bool kSponge>
__device__ __forceinline__ R collide_moments(R drho, R j[3], const R P[6], R omega1, R rho0,
                                             R chi, R rho_ref, const R uref[3], R base,
                                             R out[L::Q], CellMoments<R>* mo = nullptr) {
  Coeffs<L, R> c;
  const R rho = collide_coeffs<L, R, kSponge>(drho, j, P, omega1, rho0, chi, rho_ref, uref, c, mo);
  rebuild_from<L, R>(c, base, out);
  return rho;
}

// Collision of one cell from its pre-collision deviations h; out receives
// post-collision deviations.
template <class L, class R, bool kSponge>
__device__ __forceinline__ R collide(const R h[L::Q], R omega1, R rho0, R chi, R rho_ref,
                                     const R uref[3], R out[L::Q],
                                     CellMoments<R>* mo = nullptr) {
  R drho, j[3], P[6];
  raw_moments<L, R>(h, drho, j, P);
  return collide_moments<L, R, kSponge>(drho, j, P, omega1, rho0, chi, rho_ref, uref, (R)0,
                                        out, mo);
}

// ------------------------------------------------------------------------
// Comparator operators (Sec. II.A).  raw: the pulled stored values (f for
// the plain formats, h = f - w rho0 for the shifted ones); post receives
// values in the same domain.
// ------------------------------------------------------------------------

// LBM-BGK, eq. (standardLB) with the second-order equilibrium of eq.
// (truncatedEq) and the same damping force and modified moments as the
// regularized operator:
//   post = f - (f - feq(rho*, u)) / tau + chi (feq(rho_ref, u_ref) - feq(rho*, u)).
// The equilibria are rebuilt from their Hermite coefficients (second order
// only); base = omega rho0 for the plain formats carries the rest part of
// omega feq + chi (fref - feq).
template <class L, class S>
__device__ __forceinline__ typename S::R collide_bgk(const typename S::T raw[L::Q],
                                                     typename S::R drho,
                                                     typename S::R j[3], typename S::R omega1,
                                                     typename S::R rho0, typename S::R chi,
                                                     typename S::R rho_ref,
                                                     const typename S::R uref[3],
                                                     typename S::R post[L::Q]) {
  using R = typename S::R;
  if (chi != (R)0) {
    const R k = recip((R)1 + (R)0.5 * chi);
    drho = (drho + (R)0.5 * chi * (rho_ref - rho0)) * k;
#pragma unroll
    for (int a = 0; a < 3; ++a) j[a] = (j[a] + (R)0.5 * chi * rho_ref * uref[a]) * k;
  }
  const R rho = rho0 + drho;
  const R irho = recip(rho);
  const R u[3] = {j[0] * irho, j[1] * irho, L::D == 3 ? j[2] * irho : (R)0};
  const R omega = (R)1 - omega1;
  const R e = omega - chi;
  const R ru[3] = {rho_ref * uref[0], rho_ref * uref[1], rho_ref * uref[2]};
  Coeffs<L, R> c;
  c.m0 = e * drho + chi * (rho_ref - rho0);
#pragma unroll
  for (int a = 0; a < 3; ++a) c.m1[a] = e * j[a] + chi * ru[a];
  c.m2[0] = e * j[0] * u[0] + chi * ru[0] * uref[0];
  c.m2[1] = e * j[1] * u[1] + chi * ru[1] * uref[1];
  c.m2[2] = e * j[2] * u[2] + chi * ru[2] * uref[2];
  c.m2[3] = e * j[0] * u[1] + chi * ru[0] * uref[1];
  c.m2[4] = e * j[0] * u[2] + chi * ru[0] * uref[2];
  c.m2[5] = e * j[1] * u[2] + chi * ru[1] * uref[2];
#pragma unroll
  for (int k = 0; k < 7; ++k) c.m3[k] = (R)0;
  rebuild_from<L, R>(c, S::kShifted ? (R)0 : omega * rho0, post);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) post[i] += omega1 * (R)raw[i];
  return rho;
}

// MRT moment polynomials of D2Q9 (Lallemand & Luo, Phys. Rev. E 61, 6546,
// 2000) at an integer velocity: e, eps, q_x, q_y, p_xx, p_xy (the
// conserved rho, j_x, j_y are not relaxed), and their norms sum_i m_k(xi_i)^2.
constexpr double mrt_poly(const Dir& v, int k) {
  const double x = v.x, y = v.y, e2 = x * x + y * y;
  return k == 0   ? -4.0 + 3.0 * e2
         : k == 1 ? 4.0 - 10.5 * e2 + 4.5 * e2 * e2
         : k == 2 ? (-5.0 + 3.0 * e2) * x
         : k == 3 ? (-5.0 + 3.0 * e2) * y
         : k == 4 ? x * x - y * y
                  : x * y;
}
template <class L>
constexpr double mrt_norm(int k) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += mrt_poly(L::dir(i), k) * mrt_poly(L::dir(i), k);
  return s;
}

// LBM-MRT on D2Q9: each non-conserved moment relaxes towards its value for
// the second-order equilibrium at its own rate (s_e 1.64, s_eps 1.54,
// s_q 1.9 from Lallemand & Luo; s_nu = 1/tau), projected back with the
// orthogonal basis.  Written on deviations: m_k(f) - m_k,eq needs the rest
// state's moments e = -2 rho0, eps = rho0 only, which cancel against the
// equilibrium's own rho0 terms.
template <class L, class S>
__device__ __forceinline__ typename S::R collide_mrt(const typename S::T raw[L::Q],
                                                     typename S::R drho,
                                                     const typename S::R j[3],
                                                     typename S::R omega1, typename S::R rho0,
                                                     typename S::R post[L::Q]) {
  using R = typename S::R;
  R mh[6] = {(R)0, (R)0, (R)0, (R)0, (R)0, (R)0};
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const R h = decode<S>(raw[i], (R)L::w(i) * rho0);
    static_for<0, 6>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr double p = mrt_poly(L::dir(i), k);
      if constexpr (p != 0.0) mh[k] += (R)p * h;
    });
  });
  const R rho = rho0 + drho;
  const R irho = recip(rho);
  const R jj = (j[0] * j[0] + j[1] * j[1]) * irho;
  const R s_nu = (R)1 - omega1;
  R d[6];
  d[0] = (R)(1.64 / mrt_norm<L>(0)) * (mh[0] + (R)2 * drho - (R)3 * jj);
  d[1] = (R)(1.54 / mrt_norm<L>(1)) * (mh[1] - drho + (R)3 * jj);
  d[2] = (R)(1.9 / mrt_norm<L>(2)) * (mh[2] + j[0]);
  d[3] = (R)(1.9 / mrt_norm<L>(3)) * (mh[3] + j[1]);
  d[4] = s_nu * (R)(1.0 / mrt_norm<L>(4)) * (mh[4] - (j[0] * j[0] - j[1] * j[1]) * irho);
  d[5] = s_nu * (R)(1.0 / mrt_norm<L>(5)) * (mh[5] - j[0] * j[1] * irho);
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    R corr = (R)0;
    static_for<0, 6>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr double p = mrt_poly(L::dir(i), k);
      if constexpr (p != 0.0) corr += (R)p * d[k];
    });
    post[i] = (R)raw[i] - corr;
  });
  return rho;
}

// Hermite coefficients of f^{eqH}(rho, u) + omega1 f^{neqH}(a2, u) (initial
// state, inlet cells, refinement interfaces), rho given as its deviation
// drho from rho0.
template <class L, class R>
__device__ __forceinline__ void state_coeffs(R drho, R rho0, const R u[3], const R a2[6],
                                             R omega1, Coeffs<L, R>& c) {
  const R rho = rho0 + drho;
  c.m0 = drho;
  const R j[3] = {rho * u[0], rho * u[1], rho * u[2]};
#pragma unroll
  for (int a = 0; a < 3; ++a) c.m1[a] = j[a];
  c.m2[0] = j[0] * u[0] + omega1 * a2[0];
  c.m2[1] = j[1] * u[1] + omega1 * a2[1];
  c.m2[2] = j[2] * u[2] + omega1 * a2[2];
  c.m2[3] = j[0] * u[1] + omega1 * a2[3];
  c.m2[4] = j[0] * u[2] + omega1 * a2[4];
  c.m2[5] = j[1] * u[2] + omega1 * a2[5];
  R a3n[7], a3e[7];
  recursion3<R>(u, a2, a3n);
  cube3<R>(rho, u, a3e);
#pragma unroll
  for (int k = 0; k < 7; ++k) c.m3[k] = a3e[k] + omega1 * a3n[k];
  if constexpr (L::KH > 0)
    high_coeffs<L, R, false>(rho, u, a2, omega1, (R)0, (R)0, u, c);
}

// Deviations of f^{eqH}(rho, u) + omega1 f^{neqH}(a2, u).
template <class L, class R>
__device__ __forceinline__ void rebuild_state(R drho, R rho0, const R u[3],
                                              const R a2[6], R omega1,
                                              R out[L::Q]) {
  Coeffs<L, R> c;
  state_coeffs<L, R>(drho, rho0, u, a2, omega1, c);
  rebuild_from<L, R>(c, (R)0, out);
}

// ------------------------------------------------------------------------
// Absorbing-layer strength (Sec. II.C profile), analytic in the coordinates:
// chi = chi_max * max over faces of 3125 (L - s)(s - s0)^4 / (256 (L - s0)^5)
// with s the coordinate normal to the face (mirrored on low faces),
// s0 = n - W and L = n.
// ------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R sponge_chi(const int32_t* width, R chi_max,
                                        uint32_t x, uint32_t y, uint32_t z,
                                        uint32_t nx, uint32_t ny, uint32_t nz) {
  const uint32_t pos[3] = {x, y, z}, n[3] = {nx, ny, nz};
  R best = (R)0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int32_t W = width[f];
    if (W <= 0) continue;
    const int a = f >> 1;
    const R s = (f & 1) ? (R)pos[a] : (R)(n[a] - 1u - pos[a]);
    const R s0 = (R)(int64_t)(n[a] - (uint32_t)W);
    if (s < s0) continue;
    const R Lw = (R)W;
    const R d = (s - s0) / Lw;
    const R sig = (R)(3125.0 / 256.0) * ((R)1 - d) * (d * d) * (d * d);
    best = sig > best ? sig : best;
  }
  return chi_max * best;
}

// SplitMix64 output k of the generator seeded with `seed` (Steele, Lea &
// Flood, OOPSLA 2014), mapped to [-1, 1) with 2^-23 spacing.
__device__ __forceinline__ float splitmix_pm1(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (float)(uint32_t)(z >> 40) * (1.0f / 8388608.0f) - 1.0f;
}

}  // namespace hrlbm
