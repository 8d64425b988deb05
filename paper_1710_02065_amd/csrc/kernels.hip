// HIP kernels of the regularized LBM step and their host launchers.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace hrlbm {

// sweep arguments of one storage format from the format-neutral host block
template <class S>
__host__ __device__ inline SweepArgs<S> to_args_dev(const SweepHost& h);

// direction index for a velocity given at run time (only used after a
// free-slip reflection)
template <class L>
struct DirTable {
  int v[27];
  constexpr DirTable() : v() {
    for (int z = -1; z <= 1; ++z)
      for (int y = -1; y <= 1; ++y)
        for (int x = -1; x <= 1; ++x)
          v[(x + 1) + 3 * (y + 1) + 9 * (z + 1)] = find_dir<L>(x, y, z);
  }
};
template <class L>
__device__ __forceinline__ int dir_rt(int x, int y, int z) {
  constexpr DirTable<L> t{};
  return t.v[(x + 1) + 3 * (y + 1) + 9 * (z + 1)];
}

// ------------------------------------------------------------------------
// Pull under the face rules and the mask (left side of eq. optimizedLB read
// backwards): the source of population i is x - xi_i, mapped axis by axis
// (periodic wrap, free-slip reflection with the population mirrored,
// zero-gradient clamp, or the neighbour subdomain's values through a halo
// face); a link whose source is SOLID is bounced back halfway from this
// cell.  Applied as corrections to the periodic pull already in raw[]: only
// the directions whose source crosses a non-periodic face, or (for cells
// flagged kNearSolid) is SOLID, are loaded again.
// ------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ void pull_fixup(const SweepArgs<S>& a, uint32_t x, uint32_t y,
                                           uint32_t z, uint32_t c, bool near_solid,
                                           typename S::T raw[L::Q]) {
  const uint64_t P = a.pstride;
  const uint32_t dims[3] = {a.nx, a.ny, a.nz};
  static_for<1, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Dir v = L::dir(i);
    constexpr int vv[3] = {v.x, v.y, v.z};
    int32_t s[3] = {(int32_t)x - v.x, (int32_t)y - v.y, (int32_t)z - v.z};
    bool flip[3] = {false, false, false};
    bool cross = false;
    int hs = -1;  // halo side crossed (only the last axis has halo faces)
#pragma unroll
    for (int ax = 0; ax < L::D; ++ax) {
      if (vv[ax] == 0) continue;
      const int32_t n = (int32_t)dims[ax];
      const bool lo = s[ax] < 0, hi = s[ax] >= n;
      if (lo || hi) {
        const int32_t bc = a.face[2 * ax + (hi ? 1 : 0)];
        if (bc == kPeriodic) {
          s[ax] = lo ? s[ax] + n : s[ax] - n;
        } else {
          s[ax] = lo ? 0 : n - 1;
          flip[ax] = (bc == kFreeSlip);
          if (bc == kHalo) hs = hi ? 1 : 0;
          cross = true;
        }
      }
    }
    const uint32_t src = ((uint32_t)s[2] * a.ny + (uint32_t)s[1]) * a.nx + (uint32_t)s[0];
    if (near_solid && hs < 0 && (a.mask[src] & kKindBits) == kSolid) {
      // halfway bounce-back: the population that left this cell towards
      // the wall comes back reversed (same weight, so the same shift)
      constexpr int o = opposite<L>(i);
      raw[i] = load_pop(a.src + (uint64_t)o * P, c);
    } else if (cross) {
      int pop = i;
      if (flip[0] || flip[1] || flip[2])
        pop = dir_rt<L>(flip[0] ? -v.x : v.x, flip[1] ? -v.y : v.y,
                        flip[2] ? -v.z : v.z);
      if (hs >= 0) {
        // the source lies in the neighbour's face plane (mapped on the
        // other axes as above); a free-slip flip acts on the other axes
        // only, so the row is one of four known at compile time
        constexpr int r00 = halo_rank<L>(i);
        constexpr int r10 = halo_rank<L>(find_dir<L>(-v.x, v.y, v.z));
        constexpr int r01 = halo_rank<L>(find_dir<L>(v.x, -v.y, v.z));
        constexpr int r11 = halo_rank<L>(find_dir<L>(-v.x, -v.y, v.z));
        const int r = flip[0] ? (flip[1] ? r11 : r10) : (flip[1] ? r01 : r00);
        const uint32_t pc = L::D == 3 ? (uint32_t)s[1] * a.nx + (uint32_t)s[0] : (uint32_t)s[0];
        const typename S::T* rb = hs ? a.hrecv[1] : a.hrecv[0];
        raw[i] = load_pop(rb + (uint64_t)r * a.hplane, pc);
      } else {
        raw[i] = load_pop(a.src + (uint64_t)pop * P, src);
      }
    }
  });
}

// Halo faces on the periodic path (every other face periodic, no mask): a
// face-plane cell replaces the populations the periodic pull wrapped across
// a halo face by the neighbour's values, from the receive buffer at the
// source wrapped on the other axes.
template <class L, class S>
__device__ __forceinline__ void halo_pull_periodic(const SweepArgs<S>& a, uint32_t x,
                                                   uint32_t y, uint32_t z,
                                                   typename S::T raw[L::Q]) {
  const uint32_t zl = L::D == 3 ? z : y, nl = L::D == 3 ? a.nz : a.ny;
  const bool lo = zl == 0 && a.hrecv[0], hi = zl + 1 == nl && a.hrecv[1];
  if (!lo && !hi) return;
  static_for<1, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Dir v = L::dir(i);
    constexpr int vl = last_component<L>(v);
    if constexpr (vl != 0) {
      if ((vl > 0 && lo) || (vl < 0 && hi)) {
        int32_t sx = (int32_t)x - v.x;
        if (sx < 0) sx += (int32_t)a.nx;
        if (sx >= (int32_t)a.nx) sx -= (int32_t)a.nx;
        uint32_t pc = (uint32_t)sx;
        if constexpr (L::D == 3) {
          int32_t sy = (int32_t)y - v.y;
          if (sy < 0) sy += (int32_t)a.ny;
          if (sy >= (int32_t)a.ny) sy -= (int32_t)a.ny;
          pc += (uint32_t)sy * a.nx;
        }
        const typename S::T* rb = vl > 0 ? a.hrecv[0] : a.hrecv[1];
        raw[i] = load_pop(rb + (uint64_t)halo_rank<L>(i) * a.hplane, pc);
      }
    }
  });
}

// Pack of a face-plane cell's post-collision populations that leave
// through a halo face into that face's send buffer.
template <class L, class S>
__device__ __forceinline__ void halo_pack(const SweepArgs<S>& a, uint32_t c, uint32_t zl,
                                          uint32_t nl, const typename S::R post[L::Q]) {
  using T = typename S::T;
  const uint32_t pc = c - zl * a.hplane;
  const bool lo = zl == 0 && a.hsend[0], hi = zl + 1 == nl && a.hsend[1];
  static_for<1, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int vl = last_component<L>(L::dir(i));
    constexpr int r = halo_rank<L>(i);
    if constexpr (vl < 0) {
      if (lo) a.hsend[0][(uint64_t)r * a.hplane + pc] = (T)post[i];
    } else if constexpr (vl > 0) {
      if (hi) a.hsend[1][(uint64_t)r * a.hplane + pc] = (T)post[i];
    }
  });
}

// Pull of all populations of a cell whose neighbours need no face rule or
// bounce-back: offsets to the x-1 / x+1 (etc.) neighbours, with wrap-around
// on periodic axes.  kNt: rows are whole 64-cell tiles (nx a multiple of
// 64), so each wavefront's cells are one aligned row segment, and the
// populations with no x velocity are loaded with the non-temporal hint.
template <class L, class S, bool kNt>
__device__ __forceinline__ void pull_periodic(const SweepArgs<S>& a, uint32_t c, uint32_t x,
                                              uint32_t y, uint32_t z,
                                              typename S::T raw[L::Q]) {
  const uint64_t P = a.pstride;
  const int32_t nx = (int32_t)a.nx, nxy = (int32_t)(a.nx * a.ny);
  const int32_t ox_m = x == 0 ? nx - 1 : -1;
  const int32_t ox_p = x == a.nx - 1 ? -(nx - 1) : 1;
  const int32_t oy_m = y == 0 ? (int32_t)(a.ny - 1) * nx : -nx;
  const int32_t oy_p = y == a.ny - 1 ? -(int32_t)(a.ny - 1) * nx : nx;
  int32_t oz_m = 0, oz_p = 0;
  if constexpr (L::D == 3) {
    oz_m = z == 0 ? (int32_t)(a.nz - 1) * nxy : -nxy;
    oz_p = z == a.nz - 1 ? -(int32_t)(a.nz - 1) * nxy : nxy;
  }
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Dir v = L::dir(i);
    int32_t off = 0;
    if constexpr (v.x > 0) off += ox_m;
    if constexpr (v.x < 0) off += ox_p;
    if constexpr (v.y > 0) off += oy_m;
    if constexpr (v.y < 0) off += oy_p;
    if constexpr (v.z > 0) off += oz_m;
    if constexpr (v.z < 0) off += oz_p;
    // With aligned rows, a population with no x velocity comes from a row
    // segment aligned with this wavefront's cells, whose lines no other
    // wavefront reads; the non-temporal hint keeps those lines from
    // displacing the ones at the segment ends of the other populations,
    // which the neighbouring wavefront reads too (1 % faster on D3Q19 FP32
    // 256^3, 6 % on D2Q9 2048 x 1024; with the hint on every population,
    // no faster; on unaligned rows, where wavefronts share those lines
    // too, 3 % slower).  A template choice, not a branch: the compiler
    // merges identical loads on the two sides of a branch and drops the
    // hint.
    if constexpr (kNt && v.x == 0)
      raw[i] = load_pop_nt(a.src + (uint64_t)i * P, (uint32_t)((int32_t)c + off));
    else
      raw[i] = load_pop(a.src + (uint64_t)i * P, (uint32_t)((int32_t)c + off));
  });
}

// Refinement records of one cell's pre-collision moments: on the parent
// side the nodes on the child box's boundary planes, on the child side the
// band its parent's IMPORT nodes filter.
template <class L, class S>
__device__ __forceinline__ void record_moments(const SweepArgs<S>& a,
                                               const CellMoments<typename S::R>& mo,
                                               uint32_t x, uint32_t y, uint32_t z, uint32_t c) {
  const int64_t r =
      a.rec ? record_index<L::D>(a.rec_off, a.rec_dim, a.box_lo, a.box_hi, x, y, z) : -1;
  if (r >= 0) {
    // ten contiguous values per node (read together by the RING fill)
    typename S::R* rr = a.rec + (uint64_t)r * 10;
    rr[0] = mo.drho;
#pragma unroll
    for (int k = 0; k < 3; ++k) rr[1 + k] = mo.u[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) rr[4 + k] = mo.a2[k];
  }
  if (a.recf && in_import_band<L::D>(x, y, z, a.nx, a.ny, a.nz)) {
    // ten contiguous values per node: the IMPORT filter reads a node's
    // stress components together
    typename S::R* rc = a.recf + (uint64_t)c * 10;
    rc[0] = mo.drho;
#pragma unroll
    for (int k = 0; k < 3; ++k) rc[1 + k] = mo.u[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) rc[4 + k] = mo.a2[k];
  }
}

// Interpolation points and weights of a child node coordinate k along one
// axis (the child box starts at parent coordinate lo): a coincident node
// copies its parent node; a midpoint takes the local cubic (-1, 9, 9, -1)/16.
__device__ __forceinline__ int axis_points(int32_t lo, uint32_t k, int32_t pts[4],
                                           float wts[4]) {
  if ((k & 1u) == 0) {
    pts[0] = lo + (int32_t)(k >> 1);
    wts[0] = 1.0f;
    return 1;
  }
  const int32_t j = lo + (int32_t)(k >> 1);
  pts[0] = j - 1;
  pts[1] = j;
  pts[2] = j + 1;
  pts[3] = j + 2;
  wts[0] = -1.0f / 16.0f;
  wts[1] = 9.0f / 16.0f;
  wts[2] = 9.0f / 16.0f;
  wts[3] = -1.0f / 16.0f;
  return 4;
}

// RING node state (eq. couplingFC): interpolated rho~, u~, Pi~_neq (cubic
// in space, linear in time: wa Ma + wb Mb of the parent's two recorded
// time levels), Pi_neq rescaled by alpha_cf = tau_f / (2 tau_c), then
// f = f^{eqH}(rho~, u~) + (1 - 1/tau_f) f^{neqH}(alpha_cf Pi~_neq, u~),
// encoded for storage.  k: the node's coordinates on the child level.
template <class L, class S>
__device__ __forceinline__ void ring_node(const typename S::R* Ma, const typename S::R* Mb,
                                          typename S::R wa, typename S::R wb,
                                          typename S::R alpha, typename S::R omega1,
                                          typename S::R rho0, const int32_t lo[3],
                                          const int32_t rec_off[3], const uint32_t rec_dim[3],
                                          const uint32_t k[3], typename S::T vals[L::Q]) {
  using R = typename S::R;
  int32_t pts[3][4];
  float wts[3][4];
  int np[3];
  for (int ax = 0; ax < 3; ++ax) {
    if (ax < L::D) {
      np[ax] = axis_points(lo[ax], k[ax], pts[ax], wts[ax]);
    } else {
      np[ax] = 1;
      pts[ax][0] = rec_off[ax];
      wts[ax][0] = 1.0f;
    }
  }
  R m[10];
  for (int q = 0; q < 10; ++q) m[q] = (R)0;
  for (int i2 = 0; i2 < np[2]; ++i2)
    for (int i1 = 0; i1 < np[1]; ++i1)
      for (int i0 = 0; i0 < np[0]; ++i0) {
        const uint64_t r =
            ((uint64_t)(pts[2][i2] - rec_off[2]) * rec_dim[1] +
             (uint64_t)(pts[1][i1] - rec_off[1])) * rec_dim[0] +
            (uint64_t)(pts[0][i0] - rec_off[0]);
        const R w = (R)wts[0][i0] * (R)wts[1][i1] * (R)wts[2][i2];
        for (int q = 0; q < 10; ++q) {
          const uint64_t o = r * 10 + (uint64_t)q;
          m[q] += w * (wa * Ma[o] + wb * Mb[o]);
        }
      }
  R u[3] = {m[1], m[2], L::D == 3 ? m[3] : (R)0};
  R a2[6];
  for (int q = 0; q < 6; ++q) a2[q] = alpha * m[4 + q];
  if (L::D == 2) a2[2] = a2[4] = a2[5] = (R)0;
  R out[L::Q];
  rebuild_state<L, R>(m[0], rho0, u, a2, omega1, out);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) vals[i] = encode<S>(out[i], (R)L::w(i) * rho0);
}

// ------------------------------------------------------------------------
// The sweep: pull-stream + (sponge) + regularized collision + store.
// kGeneral = false: every face periodic (or a halo face of the last axis),
// no mask, no sponge.  The solo and
// the batched sweeps share this code, halo faces included (the batch never
// has any): one instantiation keeps their results bitwise equal.
// ------------------------------------------------------------------------
template <class L, class S, bool kGeneral, bool kNt = false>
__device__ __forceinline__ void sweep_cell(const SweepArgs<S>& a, uint32_t c) {
  using R = typename S::R;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const uint32_t row = fast_div(c, a.div_nx);
  const uint32_t x = c - row * a.nx;
  const uint32_t z = fast_div(row, a.div_ny);
  const uint32_t y = row - z * a.ny;
  const uint64_t P = a.pstride;
  // the rebuilt values are produced directly in the storage domain
  const R base = S::kShifted ? (R)0 : a.rho0;

  T raw[Q];
  R post[Q];
  R rho, drho, j[3], Pm[6];
  if constexpr (!kGeneral) {
    pull_periodic<L, S, kNt>(a, c, x, y, z, raw);
    if (a.hrecv[0] || a.hrecv[1]) halo_pull_periodic<L, S>(a, x, y, z, raw);
    stored_moments<L, S>(raw, a.rho0, drho, j, Pm);
    if constexpr (L::kColl == kCollBGK)
      rho = collide_bgk<L, S>(raw, drho, j, a.omega1, a.rho0, (R)0, a.rho_ref, a.uref, post);
    else if constexpr (L::kColl == kCollMRT)
      rho = collide_mrt<L, S>(raw, drho, j, a.omega1, a.rho0, post);
    else
      rho = collide_moments<L, R, false>(drho, j, Pm, a.omega1, a.rho0, (R)0, a.rho_ref,
                                         a.uref, base, post);
  } else {
    // a plain tile (wave-uniform, read through the scalar cache) needs no
    // mask; otherwise the interior pull is issued before the mask decides:
    // its addresses are valid for every cell, and the loads overlap the
    // mask's latency
    const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane(c) >> 6;
    const bool plain = a.tiles && a.tiles[tile];
    uint8_t m = kFluid;  // (every level on this path carries a mask)
    if (!plain) m = a.mask ? a.mask[c] : kFluid;
    pull_periodic<L, S, kNt>(a, c, x, y, z, raw);
    const uint8_t kind = m & kKindBits;
    if (kind == kRing && a.ring_Ma) {
      // a RING node of this (child) level: the coarse-to-fine fill for the
      // state this sweep produces, written here so that its stores join the
      // sweep's own instead of a separate scattered pass
      const uint32_t k[3] = {x, y, z};
      T vals[Q];
      ring_node<L, S>(a.ring_Ma, a.ring_Mb, a.ring_wa, a.ring_wb, a.ring_alpha, a.omega1,
                      a.rho0, a.ring_lo, a.ring_off, a.ring_dim, k, vals);
      static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        store_pop_nt(a.dst + (uint64_t)i * P, (uint32_t)(P * sizeof(T)), c, vals[i]);
      });
      return;
    }
    if (kind == kSolid || kind >= kCovered) return;
    // one rebuild for every kind of cell keeps the kernel's code compact
    // (the comparators collide without it)
    Coeffs<L, R> cf;
    bool rebuild = true;
    if (kind == kInlet) {
      // f^{eqH}(rho0, U u_dir (1 + noise r)), r from SplitMix64
      R u[3];
      const uint64_t bidx =
          ((a.t_new * (uint64_t)a.lstride + (uint64_t)a.level) * (uint64_t)a.ncell + c) * 3ull;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R r = (R)splitmix_pm1(a.seed, bidx + (uint64_t)k);
        u[k] = a.uin[k] * ((R)1 + a.noise * r);
      }
      if (L::D == 2) u[2] = (R)0;
      const R zero6[6] = {(R)0, (R)0, (R)0, (R)0, (R)0, (R)0};
      state_coeffs<L, R>((R)0, a.rho0, u, zero6, (R)0, cf);
      rho = a.rho0;
    } else {
      if (m & (kNearFace | kNearSolid))
        pull_fixup<L, S>(a, x, y, z, c, (m & kNearSolid) != 0, raw);
      stored_moments<L, S>(raw, a.rho0, drho, j, Pm);
      R chi = (R)0, rref = a.rho_ref, uref[3] = {a.uref[0], a.uref[1], a.uref[2]};
      if (m & kFieldSponge) {
        chi = a.sp[c];
        rref = a.sp[a.ncell + c];
#pragma unroll
        for (int k = 0; k < 3; ++k) uref[k] = a.sp[(uint64_t)(2 + k) * a.ncell + c];
      } else if (a.chi_max != (R)0) {
        chi = sponge_chi<R>(a.sponge, a.chi_max, x, y, z, a.nx, a.ny, a.nz);
      }
      if constexpr (L::kColl == kCollBGK) {
        rho = collide_bgk<L, S>(raw, drho, j, a.omega1, a.rho0, chi, rref, uref, post);
        rebuild = false;
      } else if constexpr (L::kColl == kCollMRT) {
        rho = collide_mrt<L, S>(raw, drho, j, a.omega1, a.rho0, post);
        rebuild = false;
      } else {
        // (the moments are always returned in registers; a conditional
        // pointer here would push them to scratch memory)
        CellMoments<R> mo;
        rho = collide_coeffs<L, R, true>(drho, j, Pm, a.omega1, a.rho0, chi, rref, uref, cf,
                                         &mo);
        if (a.rec || a.recf) record_moments<L, S>(a, mo, x, y, z, c);
      }
    }
    if (rebuild) rebuild_from<L, R>(cf, base, post);
  }
  // stability watchdog: a rare, benign racy store of 1
  if (!(rho > (R)0) || !(rho < (R)1e30)) a.status[0] = 1;
  {
    const uint32_t zl = L::D == 3 ? z : y, nl = L::D == 3 ? a.nz : a.ny;
    if ((zl == 0 && a.hsend[0]) || (zl + 1 == nl && a.hsend[1]))
      halo_pack<L, S>(a, c, zl, nl, post);
  }
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    store_pop_nt(a.dst + (uint64_t)i * P, (uint32_t)(P * sizeof(T)), c, (T)post[i]);
  });
}

// Wavefronts per SIMD the sweep is compiled for: 8 for the 4- and 2-byte
// formats (the HBM stream needs them; without the hint the general path's
// scalar registers alone would limit it to 7), except the D3Q27 general
// path, whose 27 pulled values need more than the 64 registers 8 waves
// leave (7 waves, no spills), and the D3Q27 comparator collisions on either
// path, which keep the 27 pulled values alive through the rebuild (7 waves:
// with 64 registers the LBM-BGK sweep spilled 3.5 KB per lane); no
// constraint for FP64.
template <class L, class S, bool kGeneral>
struct SweepWaves {
  static constexpr int value =
      sizeof(typename S::T) == 8
          ? 1
          : (L::Q == 27 && (kGeneral || L::kColl != kCollRR) ? 7 : 8);
};

template <class L, class S, bool kGeneral, bool kNt>
__global__ void __launch_bounds__(1024)
    __attribute__((amdgpu_waves_per_eu(SweepWaves<L, S, kGeneral>::value)))
    k_sweep(const SweepArgs<S> a) {
  // The hardware deals workgroups round-robin to the eight XCDs, so all
  // XCDs stream through neighbouring tiles at the same time (measured faster
  // than giving each XCD a contiguous eighth of the grid).  A pull reads
  // the 128-byte lines at a tile's ends together with the neighbouring
  // tile; with tiles shorter than 256 cells, runs of xcd_group consecutive
  // tiles (256 cells) go to one XCD so that its L2 fetches those lines
  // once: workgroup b of each block of 8 xcd_group workgroups takes tile
  // (b mod 8) xcd_group + (b div 8) of that block (the tail keeps b).
  uint32_t tile = blockIdx.x;
  const uint32_t G = a.xcd_group, span = 8u * G;
  if (G > 1 && tile < gridDim.x / span * span) {
    const uint32_t k = tile % span;
    tile = tile - k + (k % 8u) * G + k / 8u;
  }
  const uint32_t c = tile * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  sweep_cell<L, S, kGeneral, kNt>(a, c);
}

// ------------------------------------------------------------------------
// Initial state: f* = f^{eqH}(rho, u) + (1 - 1/tau) f^{neqH}(pi_neq, u),
// written to both population buffers.
// ------------------------------------------------------------------------
template <class L, class S>
__global__ void k_init(InitArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const double rho = a.rho ? a.rho[c] : a.rho0;
  R u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = (R)(a.u ? a.u[(uint64_t)k * a.ncell + c] : a.uin[k]);
  R p[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = (R)(a.pineq ? a.pineq[(uint64_t)k * a.ncell + c] : 0.0);
  if (L::D == 2) {
    u[2] = (R)0;
    p[2] = p[4] = p[5] = (R)0;
  }
  R out[L::Q];
  rebuild_state<L, R>((R)(rho - a.rho0), (R)a.rho0, u, p, (R)a.omega1, out);
  T* d0 = (T*)a.dst0;
  T* d1 = (T*)a.dst1;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const R wr = (R)L::w(i) * (R)a.rho0;
    const T v = encode<S>(out[i], wr);
    d0[(uint64_t)i * a.pstride + c] = v;
    d1[(uint64_t)i * a.pstride + c] = v;
  }
  if (a.mask_out) a.mask_out[c] = a.mask_in ? a.mask_in[c] : kFluid;
}

// ------------------------------------------------------------------------
// Moments of the stored state: rho = sum f, u = sum f xi / rho.
// ------------------------------------------------------------------------
template <class L, class S>
__global__ void k_moments(MomentArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const T* src = (const T*)a.src;
  if (a.mask && ((a.mask[c] & kKindBits) == kSolid || (a.mask[c] & kKindBits) == kCovered)) {
    if (a.rho_out) a.rho_out[c] = 0.0;
    if (a.u_out)
      for (int k = 0; k < 3; ++k) a.u_out[(uint64_t)k * a.ncell + c] = 0.0;
    return;
  }
  R drho = (R)0, j[3] = {(R)0, (R)0, (R)0};
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Dir v = L::dir(i);
    const R h = decode<S>(src[(uint64_t)i * a.pstride + c], (R)L::w(i) * (R)a.rho0);
    drho += h;
    if constexpr (v.x != 0) j[0] += (R)v.x * h;
    if constexpr (v.y != 0) j[1] += (R)v.y * h;
    if constexpr (v.z != 0) j[2] += (R)v.z * h;
  });
  const double rho = a.rho0 + (double)drho;
  if (a.rho_out) a.rho_out[c] = rho;
  if (a.u_out)
    for (int k = 0; k < 3; ++k) a.u_out[(uint64_t)k * a.ncell + c] = (double)j[k] / rho;
}

// Running sums of the density deviation x = rho - rho0 of the stored state
// and of its square, for temporal means and rms fluctuations (SOLID and
// COVERED cells add 0).
template <class L, class S>
__global__ void k_accum(AccumArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  if (a.mask && ((a.mask[c] & kKindBits) == kSolid || (a.mask[c] & kKindBits) == kCovered))
    return;
  const T* src = (const T*)a.src;
  R drho = (R)0;
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    drho += decode<S>(src[(uint64_t)i * a.pstride + c], (R)L::w(i) * (R)a.rho0);
  });
  const double x = (double)drho;
  if (a.sum1) a.sum1[c] += x;
  if (a.sum2) a.sum2[c] += x * x;
}

template <class L, class S>
__global__ void k_probe(ProbeArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n) return;
  const int64_t c = a.cells[n];
  if (c < 0 || c >= (int64_t)a.ncell) {
    a.rho_out[n] = 0.0;
    return;
  }
  if (a.mask && ((a.mask[c] & kKindBits) == kSolid || (a.mask[c] & kKindBits) == kCovered)) {
    a.rho_out[n] = 0.0;
    return;
  }
  const T* src = (const T*)a.src;
  R drho = (R)0;
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    drho += decode<S>(src[(uint64_t)i * a.pstride + c], (R)L::w(i) * (R)a.rho0);
  });
  a.rho_out[n] = a.rho0 + (double)drho;
}

// Force on the SOLID cells by momentum exchange (Ladd; Mei et al. 2002):
// for every link of a FLUID cell whose pulled source (under the face rules,
// as in the sweep's pull) is SOLID, the post-collision population f*_j moving
// into the wall (xi_j = -xi_i) returns reversed, so the wall receives
// 2 f*_j xi_j.
template <class L, class S>
__global__ void __launch_bounds__(kRedThreads) k_force(ReduceArgs a) {
  using T = typename S::T;
  double F[3] = {0.0, 0.0, 0.0};
  const uint32_t n = a.nx * a.ny * a.nz;
  const T* src = (const T*)a.src;
  const int32_t dims[3] = {(int32_t)a.nx, (int32_t)a.ny, (int32_t)a.nz};
  if (a.mask) {
    for (uint32_t c = blockIdx.x * kRedThreads + threadIdx.x; c < n;
         c += kRedBlocks * kRedThreads) {
      const uint8_t m = a.mask[c];
      if ((m & kKindBits) != kFluid || !(m & (kNearSolid | kNearFace))) continue;
      const int32_t p[3] = {(int32_t)(c % a.nx), (int32_t)((c / a.nx) % a.ny),
                            (int32_t)(c / (a.nx * a.ny))};
      static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Dir v = L::dir(i);
        int32_t s[3] = {p[0] - v.x, p[1] - v.y, p[2] - v.z};
#pragma unroll
        for (int ax = 0; ax < L::D; ++ax) {
          if (s[ax] >= 0 && s[ax] < dims[ax]) continue;
          const bool hi = s[ax] >= dims[ax];
          if (a.face[2 * ax + (hi ? 1 : 0)] == kPeriodic)
            s[ax] = hi ? s[ax] - dims[ax] : s[ax] + dims[ax];
          else
            s[ax] = hi ? dims[ax] - 1 : 0;
        }
        const uint32_t sc = ((uint32_t)s[2] * a.ny + (uint32_t)s[1]) * a.nx + (uint32_t)s[0];
        if ((a.mask[sc] & kKindBits) == kSolid) {
          constexpr int o = opposite<L>(i);
          constexpr Dir w = L::dir(o);
          const T raw = src[(uint64_t)o * a.pstride + c];
          const double f = S::kShifted ? (double)raw + L::w(o) * a.rho0 : (double)raw;
          if constexpr (w.x != 0) F[0] += 2.0 * w.x * f;
          if constexpr (w.y != 0) F[1] += 2.0 * w.y * f;
          if constexpr (w.z != 0) F[2] += 2.0 * w.z * f;
        }
      });
    }
  }
  block_partial<3>(F, a.partial);
}

// Totals of the stored state over the updated cells (every kind but SOLID
// and COVERED): sum of rho - rho0 and of the momentum j = sum f xi.
template <class L, class S>
__global__ void __launch_bounds__(kRedThreads) k_totals(ReduceArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const uint32_t n = a.nx * a.ny * a.nz;
  const T* src = (const T*)a.src;
  for (uint32_t c = blockIdx.x * kRedThreads + threadIdx.x; c < n;
       c += kRedBlocks * kRedThreads) {
    if (a.mask) {
      const uint8_t k = a.mask[c] & kKindBits;
      if (k == kSolid || k == kCovered) continue;
    }
    R drho = (R)0, j[3] = {(R)0, (R)0, (R)0};
    static_for<0, L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr Dir v = L::dir(i);
      const R h = decode<S>(src[(uint64_t)i * a.pstride + c], (R)L::w(i) * (R)a.rho0);
      drho += h;
      if constexpr (v.x != 0) j[0] += (R)v.x * h;
      if constexpr (v.y != 0) j[1] += (R)v.y * h;
      if constexpr (v.z != 0) j[2] += (R)v.z * h;
    });
    acc[0] += (double)drho;
    for (int k = 0; k < 3; ++k) acc[k + 1] += (double)j[k];
  }
  block_partial<4>(acc, a.partial);
}

// canonical FP64 [q][N] <-> native storage
template <class L, class S>
__global__ void k_get_pop(PopArgs a) {
  using T = typename S::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const T* src = (const T*)a.native;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double v = (double)src[(uint64_t)i * a.pstride + c];
    a.canon[(uint64_t)i * a.ncell + c] = S::kShifted ? v + L::w(i) * a.rho0 : v;
  }
}

template <class L, class S>
__global__ void k_set_pop(PopArgs a) {
  using T = typename S::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  T* dst = (T*)a.native;
  T* dst2 = (T*)a.native2;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double f = a.canon[(uint64_t)i * a.ncell + c];
    const T v = (T)(S::kShifted ? f - L::w(i) * a.rho0 : f);
    dst[(uint64_t)i * a.pstride + c] = v;
    if (dst2) dst2[(uint64_t)i * a.pstride + c] = v;
  }
}

// ------------------------------------------------------------------------
// Persistent batched sweep (serving): a fixed grid walks the (job, tile)
// work list of every resident context; the step index comes from device
// memory plus the launch's offset s_off (a captured sequence of launches
// carries offsets 0, 1, ... and advances the base once at its end), so the
// sequence replays for any job table.
// Each cell runs the same sweep_cell instantiation as a solo launch of its
// context, so results are bitwise those of lbm_step.
// ------------------------------------------------------------------------
template <class L, class S, bool kGeneral>
__device__ __forceinline__ void batch_cell(const BatchJob& J, int32_t s, uint32_t c) {
  SweepArgs<S> a = to_args_dev<S>(J.h);
  const int p = (J.cur0 + s) & 1;
  a.src = (const typename S::T*)J.buf[p];
  a.dst = (typename S::T*)J.buf[p ^ 1];
  a.t_new = J.t0 + (uint64_t)s + 1ull;
  a.ncell = J.h.nx * J.h.ny * J.h.nz;
  a.div_nx = FastDiv{J.div_nx[0], J.div_nx[1], J.div_nx[2]};
  a.div_ny = FastDiv{J.div_ny[0], J.div_ny[1], J.div_ny[2]};
  sweep_cell<L, S, kGeneral>(a, c);
}

// Wavefronts per SIMD of the batched sweep: those of the solo sweep, one
// fewer on the 3D general path, where the job lookup's registers on top of
// the sweep's made 8 (D3Q19) and 7 (D3Q27) waves spill.
template <class L, class S, bool kGeneral>
struct BatchWaves {
  static constexpr int value =
      L::D == 3 && kGeneral && sizeof(typename S::T) < 8 ? SweepWaves<L, S, kGeneral>::value - 1
                                                         : SweepWaves<L, S, kGeneral>::value;
};

// One kernel per (lattice, storage, path): the contexts of a batch are
// grouped so, which keeps each kernel as lean as the solo sweep.
template <class L, class S, bool kGeneral>
__global__ void __launch_bounds__(1024)
    __attribute__((amdgpu_waves_per_eu(BatchWaves<L, S, kGeneral>::value)))
    k_batch(const BatchJob* __restrict__ jobs, const BatchHeader* __restrict__ hdr,
            int32_t s_off) {
  const int32_t s = hdr->step + s_off;
  const uint32_t njobs = hdr->njobs, total = hdr->total_tiles;
  uint32_t lo = 0;  // job of the previous tile: this workgroup's tiles increase
  for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    // last job whose first tile is <= tile: usually the previous tile's job
    // (one table read), else a binary search over the jobs after it
    if (lo + 1 < njobs && jobs[lo + 1].tile_begin <= tile) {
      uint32_t hi = njobs;
      ++lo;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].tile_begin <= tile) lo = mid; else hi = mid;
      }
    }
    const BatchJob& J = jobs[lo];
    if ((int64_t)s >= J.steps) continue;
    const uint32_t c = (tile - J.tile_begin) * blockDim.x + threadIdx.x;
    if (c >= J.h.nx * J.h.ny * J.h.nz) continue;
    batch_cell<L, S, kGeneral>(J, s, c);
  }
}

__global__ void k_batch_bump(BatchHeader* hdr, int32_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->step += by;
}

// Flag bits of every cell's mask byte: kNearSolid if a neighbour reached
// by the pull is SOLID (after periodic wrap), kNearFace if the cell lies on a
// face whose rule is not periodic.
template <class L>
__global__ void k_flags(FlagsArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = a.nx * a.ny * a.nz;
  if (c >= n) return;
  const int32_t p[3] = {(int32_t)(c % a.nx), (int32_t)((c / a.nx) % a.ny),
                        (int32_t)(c / (a.nx * a.ny))};
  const int32_t dims[3] = {(int32_t)a.nx, (int32_t)a.ny, (int32_t)a.nz};
  uint8_t flags = 0;
  for (int ax = 0; ax < L::D; ++ax)
    if ((p[ax] == 0 && a.face[2 * ax] != kPeriodic) ||
        (p[ax] == dims[ax] - 1 && a.face[2 * ax + 1] != kPeriodic))
      flags |= kNearFace;
  // sources mapped as the pull maps them: periodic wrap, or the face row
  // for the other rules
  for (int i = 1; i < L::Q; ++i) {
    const Dir v = L::dir(i);
    int32_t s[3] = {p[0] - v.x, p[1] - v.y, p[2] - v.z};
    for (int ax = 0; ax < 3; ++ax) {
      if (s[ax] < 0 || s[ax] >= dims[ax]) {
        if (a.face[2 * ax] == kPeriodic)
          s[ax] = (s[ax] + dims[ax]) % dims[ax];
        else
          s[ax] = s[ax] < 0 ? 0 : dims[ax] - 1;
      }
    }
    if ((a.mask[((uint32_t)s[2] * a.ny + (uint32_t)s[1]) * a.nx + (uint32_t)s[0]] & kKindBits) ==
        kSolid)
      flags |= kNearSolid;
  }
  a.mask[c] = (uint8_t)((a.mask[c] & kKindBits) | flags);
}

// Absorbing layer given per cell: convert to the compute type and flag the
// cells with chi > 0 (the flag is cleared elsewhere).
template <class R>
__global__ void k_set_sponge(SpongeArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  R* sp = (R*)a.sp;
  const double chi = a.chi[c];
  sp[c] = (R)chi;
  sp[a.n + c] = (R)(a.rho_ref ? a.rho_ref[c] : a.rho_ref0);
  for (int k = 0; k < 3; ++k)
    sp[(uint64_t)(2 + k) * a.n + c] =
        (R)(a.u_ref ? a.u_ref[(uint64_t)k * a.n + c] : a.u_ref0[k]);
  const uint8_t m = a.mask[c];
  a.mask[c] = chi > 0.0 ? (uint8_t)(m | kFieldSponge) : (uint8_t)(m & ~kFieldSponge);
}

hipError_t launch_set_sponge(int storage, const SpongeArgs& a, hipStream_t st) {
  const uint32_t blocks = (a.n + 255) / 256;
  if (storage == 0)
    hipLaunchKernelGGL(k_set_sponge<double>, dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_set_sponge<float>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Tile summary: tiles[t] = 1 when the 64 cells [64 t, 64 t + 64) (those
// that exist) are all FLUID without flags.
__global__ void k_tiles(FlagsArgs a) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = a.nx * a.ny * a.nz;
  const uint32_t c0 = t * 64u;
  if (c0 >= n) return;
  const uint32_t c1 = c0 + 64u < n ? c0 + 64u : n;
  uint8_t plain = 1;
  for (uint32_t c = c0; c < c1; ++c)
    if (a.mask[c] != kFluid) plain = 0;
  a.tiles[t] = plain;
}

// Halo faces outside the sweep (after initialisation or an import of
// populations): the face planes' leaving populations into the send
// buffers, as the sweep packs them, and, with `entering`, the same planes'
// entering populations into the receive buffers (the face behaves as a
// zero-gradient face until the first exchange).
template <class L, class S>
__global__ void k_halo_pack(HaloArgs h) {
  using T = typename S::T;
  const uint32_t pc = blockIdx.x * blockDim.x + threadIdx.x;
  if (pc >= h.hplane) return;
  const T* src = (const T*)h.src;
  const uint32_t nl = L::D == 3 ? h.nz : h.ny;
  for (int side = 0; side < 2; ++side) {
    if (!h.hsend[side]) continue;
    const uint32_t zl = side ? nl - 1 : 0;
    const uint64_t c = (uint64_t)zl * h.hplane + pc;
    T* send = (T*)h.hsend[side];
    T* recv = (T*)h.hrecv[side];
    static_for<1, L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int vl = last_component<L>(L::dir(i));
      const T v = src[(uint64_t)i * h.pstride + c];
      const uint64_t o = (uint64_t)halo_rank<L>(i) * h.hplane + pc;
      if (vl == (side ? 1 : -1)) send[o] = v;
      if (h.entering && vl == (side ? -1 : 1)) recv[o] = v;
    });
  }
}

template <class L>
static void halo_pack_l(int storage, const HaloArgs& a, hipStream_t st) {
  const uint32_t blocks = (a.hplane + 255) / 256;
  switch (storage) {
    case 0: hipLaunchKernelGGL((k_halo_pack<L, StoreF64>), dim3(blocks), dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_halo_pack<L, StoreF32>), dim3(blocks), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_halo_pack<L, StoreF32S>), dim3(blocks), dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_halo_pack<L, StoreF16S>), dim3(blocks), dim3(256), 0, st, a); break;
  }
}

hipError_t launch_halo_pack(int lattice, int storage, const HaloArgs& a, hipStream_t st) {
  switch (lattice) {
    case 9: halo_pack_l<Lattice<9>>(storage, a, st); break;
    case 19: halo_pack_l<Lattice<19>>(storage, a, st); break;
    case 27: halo_pack_l<Lattice<27>>(storage, a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int halo_count_of(int lattice) {
  switch (lattice) {
    case 9: return halo_count<Lattice<9>>();
    case 19: return halo_count<Lattice<19>>();
    case 27: return halo_count<Lattice<27>>();
  }
  return 0;
}

// ------------------------------------------------------------------------
// Two-level refinement kernels (Sec. II.B)
// ------------------------------------------------------------------------
__global__ void k_roles(RolesArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = a.nx * a.ny * a.nz;
  if (c >= n) return;
  const uint32_t p[3] = {c % a.nx, (c / a.nx) % a.ny, c / (a.nx * a.ny)};
  const uint32_t dims[3] = {a.nx, a.ny, a.nz};
  if (a.child) {
    bool inside = true, deep = true;
    for (int ax = 0; ax < a.dim; ++ax) {
      const int32_t v = (int32_t)p[ax];
      if (v < a.lo[ax] + 1 || v > a.hi[ax] - 1) inside = false;
      if (v < a.lo[ax] + 2 || v > a.hi[ax] - 2) deep = false;
    }
    if (inside) a.mask[c] = deep ? kCovered : kImport;
  }
  if (a.ring) {
    bool ring = false;
    for (int ax = 0; ax < a.dim; ++ax)
      if (p[ax] == 0 || p[ax] == dims[ax] - 1) ring = true;
    if (ring) a.mask[c] = kRing;
  }
}

// coarse moments at t = 0 taken from the initial fields (NULL fields mean
// rho0, the inlet velocity and zero, as in the initialisation)
template <class L, class S>
__global__ void k_record_fields(RecordFieldsArgs a) {
  using R = typename S::R;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = a.nx * a.ny * a.nz;
  if (c >= n) return;
  const int64_t r = record_index<L::D>(a.rec_off, a.rec_dim, a.box_lo, a.box_hi, c % a.nx,
                                       (c / a.nx) % a.ny, c / (a.nx * a.ny));
  if (r < 0) return;
  R v[10];
  v[0] = (R)((a.rho ? a.rho[c] : a.rho0) - a.rho0);
  for (int k = 0; k < 3; ++k) v[1 + k] = (R)(a.u ? a.u[(uint64_t)k * n + c] : a.uin[k]);
  for (int k = 0; k < 6; ++k) v[4 + k] = (R)(a.pineq ? a.pineq[(uint64_t)k * n + c] : 0.0);
  if (L::D == 2) v[3] = v[6] = v[8] = v[9] = (R)0;
  R* ra = (R*)a.rec_a;
  R* rb = (R*)a.rec_b;
  for (int k = 0; k < 10; ++k) {
    ra[(uint64_t)r * 10 + k] = v[k];
    rb[(uint64_t)r * 10 + k] = v[k];
  }
}

// RING nodes of a child level from a list (the fill after initialisation;
// during stepping the child's sweep rebuilds them itself, see sweep_cell).
template <class L, class S>
__global__ void k_ring(RingArgs a) {
  using R = typename S::R;
  using T = typename S::T;
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n) return;
  const uint32_t cf = a.list[n];
  const uint32_t k[3] = {cf % a.fnx, (cf / a.fnx) % a.fny, cf / (a.fnx * a.fny)};
  T vals[L::Q];
  ring_node<L, S>((const R*)a.Ma, (const R*)a.Mb, (R)a.wa, (R)a.wb, (R)a.alpha, (R)a.omega1,
                  (R)a.rho0, a.lo, a.rec_off, a.rec_dim, k, vals);
  T* dst = (T*)a.dst;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) dst[(uint64_t)i * a.pstride + cf] = vals[i];
}

// IMPORT node state (eq. couplingCF): rho, u of the coincident child node
// and the (1/4, 1/2, 1/4)-filtered Pi_neq of its 3^D child neighbours, all
// pre-collision moments of the child at the common time, recorded by the
// child's last sweep; Pi_neq rescaled by alpha_fc = 2 tau_c / tau_f;
// f = f^{eqH}(rho, u) + (1 - 1/tau_c) f^{neqH}.
template <class L, class S>
__global__ void k_import(ImportArgs ia) {
  using R = typename S::R;
  using T = typename S::T;
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ia.n) return;
  const uint32_t cc = ia.list[n];
  const int32_t p[3] = {(int32_t)(cc % ia.cnx), (int32_t)((cc / ia.cnx) % ia.cny),
                        (int32_t)(cc / (ia.cnx * ia.cny))};
  int32_t kc[3];
  for (int ax = 0; ax < 3; ++ax) kc[ax] = ax < L::D ? 2 * (p[ax] - ia.lo[ax]) : 0;
  const R* M = (const R*)ia.recf;
  const R w1[3] = {(R)0.25, (R)0.5, (R)0.25};
  const int oz = L::D == 3 ? 1 : 0;
  R acc[6] = {(R)0, (R)0, (R)0, (R)0, (R)0, (R)0};
  for (int o2 = -oz; o2 <= oz; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        const uint64_t c = ((uint64_t)(kc[2] + o2) * ia.fny + (uint64_t)(kc[1] + o1)) * ia.fnx +
                           (uint64_t)(kc[0] + o0);
        const R w = w1[o0 + 1] * w1[o1 + 1] * (oz ? w1[o2 + 1] : (R)1);
        for (int q = 0; q < 6; ++q) acc[q] += w * M[c * 10 + 4 + q];
      }
  const uint64_t c0 = ((uint64_t)kc[2] * ia.fny + (uint64_t)kc[1]) * ia.fnx + (uint64_t)kc[0];
  const R drho_c = M[c0 * 10];
  const R u_c[3] = {M[c0 * 10 + 1], M[c0 * 10 + 2], L::D == 3 ? M[c0 * 10 + 3] : (R)0};
  for (int q = 0; q < 6; ++q) acc[q] *= (R)ia.alpha;
  R out[L::Q];
  rebuild_state<L, R>(drho_c, (R)ia.rho0, u_c, acc, (R)ia.omega1, out);
  T* dst = (T*)ia.dst;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    dst[(uint64_t)i * ia.pstride + cc] = encode<S>(out[i], (R)L::w(i) * (R)ia.rho0);
}

// ------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------
template <class S>
static SweepArgs<S> to_args(const SweepHost& h) {
  return to_args_dev<S>(h);
}

template <class S>
__host__ __device__ inline SweepArgs<S> to_args_dev(const SweepHost& h) {
  using T = typename S::T;
  using R = typename S::R;
  SweepArgs<S> a;
  a.src = (const T*)h.src;
  a.dst = (T*)h.dst;
  a.mask = h.mask;
  a.tiles = h.tiles;
  a.status = h.status;
  a.nx = h.nx;
  a.ny = h.ny;
  a.nz = h.nz;
  a.ncell = h.nx * h.ny * h.nz;
  a.pstride = h.pstride;
#if !defined(__HIP_DEVICE_COMPILE__)
  a.div_nx = make_fastdiv(h.nx);
  a.div_ny = make_fastdiv(h.ny);
#endif
  a.omega1 = (R)(1.0 - 1.0 / h.tau);
  a.rho0 = (R)h.rho0;
  a.chi_max = (R)h.chi_max;
  a.rho_ref = (R)h.rho_ref;
  for (int k = 0; k < 3; ++k) {
    a.uref[k] = (R)h.uref[k];
    a.uin[k] = (R)h.uin[k];
  }
  a.noise = (R)h.noise;
  for (int f = 0; f < 6; ++f) {
    a.face[f] = h.face[f];
    a.sponge[f] = h.sponge[f];
  }
  a.seed = h.seed;
  a.t_new = h.t_new;
  a.level = h.level;
  a.lstride = h.lstride;
  a.ntiles = 0;
  a.xcd_group = 1;
  a.rec = (R*)h.rec;
  a.recf = (R*)h.recf;
  a.sp = (const R*)h.sp;
  for (int k = 0; k < 3; ++k) {
    a.rec_off[k] = h.rec_off[k];
    a.rec_dim[k] = h.rec_dim[k];
    a.box_lo[k] = h.box_lo[k];
    a.box_hi[k] = h.box_hi[k];
  }
  a.rec_n = h.rec_n;
  a.ring_Ma = (const R*)h.ring_Ma;
  a.ring_Mb = (const R*)h.ring_Mb;
  a.ring_wa = (R)h.ring_wa;
  a.ring_wb = (R)h.ring_wb;
  a.ring_alpha = (R)h.ring_alpha;
  for (int k = 0; k < 3; ++k) {
    a.ring_lo[k] = h.ring_lo[k];
    a.ring_off[k] = h.ring_off[k];
    a.ring_dim[k] = h.ring_dim[k];
  }
  for (int k = 0; k < 2; ++k) {
    a.hrecv[k] = (const T*)h.hrecv[k];
    a.hsend[k] = (T*)h.hsend[k];
  }
  a.hplane = h.hplane;
  return a;
}

template <class L, class S>
static hipError_t launch_sweep_t(const SweepHost& h, int block, hipStream_t st) {
  SweepArgs<S> a = to_args<S>(h);
  const uint32_t blocks = (a.ncell + block - 1) / block;
  a.ntiles = blocks;
  a.xcd_group = block < 256 ? 256u / (uint32_t)block : 1u;
  // rows of whole 64-cell tiles: the pull with the non-temporal hint
  const bool nt = h.nx % 64u == 0u;
  if (h.general && nt)
    hipLaunchKernelGGL((k_sweep<L, S, true, true>), dim3(blocks), dim3(block), 0, st, a);
  else if (h.general)
    hipLaunchKernelGGL((k_sweep<L, S, true, false>), dim3(blocks), dim3(block), 0, st, a);
  else if (nt)
    hipLaunchKernelGGL((k_sweep<L, S, false, true>), dim3(blocks), dim3(block), 0, st, a);
  else
    hipLaunchKernelGGL((k_sweep<L, S, false, false>), dim3(blocks), dim3(block), 0, st, a);
  return hipGetLastError();
}

template <class L>
static hipError_t launch_sweep_l(const SweepHost& h, int storage, int block,
                                 hipStream_t st) {
  switch (storage) {
    case 0: return launch_sweep_t<L, StoreF64>(h, block, st);
    case 1: return launch_sweep_t<L, StoreF32>(h, block, st);
    case 2: return launch_sweep_t<L, StoreF32S>(h, block, st);
    case 3: return launch_sweep_t<L, StoreF16S>(h, block, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(int lattice, int storage, const SweepHost& h, int block,
                        hipStream_t st) {
  switch (lattice) {
    case 9: return launch_sweep_l<Lattice<9>>(h, storage, block, st);
    case 19: return launch_sweep_l<Lattice<19>>(h, storage, block, st);
    case 27: return launch_sweep_l<Lattice<27>>(h, storage, block, st);
    case kFullOrderCode + 9: return launch_sweep_l<Lattice<9, true>>(h, storage, block, st);
    case kFullOrderCode + 27: return launch_sweep_l<Lattice<27, true>>(h, storage, block, st);
    case kBgkCode + 9: return launch_sweep_l<Lattice<9, false, kCollBGK>>(h, storage, block, st);
    case kBgkCode + 19: return launch_sweep_l<Lattice<19, false, kCollBGK>>(h, storage, block, st);
    case kBgkCode + 27: return launch_sweep_l<Lattice<27, false, kCollBGK>>(h, storage, block, st);
    case kMrtCode + 9: return launch_sweep_l<Lattice<9, false, kCollMRT>>(h, storage, block, st);
  }
  return hipErrorInvalidValue;
}

// dispatch of the companion kernels over lattice and storage
#define HRLBM_DISPATCH(NAME, ARGS, FULL)                                      \
  template <class L, class S>                                                 \
  static void NAME##_t(const ARGS& a, uint32_t n, hipStream_t st) {           \
    const uint32_t blocks = (n + 255) / 256;                                  \
    if (blocks) hipLaunchKernelGGL((k_##NAME<L, S>), dim3(blocks), dim3(256), 0, st, a); \
  }                                                                           \
  template <class L>                                                          \
  static void NAME##_l(int storage, const ARGS& a, uint32_t n, hipStream_t st) { \
    switch (storage) {                                                        \
      case 0: NAME##_t<L, StoreF64>(a, n, st); break;                         \
      case 1: NAME##_t<L, StoreF32>(a, n, st); break;                         \
      case 2: NAME##_t<L, StoreF32S>(a, n, st); break;                        \
      case 3: NAME##_t<L, StoreF16S>(a, n, st); break;                        \
    }                                                                         \
  }                                                                           \
  hipError_t launch_##NAME(int lattice, int storage, const ARGS& a, uint32_t n, \
                           hipStream_t st) {                                  \
    switch (lattice) {                                                        \
      case 9: NAME##_l<Lattice<9>>(storage, a, n, st); break;                 \
      case 19: NAME##_l<Lattice<19>>(storage, a, n, st); break;               \
      case 27: NAME##_l<Lattice<27>>(storage, a, n, st); break;               \
      FULL(NAME)                                                              \
      default: return hipErrorInvalidValue;                                   \
    }                                                                         \
    return hipGetLastError();                                                 \
  }
// extra cases of the kernels that rebuild populations (collision order)
#define HRLBM_FULL_CASES(NAME)                                                   \
  case kFullOrderCode + 9: NAME##_l<Lattice<9, true>>(storage, a, n, st); break; \
  case kFullOrderCode + 27: NAME##_l<Lattice<27, true>>(storage, a, n, st); break;
#define HRLBM_NO_CASES(NAME)

HRLBM_DISPATCH(init, InitArgs, HRLBM_FULL_CASES)
HRLBM_DISPATCH(moments, MomentArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(probe, ProbeArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(accum, AccumArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(get_pop, PopArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(set_pop, PopArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(record_fields, RecordFieldsArgs, HRLBM_NO_CASES)
HRLBM_DISPATCH(ring, RingArgs, HRLBM_FULL_CASES)
HRLBM_DISPATCH(import, ImportArgs, HRLBM_FULL_CASES)

void fill_fastdiv(uint32_t d, uint32_t out[3]) {
  const FastDiv f = make_fastdiv(d);
  out[0] = f.d;
  out[1] = f.m;
  out[2] = f.s;
}

// Batch kernel variants: variant = lattice code * 16 + storage * 2 + general.
template <class L, class S, bool G>
static hipError_t batch_t(bool query, const BatchJob* jobs, BatchHeader* hdr, int32_t s_off,
                          int block, int grid, hipStream_t st, int* per) {
  if (query)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_batch<L, S, G>, block, 0);
  hipLaunchKernelGGL((k_batch<L, S, G>), dim3(grid), dim3(block), 0, st, jobs, hdr, s_off);
  return hipGetLastError();
}

template <class L>
static hipError_t batch_l(int storage, bool general, bool query, const BatchJob* jobs,
                          BatchHeader* hdr, int32_t s_off, int block, int grid, hipStream_t st,
                          int* per) {
#define HRLBM_BATCH(S)                                                            \
  return general ? batch_t<L, S, true>(query, jobs, hdr, s_off, block, grid, st, per)    \
                 : batch_t<L, S, false>(query, jobs, hdr, s_off, block, grid, st, per);
  switch (storage) {
    case 0: HRLBM_BATCH(StoreF64)
    case 1: HRLBM_BATCH(StoreF32)
    case 2: HRLBM_BATCH(StoreF32S)
    case 3: HRLBM_BATCH(StoreF16S)
  }
#undef HRLBM_BATCH
  return hipErrorInvalidValue;
}

static hipError_t batch_dispatch(int variant, bool query, const BatchJob* jobs,
                                 BatchHeader* hdr, int32_t s_off, int block, int grid,
                                 hipStream_t st, int* per) {
  const int lattice = variant / 16, storage = (variant / 2) % 8;
  const bool general = variant & 1;
  switch (lattice) {
    case 9: return batch_l<Lattice<9>>(storage, general, query, jobs, hdr, s_off, block, grid, st, per);
    case 19: return batch_l<Lattice<19>>(storage, general, query, jobs, hdr, s_off, block, grid, st, per);
    case 27: return batch_l<Lattice<27>>(storage, general, query, jobs, hdr, s_off, block, grid, st, per);
    case kFullOrderCode + 9:
      return batch_l<Lattice<9, true>>(storage, general, query, jobs, hdr, s_off, block, grid, st, per);
    case kFullOrderCode + 27:
      return batch_l<Lattice<27, true>>(storage, general, query, jobs, hdr, s_off, block, grid, st, per);
    case kBgkCode + 9:
      return batch_l<Lattice<9, false, kCollBGK>>(storage, general, query, jobs, hdr, s_off, block, grid,
                                                  st, per);
    case kBgkCode + 19:
      return batch_l<Lattice<19, false, kCollBGK>>(storage, general, query, jobs, hdr, s_off, block,
                                                   grid, st, per);
    case kBgkCode + 27:
      return batch_l<Lattice<27, false, kCollBGK>>(storage, general, query, jobs, hdr, s_off, block,
                                                   grid, st, per);
    case kMrtCode + 9:
      return batch_l<Lattice<9, false, kCollMRT>>(storage, general, query, jobs, hdr, s_off, block, grid,
                                                  st, per);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(int variant, const BatchJob* jobs, BatchHeader* hdr, int32_t s_off,
                        int block, int grid, hipStream_t st) {
  return batch_dispatch(variant, false, jobs, hdr, s_off, block, grid, st, nullptr);
}

hipError_t launch_batch_bump(BatchHeader* hdr, int32_t by, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_bump, dim3(1), dim3(64), 0, st, hdr, by);
  return hipGetLastError();
}

int batch_grid(int variant, int block) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (batch_dispatch(variant, true, nullptr, nullptr, 0, block, 0, nullptr, &per) != hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

hipError_t launch_flags(int lattice, const FlagsArgs& a, hipStream_t st) {
  const uint32_t n = a.nx * a.ny * a.nz;
  const uint32_t blocks = (n + 255) / 256;
  switch (lattice) {
    case 9: hipLaunchKernelGGL(k_flags<Lattice<9>>, dim3(blocks), dim3(256), 0, st, a); break;
    case 19: hipLaunchKernelGGL(k_flags<Lattice<19>>, dim3(blocks), dim3(256), 0, st, a); break;
    case 27: hipLaunchKernelGGL(k_flags<Lattice<27>>, dim3(blocks), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.tiles) return e;
  return launch_tiles(a, st);
}

hipError_t launch_tiles(const FlagsArgs& a, hipStream_t st) {
  const uint32_t n = a.nx * a.ny * a.nz;
  const uint32_t ntile = (n + 63) / 64;
  hipLaunchKernelGGL(k_tiles, dim3((ntile + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <class L>
static void reduce_l(bool totals, int storage, const ReduceArgs& a, hipStream_t st) {
  const dim3 g(kRedBlocks), b(kRedThreads);
#define HRLBM_RED(S)                                                          \
  if (totals)                                                                 \
    hipLaunchKernelGGL((k_totals<L, S>), g, b, 0, st, a);                     \
  else                                                                        \
    hipLaunchKernelGGL((k_force<L, S>), g, b, 0, st, a);
  switch (storage) {
    case 0: HRLBM_RED(StoreF64) break;
    case 1: HRLBM_RED(StoreF32) break;
    case 2: HRLBM_RED(StoreF32S) break;
    case 3: HRLBM_RED(StoreF16S) break;
  }
#undef HRLBM_RED
}

static hipError_t launch_reduce(bool totals, int lattice, int storage, const ReduceArgs& a,
                                hipStream_t st) {
  switch (lattice) {
    case 9: reduce_l<Lattice<9>>(totals, storage, a, st); break;
    case 19: reduce_l<Lattice<19>>(totals, storage, a, st); break;
    case 27: reduce_l<Lattice<27>>(totals, storage, a, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (totals)
    hipLaunchKernelGGL(k_reduce_final<4>, dim3(1), dim3(kRedThreads), 0, st, a.partial, a.out);
  else
    hipLaunchKernelGGL(k_reduce_final<3>, dim3(1), dim3(kRedThreads), 0, st, a.partial, a.out);
  return hipGetLastError();
}

hipError_t launch_force(int lattice, int storage, const ReduceArgs& a, hipStream_t st) {
  return launch_reduce(false, lattice, storage, a, st);
}

hipError_t launch_totals(int lattice, int storage, const ReduceArgs& a, hipStream_t st) {
  return launch_reduce(true, lattice, storage, a, st);
}

hipError_t launch_roles(const RolesArgs& a, uint32_t n, hipStream_t st) {
  const uint32_t blocks = (n + 255) / 256;
  if (blocks) hipLaunchKernelGGL(k_roles, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hrlbm
