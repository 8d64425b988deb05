// The state of a fully periodic grid stored as moments (storages LBM_M64
// and LBM_M32), with its own sweep and companion kernels.
//
// Without a sponge the regularized collision (eq. optimizedLB) leaves every
// cell at f*_i = w_i rho0 + w_i H_i(drho, u, a2*): the Hermite expansion of
// eqs. (eqH) and (neqH) whose coefficients all follow from rho, u and the
// post-collision non-equilibrium stress a2* = (1 - 1/tau) a2_neq (the third
// and higher orders by eqs. recursive1 and recursive2, which are linear in
// a2_neq).  A cell's state is therefore ten numbers (drho, u, a2*; six in
// 2D) instead of q populations, and one update moves 2 x 10 values through
// HBM instead of 2 x q.
//
// The sweep marches workgroups through the grid plane by plane (z in 3D,
// y in 2D).  For each plane a workgroup rebuilds the post-collision
// populations of its tile plus a one-cell halo into LDS (each population
// from the plane it streams out of), pulls every interior cell's q
// populations from there, collides, and stores the new moments.  A halo
// cell is rebuilt again by the neighbouring tile, only for the populations
// that tile pulls from it, and its moments are read again (from L2 when
// the neighbour read them recently).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace hrlbm {

// Moments per cell: drho, u_x, u_y, u_z, a2*_xx, yy, zz, xy, xz, yz in 3D;
// drho, u_x, u_y, a2*_xx, yy, xy in 2D.
template <class L>
struct MState {
  static constexpr int NM = L::D == 3 ? 10 : 6;
  // component of the packed 6-vector (xx, yy, zz, xy, xz, yz) stored at
  // slot 1 + D + k, or -1
  static constexpr int a2_slot(int k) {
    return L::D == 3 ? 1 + 3 + k : (k == 0 ? 3 : k == 1 ? 4 : k == 3 ? 5 : -1);
  }
};

// Workgroup tile: TX x TY interior cells of a plane, HX x HY with the
// halo.  3D: TY wavefronts of interior cells (one lane per cell) and three
// halo wavefronts (the two halo rows, then both halo columns with their
// corners); 2D: one thread per halo-row slot (NT >= HX, whole wavefronts).
template <class L, class R>
struct MTile {
  static constexpr int TX = L::D == 3 ? 64 : 254;
  static constexpr int TY = L::D == 3 ? (sizeof(R) == 8 ? 2 : 8) : 1;
  static constexpr int HX = TX + 2;
  static constexpr int HY = L::D == 3 ? TY + 2 : 1;
  static constexpr int SLOTS = HX * HY;
  static constexpr int NT = L::D == 3 ? (TY + 3) * 64 : (SLOTS + 63) / 64 * 64;
  static_assert(L::D == 2 || (TX == 64 && 2 * HY <= 64), "3D halo wavefronts");
  // LDS planes: with two, consecutive iterations alternate and one barrier
  // per plane suffices (measured slower: the doubled LDS halves the
  // workgroups a CU holds)
  static constexpr int NB = 1;
};

// velocity component along the marching axis, and the in-plane LDS offset
template <class L>
constexpr int march_of(int i) {
  return L::D == 3 ? L::dir(i).z : L::dir(i).y;
}
template <class L, int HX>
constexpr int plane_shift(int i) {
  return L::dir(i).x + (L::D == 3 ? L::dir(i).y * HX : 0);
}

// What a thread rebuilds.  kInterior: its own output cell, every
// population (those with no in-plane velocity stay in registers);
// kRowLo / kRowHi: a halo-row cell below / above the tile, only the
// populations with xi_y = +1 / -1 (the only ones an interior cell pulls
// from there); kCols: a halo-column cell, only those with xi_x != 0;
// kAny: one halo-row slot of a 2D row tile, every population.
enum MRole { kAny = -1, kInterior = 0, kRowLo = 1, kRowHi = 2, kCols = 3 };

template <class L, int ROLE>
constexpr bool role_needs(int i) {
  return ROLE == kRowLo   ? L::dir(i).y == 1
         : ROLE == kRowHi ? L::dir(i).y == -1
         : ROLE == kCols  ? L::dir(i).x != 0
                          : true;
}

// populations of its own cell that an interior thread pulls from registers
template <class L, int HX, int ROLE>
constexpr bool in_regs(int i) {
  return ROLE == kInterior && plane_shift<L, HX>(i) == 0;
}

template <class R>
struct MSweepArgs {
  const R* src;
  R* dst;
  int* status;
  uint32_t px, py, pm;  // plane extents (x, y; y = 1 in 2D) and marching extent
  uint32_t tiles_x, tiles_y, zc, nblocks;
  uint32_t xcd_order;   // 1: each XCD walks a contiguous range of tiles
  uint64_t pstride;
  R omega1, rho0;
};

// Moments of one cell (shifted density, velocity, a2*) from the state array.
template <class L, class R>
__device__ __forceinline__ void load_state(const R* src, uint64_t P, uint32_t c,
                                           R m[MState<L>::NM]) {
#pragma unroll
  for (int k = 0; k < MState<L>::NM; ++k) m[k] = load_pop(src + (uint64_t)k * P, c);
}

// Post-collision deviations h_i = f*_i - w_i rho0 of a cell from its moments.
template <class L, class R>
__device__ __forceinline__ void rebuild_cell(const R m[MState<L>::NM], R rho0, R h[L::Q]) {
  const R u[3] = {m[1], m[2], L::D == 3 ? m[3] : (R)0};
  R a2[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = MState<L>::a2_slot(k);
    a2[k] = s >= 0 ? m[s] : (R)0;
  }
  // a2 already carries the factor 1 - 1/tau
  rebuild_state<L, R>(m[0], rho0, u, a2, (R)1, h);
}

// Moments of a cell from its deviations h (pre-collision), collided:
// rho, u conserved, a2* = omega1 a2_neq.  Returns rho.
template <class L, class R>
__device__ __forceinline__ R collide_state(const R h[L::Q], R omega1, R rho0,
                                           R m[MState<L>::NM]) {
  R drho, j[3], P[6];
  raw_moments<L, R>(h, drho, j, P);
  const R rho = rho0 + drho;
  const R irho = recip(rho);
  const R u[3] = {j[0] * irho, j[1] * irho, L::D == 3 ? j[2] * irho : (R)0};
  R a2[6];
  noneq_stress<L, R>(drho, j, u, P, a2);
  m[0] = drho;
  m[1] = u[0];
  m[2] = u[1];
  if constexpr (L::D == 3) m[3] = u[2];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = MState<L>::a2_slot(k);
    if (s >= 0) m[s] = omega1 * a2[k];
  }
  return rho;
}

// One thread's march through planes m0 ... m1 - 1.  Iteration m (output
// plane m) writes, for the thread's slot, the populations that stream into
// plane m: those with a +1 marching component from plane m - 1, 0 from
// plane m, -1 from plane m + 1 (rebuilt from moments loaded one iteration
// ahead); the thread keeps the parts it will write in the next two
// iterations in registers.  After a barrier every interior cell pulls its
// q populations from the slots at x - xi, collides and stores its moments;
// a second barrier protects the LDS plane before it is rewritten.  Every
// thread of a workgroup runs the same number of iterations and barriers.
// The loads are issued for every thread and iteration (threads without a
// slot load a valid cell and write nothing), so they stay in flight across
// the barriers instead of being waited for at a branch.
template <class L, class R, int ROLE>
__device__ __forceinline__ void march(const MSweepArgs<R>& a, R* lds, uint32_t scell,
                                      uint32_t slds, bool sown, uint32_t ocell, uint32_t olds,
                                      bool oown, uint32_t m0, uint32_t m1) {
  using G = MTile<L, R>;
  constexpr int Q = L::Q, NM = MState<L>::NM;
  constexpr bool kCollide = ROLE == kAny || ROLE == kInterior;
  const uint32_t plane = a.px * a.py;
  const uint64_t P = a.pstride;
  auto wrap_m = [&](uint32_t m, int d) -> uint32_t {
    return (m + a.pm + (uint32_t)d) % a.pm;
  };

  // carried parts: up1 = +1 part of plane m - 1, up2 = +1 part of plane m,
  // mid = 0 part of plane m; nxt = moments of plane m + 1.  Two warm-up
  // iterations fill them through the same code as the others (so every
  // plane is rebuilt by the same instructions whatever the chunk length).
  // Populations the role does not need are never used and drop out.
  R up1[Q], up2[Q], mid[Q], nxt[NM];
  load_state<L, R>(a.src, P, wrap_m(m0, -1) * plane + scell, nxt);
  // not unrolled or peeled: a peeled warm-up copy may round differently
#pragma clang loop unroll(disable)
  for (int it = -2; it < (int)(m1 - m0); ++it) {
    R v[Q];
    {
      R h[Q];
      rebuild_cell<L, R>(nxt, a.rho0, h);
      // moments of plane m0 + it + 2 (wrapped: always a valid plane)
      load_state<L, R>(a.src, P, wrap_m(m0, it + 2) * plane + scell, nxt);
      static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (march_of<L>(i) > 0) {
          v[i] = up1[i];
          up1[i] = up2[i];
          up2[i] = h[i];
        } else if constexpr (march_of<L>(i) == 0) {
          v[i] = mid[i];
          mid[i] = h[i];
        } else {
          v[i] = h[i];
        }
      });
    }
    if (it < 0) continue;
    const uint32_t m = m0 + (uint32_t)it;
    R* buf = lds + (G::NB == 2 ? (uint32_t)(it & 1) * (Q * G::SLOTS) : 0u);
    if (sown) {
      static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (role_needs<L, ROLE>(i) && !in_regs<L, G::HX, ROLE>(i)) buf[i * G::SLOTS + slds] = v[i];
      });
    }
    __syncthreads();
    if constexpr (kCollide) {
      if (oown) {
        R h[Q], mo[NM];
        static_for<0, Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (in_regs<L, G::HX, ROLE>(i))
            h[i] = v[i];
          else
            h[i] = buf[i * G::SLOTS + (int)olds - plane_shift<L, G::HX>(i)];
        });
        const R rho = collide_state<L, R>(h, a.omega1, a.rho0, mo);
        // stability watchdog: a rare, benign racy store of 1
        if (!(rho > (R)0) || !(rho < (R)1e30)) a.status[0] = 1;
        const uint32_t c = m * plane + ocell;
#pragma unroll
        for (int k = 0; k < NM; ++k)
          store_pop_nt(a.dst + (uint64_t)k * P, (uint32_t)(P * sizeof(R)), c, mo[k]);
      }
    }
    if constexpr (G::NB == 1) __syncthreads();
  }
}

// ------------------------------------------------------------------------
// The sweep: one workgroup per tile and chunk of planes.  In 3D the
// wavefront index (uniform, read into a scalar register) selects the role,
// so each wavefront runs one specialised march and the halo wavefronts
// rebuild only the populations the interior pulls from them (5 of 19 on
// the rows, 10 of 19 on the columns for D3Q19).
// ------------------------------------------------------------------------
template <class L, class R>
__global__ void __launch_bounds__((MTile<L, R>::NT)) k_msweep(const MSweepArgs<R> a) {
  using G = MTile<L, R>;
  __shared__ R lds_all[G::NB * L::Q * G::SLOTS];

  uint32_t b = blockIdx.x;
  if (a.xcd_order) b = (b % 8u) * (a.nblocks / 8u) + b / 8u;
  const uint32_t bx = b % a.tiles_x;
  const uint32_t r = b / a.tiles_x;
  const uint32_t by = r % a.tiles_y;
  const uint32_t ch = r / a.tiles_y;
  const uint32_t x0 = bx * G::TX, y0 = by * G::TY;
  const uint32_t wx = min((uint32_t)G::TX, a.px - x0);
  const uint32_t wy = L::D == 3 ? min((uint32_t)G::TY, a.py - y0) : 1u;
  const uint32_t m0 = ch * a.zc, m1 = min(a.pm, m0 + a.zc);
  const uint32_t tid = threadIdx.x;

  if constexpr (L::D == 3) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / 64u);
    const uint32_t lane = tid % 64u;
    const uint32_t hy = wy + 2;
    if (wave < (uint32_t)G::TY) {
      // interior: lane = x, wave = y of the output cell, which is also the
      // slot it rebuilds; lanes outside a ragged tile load a valid cell
      const bool own = lane < wx && wave < wy;
      const uint32_t ox = min(lane, wx - 1), oy = min(wave, wy - 1);
      const uint32_t ocell = (y0 + oy) * a.px + x0 + ox;
      const uint32_t olds = (oy + 1) * G::HX + ox + 1;
      march<L, R, kInterior>(a, lds_all, ocell, olds, own, ocell, olds, own, m0, m1);
    } else if (wave < (uint32_t)G::TY + 2) {
      // halo row below (y0 - 1) or above (y0 + wy) the tile, x0 ... x0 + wx - 1
      const bool lo = wave == (uint32_t)G::TY;
      const uint32_t sx = min(lane, wx - 1) + 1, sy = lo ? 0u : wy + 1;
      const uint32_t gy = lo ? (y0 + a.py - 1) % a.py : (y0 + wy) % a.py;
      const uint32_t scell = gy * a.px + x0 + sx - 1;
      const uint32_t slds = sy * G::HX + sx;
      if (lo)
        march<L, R, kRowLo>(a, lds_all, scell, slds, lane < wx, 0u, 0u, false, m0, m1);
      else
        march<L, R, kRowHi>(a, lds_all, scell, slds, lane < wx, 0u, 0u, false, m0, m1);
    } else {
      // halo columns x0 - 1 (lanes 0 ... hy - 1) and x0 + wx (the next hy
      // lanes), halo rows included.  The clamp of the idle lanes follows
      // the select: with it inside the second arm (min(lane - hy, hy - 1))
      // this compiler (ROCm 7.2 clang) dropped the first arm from the
      // device code.
      const bool left = lane < hy;
      const uint32_t sy = min(left ? lane : lane - hy, hy - 1);
      const uint32_t sx = left ? 0u : wx + 1;
      const uint32_t gx = left ? (x0 + a.px - 1) % a.px : (x0 + wx) % a.px;
      const uint32_t gy = (y0 + sy + a.py - 1) % a.py;
      march<L, R, kCols>(a, lds_all, gy * a.px + gx, sy * G::HX + sx, lane < 2 * hy, 0u, 0u,
                         false, m0, m1);
    }
  } else {
    // 2D: thread = slot of the halo row (x0 - 1 ... x0 + wx), the first wx
    // threads also own the output cells x0 ... x0 + wx - 1
    const uint32_t hx = wx + 2;
    const bool sown = tid < hx;
    const uint32_t sx = sown ? tid : 0u;
    const uint32_t scell = (x0 + sx + a.px - 1) % a.px;
    const bool oown = tid < wx;
    march<L, R, kAny>(a, lds_all, scell, sx, sown, y0 * a.px + x0 + tid, tid + 1, oown, m0, m1);
  }
}

template <class L, class R>
static hipError_t msweep_t(const SweepHost& h, int block, hipStream_t st) {
  using G = MTile<L, R>;
  MSweepArgs<R> a{};
  a.src = (const R*)h.src;
  a.dst = (R*)h.dst;
  a.status = h.status;
  a.px = h.nx;
  a.py = L::D == 3 ? h.ny : 1u;
  a.pm = L::D == 3 ? h.nz : h.ny;
  a.tiles_x = (a.px + G::TX - 1) / G::TX;
  a.tiles_y = (a.py + G::TY - 1) / G::TY;
  const uint32_t ntile = a.tiles_x * a.tiles_y;
  // planes per workgroup: block / 16 when given (the autotuner's
  // candidates 64 ... 1024 give 4 ... 64), else enough workgroups to fill
  // the device several times over
  uint32_t zc;
  if (block > 0) {
    zc = (uint32_t)block / 16u;
  } else {
    const uint32_t want = 2048u;
    const uint32_t chunks = (want + ntile - 1) / ntile;
    zc = (a.pm + chunks - 1) / chunks;
  }
  zc = zc < 4u ? 4u : (zc > 64u ? 64u : zc);
  a.zc = zc;
  const uint32_t chunks = (a.pm + zc - 1) / zc;
  a.nblocks = ntile * chunks;
  a.xcd_order = a.nblocks % 8u == 0u ? 1u : 0u;
  a.pstride = h.pstride;
  a.omega1 = (R)(1.0 - 1.0 / h.tau);
  a.rho0 = (R)h.rho0;
  hipLaunchKernelGGL((k_msweep<L, R>), dim3(a.nblocks), dim3(G::NT), 0, st, a);
  return hipGetLastError();
}

template <class L>
static hipError_t msweep_l(int storage, const SweepHost& h, int block, hipStream_t st) {
  return storage == kM64 ? msweep_t<L, double>(h, block, st) : msweep_t<L, float>(h, block, st);
}

hipError_t launch_msweep(int lattice, int storage, const SweepHost& h, int block,
                         hipStream_t st) {
  switch (lattice) {
    case 9: return msweep_l<Lattice<9>>(storage, h, block, st);
    case 19: return msweep_l<Lattice<19>>(storage, h, block, st);
    case 27: return msweep_l<Lattice<27>>(storage, h, block, st);
    case kFullOrderCode + 9: return msweep_l<Lattice<9, true>>(storage, h, block, st);
    case kFullOrderCode + 27: return msweep_l<Lattice<27, true>>(storage, h, block, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------
// Companion kernels of the moment storages.
// ------------------------------------------------------------------------

// Initial state f^{eqH}(rho, u) + (1 - 1/tau) f^{neqH}(pi_neq, u): its
// moments drho, u and a2* = (1 - 1/tau) pi_neq, in both buffers.
template <class L, class R>
__global__ void k_minit(InitArgs a) {
  constexpr int NM = MState<L>::NM;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  R m[NM];
  m[0] = (R)((a.rho ? a.rho[c] : a.rho0) - a.rho0);
#pragma unroll
  for (int k = 0; k < L::D; ++k) m[1 + k] = (R)(a.u ? a.u[(uint64_t)k * a.ncell + c] : a.uin[k]);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = MState<L>::a2_slot(k);
    if (s >= 0) m[s] = (R)(a.omega1 * (a.pineq ? a.pineq[(uint64_t)k * a.ncell + c] : 0.0));
  }
  R* d0 = (R*)a.dst0;
  R* d1 = (R*)a.dst1;
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    d0[(uint64_t)k * a.pstride + c] = m[k];
    d1[(uint64_t)k * a.pstride + c] = m[k];
  }
}

template <class L, class R>
__global__ void k_mmoments(MomentArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const R* s = (const R*)a.src;
  if (a.rho_out) a.rho_out[c] = a.rho0 + (double)s[c];
  if (a.u_out)
    for (int k = 0; k < 3; ++k)
      a.u_out[(uint64_t)k * a.ncell + c] = k < L::D ? (double)s[(uint64_t)(1 + k) * a.pstride + c] : 0.0;
}

template <class R>
__global__ void k_mprobe(ProbeArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n) return;
  const int64_t c = a.cells[n];
  a.rho_out[n] = (c < 0 || c >= (int64_t)a.ncell) ? 0.0 : a.rho0 + (double)((const R*)a.src)[c];
}

template <class R>
__global__ void k_maccum(AccumArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const double x = (double)((const R*)a.src)[c];
  if (a.sum1) a.sum1[c] += x;
  if (a.sum2) a.sum2[c] += x * x;
}

// Totals: sum of rho - rho0 and of j = rho u (same fixed reduction order as
// the population storages' totals).
template <class L, class R>
__global__ void __launch_bounds__(kRedThreads) k_mtotals(ReduceArgs a) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const uint32_t n = a.nx * a.ny * a.nz;
  const R* s = (const R*)a.src;
  for (uint32_t c = blockIdx.x * kRedThreads + threadIdx.x; c < n;
       c += kRedBlocks * kRedThreads) {
    const R drho = s[c];
    const R rho = (R)a.rho0 + drho;
    acc[0] += (double)drho;
    for (int k = 0; k < L::D; ++k) acc[k + 1] += (double)(rho * s[(uint64_t)(1 + k) * a.pstride + c]);
  }
  block_partial<4>(acc, a.partial);
}

// no SOLID cells on a moment-stored grid: the force is zero
__global__ void k_mzero3(double* out) {
  if (threadIdx.x < 3) out[threadIdx.x] = 0.0;
}

// canonical FP64 populations [q][N] from the moments (rebuilt in R)
template <class L, class R>
__global__ void k_mget_pop(PopArgs a) {
  constexpr int NM = MState<L>::NM;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  R m[NM], h[L::Q];
  load_state<L, R>((const R*)a.native, a.pstride, c, m);
  rebuild_cell<L, R>(m, (R)a.rho0, h);
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    a.canon[(uint64_t)i * a.ncell + c] = (double)h[i] + L::w(i) * a.rho0;
}

// moments of canonical populations (a regularized state is kept exactly;
// any other state is projected onto drho, u, a2*)
template <class L, class R>
__global__ void k_mset_pop(PopArgs a) {
  constexpr int NM = MState<L>::NM;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  double h[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) h[i] = a.canon[(uint64_t)i * a.ncell + c] - L::w(i) * a.rho0;
  double drho, j[3], P[6];
  raw_moments<L, double>(h, drho, j, P);
  const double rho = a.rho0 + drho;
  const double u[3] = {j[0] / rho, j[1] / rho, L::D == 3 ? j[2] / rho : 0.0};
  double a2[6];
  noneq_stress<L, double>(drho, j, u, P, a2);
  R m[NM];
  m[0] = (R)drho;
#pragma unroll
  for (int k = 0; k < L::D; ++k) m[1 + k] = (R)u[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = MState<L>::a2_slot(k);
    if (s >= 0) m[s] = (R)a2[k];
  }
  R* d0 = (R*)a.native;
  R* d1 = (R*)a.native2;
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    d0[(uint64_t)k * a.pstride + c] = m[k];
    if (d1) d1[(uint64_t)k * a.pstride + c] = m[k];
  }
}

static inline uint32_t grid_of(uint32_t n, uint32_t b) { return (n + b - 1) / b; }

#define HRLBM_MDISPATCH(LAUNCH)                                                        \
  switch (lattice) {                                                                   \
    case 9: LAUNCH(Lattice<9>); break;                                                 \
    case 19: LAUNCH(Lattice<19>); break;                                               \
    case 27: LAUNCH(Lattice<27>); break;                                               \
    case kFullOrderCode + 9: LAUNCH(Lattice<9 HRLBM_COMMA true>); break;               \
    case kFullOrderCode + 27: LAUNCH(Lattice<27 HRLBM_COMMA true>); break;             \
    default: return hipErrorInvalidValue;                                              \
  }
#define HRLBM_COMMA ,

hipError_t launch_minit(int lattice, int storage, const InitArgs& a, hipStream_t st) {
  if (a.ncell == 0) return hipSuccess;
#define HRLBM_L(LT)                                                                   \
  if (storage == kM64)                                                               \
    hipLaunchKernelGGL((k_minit<LT, double>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a); \
  else                                                                               \
    hipLaunchKernelGGL((k_minit<LT, float>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  HRLBM_MDISPATCH(HRLBM_L)
#undef HRLBM_L
  return hipGetLastError();
}

hipError_t launch_mmoments(int lattice, int storage, const MomentArgs& a, hipStream_t st) {
  if (a.ncell == 0) return hipSuccess;
#define HRLBM_L(LT)                                                                   \
  if (storage == kM64)                                                               \
    hipLaunchKernelGGL((k_mmoments<LT, double>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a); \
  else                                                                               \
    hipLaunchKernelGGL((k_mmoments<LT, float>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  HRLBM_MDISPATCH(HRLBM_L)
#undef HRLBM_L
  return hipGetLastError();
}

hipError_t launch_mprobe(int storage, const ProbeArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (storage == kM64)
    hipLaunchKernelGGL((k_mprobe<double>), dim3(grid_of((uint32_t)a.n, 256)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_mprobe<float>), dim3(grid_of((uint32_t)a.n, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_maccum(int storage, const AccumArgs& a, hipStream_t st) {
  if (a.ncell == 0) return hipSuccess;
  if (storage == kM64)
    hipLaunchKernelGGL((k_maccum<double>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_maccum<float>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mtotals(int lattice, int storage, const ReduceArgs& a, hipStream_t st) {
#define HRLBM_L(LT)                                                                   \
  if (storage == kM64)                                                               \
    hipLaunchKernelGGL((k_mtotals<LT, double>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, a); \
  else                                                                               \
    hipLaunchKernelGGL((k_mtotals<LT, float>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, a);
  HRLBM_MDISPATCH(HRLBM_L)
#undef HRLBM_L
  hipLaunchKernelGGL((k_reduce_final<4>), dim3(1), dim3(kRedThreads), 0, st, a.partial, a.out);
  return hipGetLastError();
}

hipError_t launch_mforce(const ReduceArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_mzero3, dim3(1), dim3(64), 0, st, a.out);
  return hipGetLastError();
}

hipError_t launch_mget_pop(int lattice, int storage, const PopArgs& a, hipStream_t st) {
  if (a.ncell == 0) return hipSuccess;
#define HRLBM_L(LT)                                                                   \
  if (storage == kM64)                                                               \
    hipLaunchKernelGGL((k_mget_pop<LT, double>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a); \
  else                                                                               \
    hipLaunchKernelGGL((k_mget_pop<LT, float>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  HRLBM_MDISPATCH(HRLBM_L)
#undef HRLBM_L
  return hipGetLastError();
}

hipError_t launch_mset_pop(int lattice, int storage, const PopArgs& a, hipStream_t st) {
  if (a.ncell == 0) return hipSuccess;
#define HRLBM_L(LT)                                                                   \
  if (storage == kM64)                                                               \
    hipLaunchKernelGGL((k_mset_pop<LT, double>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a); \
  else                                                                               \
    hipLaunchKernelGGL((k_mset_pop<LT, float>), dim3(grid_of(a.ncell, 256)), dim3(256), 0, st, a);
  HRLBM_MDISPATCH(HRLBM_L)
#undef HRLBM_L
  return hipGetLastError();
}

}  // namespace hrlbm
