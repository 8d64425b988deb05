// HIP kernels of the regularized LBM step and their host launchers.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "launch.hpp"

namespace hrlbm {

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

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
// The sweep: pull-stream + (sponge) + regularized collision + store.
// kGeneral = false: every face periodic, no mask, no sponge.
// ------------------------------------------------------------------------
template <class L, class S, bool kGeneral>
__global__ void __launch_bounds__(1024)
    k_sweep(const SweepArgs<S> a) {
  using R = typename S::R;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t c = tile * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  const uint32_t row = fast_div(c, a.div_nx);
  const uint32_t x = c - row * a.nx;
  const uint32_t z = fast_div(row, a.div_ny);
  const uint32_t y = row - z * a.ny;
  const uint64_t P = a.pstride;

  R h[Q];
  R post[Q];
  R rho;
  if constexpr (!kGeneral) {
    // periodic wrap: offsets to the x-1 / x+1 (etc.) neighbours
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
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr Dir v = L::dir(i);
      int32_t off = 0;
      if constexpr (v.x > 0) off += ox_m;
      if constexpr (v.x < 0) off += ox_p;
      if constexpr (v.y > 0) off += oy_m;
      if constexpr (v.y < 0) off += oy_p;
      if constexpr (v.z > 0) off += oz_m;
      if constexpr (v.z < 0) off += oz_p;
      const R wr = (R)L::w(i) * a.rho0;
      h[i] = decode<S>(a.src[(uint64_t)i * P + (uint32_t)((int32_t)c + off)], wr);
    });
    rho = collide<L, R, false>(h, a.omega1, a.rho0, (R)0, a.rho_ref, a.uref, post);
  } else {
    uint8_t m = kFluid;
    if (a.mask) m = a.mask[c];
    if (m == kSolid) return;
    if (m == kInlet) {
      // f^{eqH}(rho0, U u_dir (1 + noise r)), r from SplitMix64
      R u[3];
      const uint64_t base =
          ((a.t_new * 2ull + (uint64_t)a.level) * (uint64_t)a.ncell + c) * 3ull;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R r = (R)splitmix_pm1(a.seed, base + (uint64_t)k);
        u[k] = a.uin[k] * ((R)1 + a.noise * r);
      }
      if (L::D == 2) u[2] = (R)0;
      const R zero6[6] = {(R)0, (R)0, (R)0, (R)0, (R)0, (R)0};
      rebuild_state<L, R>((R)0, a.rho0, u, zero6, (R)0, post);
      static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const R wr = (R)L::w(i) * a.rho0;
        __builtin_nontemporal_store(encode<S>(post[i], wr), &a.dst[(uint64_t)i * P + c]);
      });
      return;
    }
    const uint32_t dims[3] = {a.nx, a.ny, a.nz};
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr Dir v = L::dir(i);
      constexpr int vv[3] = {v.x, v.y, v.z};
      int32_t s[3] = {(int32_t)x - v.x, (int32_t)y - v.y, (int32_t)z - v.z};
      bool flip[3] = {false, false, false};
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
          }
        }
      }
      const uint32_t src = ((uint32_t)s[2] * a.ny + (uint32_t)s[1]) * a.nx + (uint32_t)s[0];
      const R wr = (R)L::w(i) * a.rho0;
      if (a.mask && a.mask[src] == kSolid) {
        // halfway bounce-back: the population that left this cell towards
        // the wall comes back reversed
        constexpr int o = opposite<L>(i);
        h[i] = decode<S>(a.src[(uint64_t)o * P + c], wr);
      } else {
        int pop = i;
        if (flip[0] || flip[1] || flip[2])
          pop = dir_rt<L>(flip[0] ? -v.x : v.x, flip[1] ? -v.y : v.y,
                          flip[2] ? -v.z : v.z);
        h[i] = decode<S>(a.src[(uint64_t)pop * P + src], wr);
      }
    });
    R chi = (R)0;
    if (a.chi_max != (R)0)
      chi = sponge_chi<R>(a.sponge, a.chi_max, x, y, z, a.nx, a.ny, a.nz);
    rho = collide<L, R, true>(h, a.omega1, a.rho0, chi, a.rho_ref, a.uref, post);
  }
  // stability watchdog: a rare, benign racy store of 1
  if (!(rho > (R)0) || !(rho < (R)1e30)) a.status[0] = 1;
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const R wr = (R)L::w(i) * a.rho0;
    __builtin_nontemporal_store(encode<S>(post[i], wr), &a.dst[(uint64_t)i * P + c]);
  });
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
  if (a.mask && a.mask[c] == kSolid) {
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
  if (a.mask && a.mask[c] == kSolid) {
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
// Host launchers
// ------------------------------------------------------------------------
template <class S>
static SweepArgs<S> to_args(const SweepHost& h) {
  using T = typename S::T;
  using R = typename S::R;
  SweepArgs<S> a;
  a.src = (const T*)h.src;
  a.dst = (T*)h.dst;
  a.mask = h.mask;
  a.status = h.status;
  a.nx = h.nx;
  a.ny = h.ny;
  a.nz = h.nz;
  a.ncell = h.nx * h.ny * h.nz;
  a.pstride = h.pstride;
  a.div_nx = make_fastdiv(h.nx);
  a.div_ny = make_fastdiv(h.ny);
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
  return a;
}

template <class L, class S>
static hipError_t launch_sweep_t(const SweepHost& h, int block, hipStream_t st) {
  SweepArgs<S> a = to_args<S>(h);
  const uint32_t blocks = (a.ncell + block - 1) / block;
  a.ntiles = blocks;
  if (h.general)
    hipLaunchKernelGGL((k_sweep<L, S, true>), dim3(blocks), dim3(block), 0, st, a);
  else
    hipLaunchKernelGGL((k_sweep<L, S, false>), dim3(blocks), dim3(block), 0, st, a);
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
  }
  return hipErrorInvalidValue;
}

// dispatch of the companion kernels over lattice and storage
#define HRLBM_DISPATCH(NAME, ARGS)                                            \
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
      default: return hipErrorInvalidValue;                                   \
    }                                                                         \
    return hipGetLastError();                                                 \
  }

HRLBM_DISPATCH(init, InitArgs)
HRLBM_DISPATCH(moments, MomentArgs)
HRLBM_DISPATCH(probe, ProbeArgs)
HRLBM_DISPATCH(get_pop, PopArgs)
HRLBM_DISPATCH(set_pop, PopArgs)

}  // namespace hrlbm
