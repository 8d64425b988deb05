// Host-side argument blocks and launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hrlbm {

// One sweep of one grid: src -> dst.
struct SweepHost {
  const void* src;
  void* dst;
  const uint8_t* mask;  // nullptr = all fluid
  int* status;
  uint32_t nx, ny, nz;
  uint64_t pstride;
  double tau, rho0;
  double chi_max, rho_ref, uref[3];
  double uin[3], noise;
  int32_t face[6], sponge[6];
  uint64_t seed, t_new;
  int32_t level;
  bool general;  // false: all periodic, no mask, no sponge
};

struct InitArgs {
  const double* rho;
  const double* u;
  const double* pineq;
  const uint8_t* mask_in;
  uint8_t* mask_out;
  void* dst0;
  void* dst1;
  uint32_t ncell;
  uint64_t pstride;
  double rho0, omega1, uin[3];
};

struct MomentArgs {
  const void* src;
  const uint8_t* mask;
  double* rho_out;
  double* u_out;
  uint32_t ncell;
  uint64_t pstride;
  double rho0;
};

struct ProbeArgs {
  const void* src;
  const uint8_t* mask;
  const int64_t* cells;
  double* rho_out;
  int n;
  uint32_t ncell;
  uint64_t pstride;
  double rho0;
};

struct PopArgs {
  void* native;
  void* native2;  // optional second buffer (set only)
  double* canon;
  uint32_t ncell;
  uint64_t pstride;
  double rho0;
};

hipError_t launch_sweep(int lattice, int storage, const SweepHost& h, int block,
                        hipStream_t st);
hipError_t launch_init(int lattice, int storage, const InitArgs& a, uint32_t n,
                       hipStream_t st);
hipError_t launch_moments(int lattice, int storage, const MomentArgs& a,
                          uint32_t n, hipStream_t st);
hipError_t launch_probe(int lattice, int storage, const ProbeArgs& a,
                        uint32_t n, hipStream_t st);
hipError_t launch_get_pop(int lattice, int storage, const PopArgs& a,
                          uint32_t n, hipStream_t st);
hipError_t launch_set_pop(int lattice, int storage, const PopArgs& a,
                          uint32_t n, hipStream_t st);

}  // namespace hrlbm
