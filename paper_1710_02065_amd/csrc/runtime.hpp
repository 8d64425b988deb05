// Context and level state shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>

#include "../../include/lbm.h"
#include "launch.hpp"

namespace hrlbm {

struct Level {
  int level = 0;
  int q = 0;
  int64_t nx = 0, ny = 0, nz = 0, N = 0;
  double tau = 0.6;
  double chi_max = 0.0;
  int32_t face[6] = {0, 0, 0, 0, 0, 0};
  int32_t sponge[6] = {0, 0, 0, 0, 0, 0};
  uint64_t pstride = 0;
  size_t buf_bytes = 0, bytes = 0, base_off = 0;
  size_t off_buf[2] = {0, 0}, off_mask = 0, off_tiles = 0, off_sponge = 0;
  void* buf[2] = {nullptr, nullptr};
  uint8_t* mask = nullptr;
  uint8_t* tiles = nullptr;  // per 64-cell tile: 1 = plain fluid (see k_tiles)
  void* sp = nullptr;        // per-cell absorbing layer (LBM_SPONGE_FIELD)
  // halo faces of the last axis (slab decomposition): send and receive
  // buffers per side (nullptr where the face is not LBM_HALO), each
  // halo_bytes, hplane cells per face plane
  size_t off_halo = 0, halo_bytes = 0;
  void* hsend[2] = {nullptr, nullptr};
  void* hrecv[2] = {nullptr, nullptr};
  uint32_t hplane = 0;
  bool field_sponge = false; // set by lbm_set_sponge since the last init
  bool has_mask = false;
  bool initialised = false;
  int cur = 0;    // buffer holding the current state
  int64_t t = 0;  // time index on this level
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct Refinement;  // two-level coupling state (refine.hip)

}  // namespace hrlbm

namespace hrlbm {
constexpr int kMaxLevels = LBM_MAX_LEVELS;
}  // namespace hrlbm

struct lbm_ctx {
  lbm_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  int nlevels = 1;
  hrlbm::Level lv[hrlbm::kMaxLevels];
  double uin[3] = {0, 0, 0};
  char* mem = nullptr;
  bool owns_mem = false;
  size_t total_bytes = 0;
  int* status = nullptr;
  double* reduce = nullptr;  // kRedBlocks x kRedMax partial sums
  bool status_cleared = false;
  bool unstable = false;
  bool initialised = false;
  bool has_inlet = false;
  int64_t t = 0;
  int block = 256;
  std::map<int, hrlbm::GraphEntry> graphs;
  // interface l couples level l (parent) and level l + 1 (child)
  hrlbm::Refinement* ref[hrlbm::kMaxLevels - 1] = {};
  ~lbm_ctx();
};

namespace hrlbm {

// Lattice code the collision kernels are dispatched on: the lattice id,
// plus kFullOrderCode with LBM_FULL_ORDER.
inline int kernel_lattice(const lbm_config& c) {
  return c.lattice + ((c.flags & LBM_FULL_ORDER) ? kFullOrderCode : 0);
}
// Lattice code of the sweep: kernel_lattice, or a comparator collision.
inline int sweep_lattice(const lbm_config& c) {
  if (c.flags & LBM_BGK) return c.lattice + kBgkCode;
  if (c.flags & LBM_MRT) return c.lattice + kMrtCode;
  return kernel_lattice(c);
}

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
int lattice_dim(int lattice);
size_t storage_bytes(int storage);
uint64_t pop_stride(uint64_t n);
int validate(const lbm_config* cfg);
// face index of side 0 (low) / 1 (high) of the last axis, the only axis
// that may carry LBM_HALO faces
int halo_face(int lattice, int side);
bool has_halo(const lbm_config& c);
void plan_layout(lbm_ctx* ctx);
void assign_pointers(lbm_ctx* ctx);
int ensure_device(const lbm_ctx* ctx);
int check_ready(const lbm_ctx* ctx);
// the sweep of one level: the population or the moment-storage kernel
hipError_t launch_step_kernel(const lbm_ctx* ctx, const SweepHost& h, int block,
                              hipStream_t st);
SweepHost sweep_args(const lbm_ctx* ctx, int level, int src_buf, uint64_t t_new);
int sweep_level(lbm_ctx* ctx, int level, hipStream_t st);
int step_ctx(lbm_ctx* ctx, int64_t n, hipStream_t st);

// workgroup size from the autotuner cache, 0 if none (serve.hip)
int tuned_block(const lbm_ctx* ctx);

// two-level refinement (refine.hip)
int validate_refinement(const lbm_config& c);
size_t plan_interface_layout(lbm_ctx* ctx, size_t off);
void assign_interface_pointers(lbm_ctx* ctx);
int refined_init_level(lbm_ctx* ctx, int level, const double* rho, const double* u,
                       const double* pineq);
int refined_after_init(lbm_ctx* ctx);
int64_t refined_updates_per_step(const lbm_ctx* ctx);
int refined_after_set(lbm_ctx* ctx, int level);
int refined_coarse_step(lbm_ctx* ctx, hipStream_t st);
// checkpoint of interface l: size and device-to-device copy of its records
// (out != nullptr: export; else import from in)
size_t refined_interface_bytes(const lbm_ctx* ctx, int l);
int refined_copy_interface(lbm_ctx* ctx, int l, void* out, const void* in);
// which of the two parent-side records of interface l holds M_l(t)
int refined_record_parity(const lbm_ctx* ctx, int l);
void set_refined_record_parity(lbm_ctx* ctx, int l, int parity);
int make_levels_refined(lbm_ctx* ctx);
void free_refinement(lbm_ctx* ctx);

}  // namespace hrlbm
