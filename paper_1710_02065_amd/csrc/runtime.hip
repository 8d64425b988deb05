// Host runtime behind the C ABI of include/lbm.h: configuration checks,
// device memory layout, the step loop (with hipGraph replay of step
// sequences), observables and population import/export.
#include <hip/hip_runtime.h>

#include <climits>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lattice.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace hrlbm {

thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int lattice_dim(int lattice) { return lattice == LBM_D2Q9 ? 2 : 3; }

size_t storage_bytes(int storage) {
  switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32:
    case LBM_F32S: return 4;
    case LBM_F16S: return 2;
    case LBM_M64: return 8;
    case LBM_M32: return 4;
  }
  return 0;
}

// stored values per cell: q populations, or the moments of a moment storage
static int values_per_cell(int lattice, int storage) {
  if (moment_storage(storage)) return lattice == LBM_D2Q9 ? 6 : 10;
  return lattice;
}

// Population stride: a multiple of 128 elements, plus a pad (128 elements
// unless HRLBM_POP_PAD says otherwise) on large grids so that power-of-two
// grids do not put every population at the same offset modulo the HBM
// channel interleave.
uint64_t pop_stride(uint64_t n) {
  static const long pad = [] {
    const char* s = std::getenv("HRLBM_POP_PAD");
    return s ? std::atol(s) : 128L;
  }();
  uint64_t p = align_up(n, 128);
  if (n >= (1u << 20)) p += (uint64_t)(pad < 0 ? 0 : pad);
  return p;
}

static bool refined(const lbm_config& c) {
  for (int a = 0; a < 3; ++a)
    if (c.refine_lo[a] != 0 || c.refine_hi[a] != 0) return true;
  return false;
}

int halo_face(int lattice, int side) { return (lattice == LBM_D2Q9 ? 2 : 4) + side; }

bool has_halo(const lbm_config& c) {
  return c.face_bc[halo_face(c.lattice, 0)] == LBM_HALO ||
         c.face_bc[halo_face(c.lattice, 1)] == LBM_HALO;
}

static double inlet_speed(const lbm_config& c) {
  return c.ma * std::sqrt(1.0 / 3.0);
}

// U * u_dir / |u_dir|
static void inlet_velocity(const lbm_config& c, double u[3]) {
  double n = std::sqrt(c.u_dir[0] * c.u_dir[0] + c.u_dir[1] * c.u_dir[1] +
                       c.u_dir[2] * c.u_dir[2]);
  const double U = inlet_speed(c);
  for (int a = 0; a < 3; ++a) u[a] = n > 0 ? U * c.u_dir[a] / n : 0.0;
  if (c.lattice == LBM_D2Q9) u[2] = 0.0;
}

int validate(const lbm_config* cfg) {
  if (!cfg) return set_error(LBM_EINVAL, "config is NULL");
  const lbm_config& c = *cfg;
  if (c.struct_size != sizeof(lbm_config))
    return set_error(LBM_EINVAL, "struct_size %u != %zu (call lbm_config_init)",
                     c.struct_size, sizeof(lbm_config));
  if (c.lattice != LBM_D2Q9 && c.lattice != LBM_D3Q19 && c.lattice != LBM_D3Q27)
    return set_error(LBM_EINVAL, "unknown lattice %d", c.lattice);
  if (storage_bytes(c.storage) == 0)
    return set_error(LBM_EINVAL, "unknown storage %d", c.storage);
  if (c.nx < 1 || c.ny < 1 || c.nz < 1)
    return set_error(LBM_EINVAL, "grid %lld x %lld x %lld", (long long)c.nx,
                     (long long)c.ny, (long long)c.nz);
  if (c.lattice == LBM_D2Q9 && c.nz != 1)
    return set_error(LBM_EINVAL, "D2Q9 needs nz == 1");
  const double cells = (double)c.nx * (double)c.ny * (double)c.nz;
  if (cells > 2147483647.0)
    return set_error(LBM_EINVAL, "grid has %.0f cells; the limit is 2^31 - 1", cells);
  // each population array is addressed with 32-bit byte offsets
  if ((double)pop_stride((uint64_t)cells) * (double)storage_bytes(c.storage) > 4294967040.0)
    return set_error(LBM_EINVAL,
                     "grid has %.0f cells: one population array would exceed 4 GiB "
                     "(limit 2^31 cells for F16S, 2^30 for F32/F32S, 2^29 for F64)", cells);
  if (!(c.tau > 0.5) || !std::isfinite(c.tau))
    return set_error(LBM_EINVAL, "tau = %g: nu = cs^2 (tau - 1/2) must be > 0", c.tau);
  if (!(c.rho0 > 0)) return set_error(LBM_EINVAL, "rho0 must be > 0");
  if ((c.flags & LBM_BGK) && (c.flags & LBM_MRT))
    return set_error(LBM_EINVAL, "LBM_BGK and LBM_MRT are exclusive");
  if ((c.flags & (LBM_BGK | LBM_MRT)) && (c.flags & LBM_FULL_ORDER))
    return set_error(LBM_EINVAL, "the comparator collisions have no LBM_FULL_ORDER");
  if ((c.flags & (LBM_BGK | LBM_MRT)) && refined(c))
    return set_error(LBM_EINVAL, "the comparator collisions run unrefined");
  if ((c.flags & LBM_MRT) &&
      (c.lattice != LBM_D2Q9 || c.chi_max != 0.0 || (c.flags & LBM_SPONGE_FIELD)))
    return set_error(LBM_EINVAL, "LBM_MRT: D2Q9 without sponge");
  if ((c.flags & LBM_FULL_ORDER) && c.lattice == LBM_D3Q19)
    return set_error(LBM_EINVAL, "LBM_FULL_ORDER needs D2Q9 or D3Q27 (D3Q19 resolves third order only)");
  if (!(c.ma >= 0) || (c.ma > 0.6 && !(c.flags & LBM_ALLOW_HIGH_MA)))
    return set_error(LBM_EINVAL, "Ma = %g outside [0, 0.6] (set LBM_ALLOW_HIGH_MA)", c.ma);
  if (!(c.chi_max >= 0))
    return set_error(LBM_EINVAL, "chi_max must be >= 0");
  for (int a = 0; a < 3; ++a) {
    const bool p0 = c.face_bc[2 * a] == LBM_PERIODIC, p1 = c.face_bc[2 * a + 1] == LBM_PERIODIC;
    if (p0 != p1)
      return set_error(LBM_EINVAL, "axis %d: both faces periodic or neither", a);
  }
  for (int f = 0; f < 6; ++f) {
    if (c.face_bc[f] < LBM_PERIODIC || c.face_bc[f] > LBM_HALO)
      return set_error(LBM_EINVAL, "face %d: unknown rule %d", f, c.face_bc[f]);
    if (c.face_bc[f] == LBM_HALO) {
      if (f / 2 != halo_face(c.lattice, 0) / 2)
        return set_error(LBM_EINVAL, "face %d: LBM_HALO only on the faces of the last axis "
                         "(z in 3D, y on D2Q9)", f);
      // the analytic layer profile would use this subdomain's own extent
      if (c.sponge_width[f] != 0)
        return set_error(LBM_EINVAL, "face %d: no absorbing layer on a halo face", f);
    }
    const int64_t n = f < 2 ? c.nx : (f < 4 ? c.ny : c.nz);
    if (c.sponge_width[f] < 0 || c.sponge_width[f] > n)
      return set_error(LBM_EINVAL, "face %d: sponge width %d", f, c.sponge_width[f]);
    if (c.lattice == LBM_D2Q9 && f >= 4 && c.sponge_width[f] != 0)
      return set_error(LBM_EINVAL, "D2Q9 has no z faces");
  }
  if (c.lattice == LBM_D2Q9 && (c.face_bc[4] != LBM_PERIODIC || c.face_bc[5] != LBM_PERIODIC))
    return set_error(LBM_EINVAL, "D2Q9: z faces must be LBM_PERIODIC");
  // Sec. II.C: sigma_eff > 0 requires chi < 4 tau (on every level; the fine
  // level has the larger tau, so the coarse tau bounds both)
  if (c.chi_max >= 4.0 * c.tau)
    return set_error(LBM_EINVAL, "chi_max = %g >= 4 tau = %g (Sec. II.C stability bound)",
                     c.chi_max, 4.0 * c.tau);
  if (c.nest_count < 0 || c.nest_count > LBM_MAX_LEVELS - 2)
    return set_error(LBM_EINVAL, "nest_count %d outside [0, %d]", c.nest_count,
                     LBM_MAX_LEVELS - 2);
  if (c.nest_count > 0 && !refined(c))
    return set_error(LBM_EINVAL, "nested boxes need the level-1 box refine_lo/hi");
  if (moment_storage(c.storage)) {
    // the stored moments rebuild the regularized post-collision state
    // exactly only where no face rule, wall, layer or interface acts
    for (int f = 0; f < 6; ++f)
      if (c.face_bc[f] != LBM_PERIODIC)
        return set_error(LBM_EINVAL, "moment storage needs every face LBM_PERIODIC");
    if (refined(c) || c.nest_count > 0)
      return set_error(LBM_EINVAL, "moment storage runs unrefined");
    if (c.chi_max != 0.0 || (c.flags & LBM_SPONGE_FIELD))
      return set_error(LBM_EINVAL, "moment storage has no absorbing layer");
    if (c.flags & (LBM_BGK | LBM_MRT))
      return set_error(LBM_EINVAL, "moment storage needs the regularized collision");
  }
  if (has_halo(c) && (refined(c) || c.nest_count > 0))
    return set_error(LBM_EINVAL, "halo faces need an unrefined context");
  if (refined(c)) return validate_refinement(c);
  return LBM_OK;
}

// device memory layout of one level: A, B, mask
static void level_layout(Level& L, int lattice, int storage, bool sponge_field) {
  const int q = lattice;
  L.q = q;
  L.pstride = pop_stride((uint64_t)L.N);
  const size_t popbytes = align_up(L.pstride * storage_bytes(storage), 256);
  L.buf_bytes = popbytes * values_per_cell(lattice, storage);
  L.off_buf[0] = 0;
  L.off_buf[1] = L.buf_bytes;
  L.off_mask = 2 * L.buf_bytes;
  L.off_tiles = align_up(L.off_mask + (size_t)L.N, 256);
  L.off_sponge = align_up(L.off_tiles + (size_t)(L.N + 63) / 64, 256);
  const size_t rsz = (storage == LBM_F64 || storage == LBM_M64) ? 8 : 4;
  L.bytes = align_up(L.off_sponge + (sponge_field ? 5 * (size_t)L.N * rsz : 0), 256);
}

void plan_layout(lbm_ctx* ctx) {
  const lbm_config& c = ctx->cfg;
  // status words first, then the partial sums of the reductions
  size_t off = 256 + align_up(sizeof(double) * kRedMax * kRedBlocks, 256);
  for (int l = 0; l < ctx->nlevels; ++l) {
    Level& L = ctx->lv[l];
    level_layout(L, c.lattice, c.storage, (c.flags & LBM_SPONGE_FIELD) != 0);
    if (l == 0 && has_halo(c)) {
      // send low, send high, receive low, receive high
      L.hplane = (uint32_t)(c.lattice == LBM_D2Q9 ? L.nx : L.nx * L.ny);
      L.halo_bytes = align_up((size_t)halo_count_of(c.lattice) * L.hplane *
                                  storage_bytes(c.storage), 256);
      L.off_halo = L.bytes;
      L.bytes += 4 * L.halo_bytes;
    }
    L.base_off = off;
    off += L.bytes;
  }
  off = plan_interface_layout(ctx, off);
  ctx->total_bytes = off;
}

}  // namespace hrlbm

using namespace hrlbm;

extern "C" {

void lbm_config_init(lbm_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(lbm_config);
  cfg->lattice = LBM_D3Q19;
  cfg->storage = LBM_F32;
  cfg->nx = cfg->ny = cfg->nz = 64;
  cfg->tau = 0.6;
  cfg->rho0 = 1.0;
  cfg->u_dir[0] = 1.0;
  cfg->rho_ref = 1.0;
}

static int make_levels(lbm_ctx* ctx) {
  const lbm_config& c = ctx->cfg;
  ctx->nlevels = 1;
  Level& L0 = ctx->lv[0];
  L0.nx = c.nx;
  L0.ny = c.ny;
  L0.nz = c.nz;
  L0.N = c.nx * c.ny * c.nz;
  L0.tau = c.tau;
  L0.level = 0;
  for (int f = 0; f < 6; ++f) {
    L0.face[f] = c.face_bc[f];
    L0.sponge[f] = c.sponge_width[f];
  }
  L0.chi_max = c.chi_max;
  if (refined(c)) return make_levels_refined(ctx);
  return LBM_OK;
}

size_t lbm_required_bytes(const lbm_config* cfg) {
  if (validate(cfg) != LBM_OK) return 0;
  lbm_ctx tmp;
  tmp.cfg = *cfg;
  if (make_levels(&tmp) != LBM_OK) return 0;
  plan_layout(&tmp);
  return tmp.total_bytes;
}

int lbm_create(const lbm_config* cfg, lbm_ctx** out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc != LBM_OK) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (cfg->device < 0 || cfg->device >= ndev)
    return set_error(LBM_EINVAL, "device %d of %d", cfg->device, ndev);
  lbm_ctx* ctx = new (std::nothrow) lbm_ctx();
  if (!ctx) return set_error(LBM_ENOMEM, "host allocation");
  ctx->cfg = *cfg;
  ctx->stream = (hipStream_t)cfg->stream;
  ctx->device = cfg->device;
  inlet_velocity(ctx->cfg, ctx->uin);
  rc = make_levels(ctx);
  if (rc != LBM_OK) {
    delete ctx;
    return rc;
  }
  plan_layout(ctx);
  ctx->block = cfg->block ? (int)cfg->block : 256;
  if (ctx->block % 64 || ctx->block < 64 || ctx->block > 1024) {
    delete ctx;
    return set_error(LBM_EINVAL, "block %u: multiple of 64 in [64, 1024]", cfg->block);
  }
  *out = ctx;
  return LBM_OK;
}

int lbm_bind_memory(lbm_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  if (ctx->mem) return set_error(LBM_ESTATE, "memory already set up (bind before lbm_init)");
  if (!dev_ptr || ((uintptr_t)dev_ptr % 256))
    return set_error(LBM_EINVAL, "buffer must be non-NULL and 256-byte aligned");
  if (bytes < ctx->total_bytes)
    return set_error(LBM_ENOMEM, "bound buffer has %zu bytes, need %zu", bytes, ctx->total_bytes);
  ctx->mem = (char*)dev_ptr;
  ctx->owns_mem = false;
  assign_pointers(ctx);
  return LBM_OK;
}

}  // extern "C"

namespace hrlbm {

void assign_pointers(lbm_ctx* ctx) {
  ctx->status = (int*)ctx->mem;
  ctx->reduce = (double*)(ctx->mem + 256);
  for (int l = 0; l < ctx->nlevels; ++l) {
    Level& L = ctx->lv[l];
    char* b = ctx->mem + L.base_off;
    L.buf[0] = b + L.off_buf[0];
    L.buf[1] = b + L.off_buf[1];
    L.mask = (uint8_t*)(b + L.off_mask);
    L.tiles = (uint8_t*)(b + L.off_tiles);
    L.sp = (ctx->cfg.flags & LBM_SPONGE_FIELD) ? (void*)(b + L.off_sponge) : nullptr;
    for (int side = 0; side < 2; ++side) {
      const bool on = L.halo_bytes && L.face[halo_face(ctx->cfg.lattice, side)] == LBM_HALO;
      L.hsend[side] = on ? b + L.off_halo + side * L.halo_bytes : nullptr;
      L.hrecv[side] = on ? b + L.off_halo + (2 + side) * L.halo_bytes : nullptr;
    }
  }
  assign_interface_pointers(ctx);
}

int ensure_device(const lbm_ctx* ctx) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  if (cur != ctx->device) {
    e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  }
  return LBM_OK;
}

static int ensure_memory(lbm_ctx* ctx) {
  if (ctx->mem) return LBM_OK;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, ctx->total_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(LBM_ENOMEM, "hipMalloc(%zu): %s", ctx->total_bytes, hipGetErrorString(e));
  }
  ctx->mem = (char*)p;
  ctx->owns_mem = true;
  assign_pointers(ctx);
  return LBM_OK;
}

// Fill the sweep arguments of level l for one step producing time t_new.
SweepHost sweep_args(const lbm_ctx* ctx, int l, int src_buf, uint64_t t_new) {
  const Level& L = ctx->lv[l];
  const lbm_config& c = ctx->cfg;
  SweepHost h{};
  h.src = L.buf[src_buf];
  h.dst = L.buf[src_buf ^ 1];
  h.mask = L.has_mask ? L.mask : nullptr;
  h.tiles = L.has_mask ? L.tiles : nullptr;
  h.status = ctx->status;
  h.nx = (uint32_t)L.nx;
  h.ny = (uint32_t)L.ny;
  h.nz = (uint32_t)L.nz;
  h.pstride = L.pstride;
  h.tau = L.tau;
  h.rho0 = c.rho0;
  h.chi_max = L.chi_max;
  h.rho_ref = c.rho_ref;
  for (int a = 0; a < 3; ++a) {
    h.uref[a] = c.lattice == LBM_D2Q9 && a == 2 ? 0.0 : c.u_ref[a];
    h.uin[a] = ctx->uin[a];
  }
  h.noise = c.inlet_noise;
  if (L.field_sponge) {
    // the per-cell layer replaces the face profile on this level
    h.sp = L.sp;
    h.chi_max = 0.0;
  }
  // halo faces also run on the periodic path (which reads them itself)
  // when every other face is periodic
  bool general = L.has_mask || L.chi_max > 0;
  for (int f = 0; f < 6; ++f) {
    h.face[f] = L.face[f];
    h.sponge[f] = L.sponge[f];
    if (L.face[f] != LBM_PERIODIC && L.face[f] != LBM_HALO) general = true;
  }
  h.seed = c.seed;
  h.t_new = t_new;
  h.level = L.level;
  h.lstride = ctx->nlevels > 2 ? (uint32_t)ctx->nlevels : 2u;
  h.general = general;
  for (int side = 0; side < 2; ++side) {
    h.hrecv[side] = L.hrecv[side];
    h.hsend[side] = L.hsend[side];
  }
  h.hplane = L.hplane;
  return h;
}

hipError_t launch_step_kernel(const lbm_ctx* ctx, const SweepHost& h, int block,
                              hipStream_t st) {
  if (moment_storage(ctx->cfg.storage))
    return launch_msweep(kernel_lattice(ctx->cfg), ctx->cfg.storage, h, block, st);
  return launch_sweep(sweep_lattice(ctx->cfg), ctx->cfg.storage, h, block, st);
}

int check_ready(const lbm_ctx* ctx) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  if (!ctx->initialised) return set_error(LBM_ESTATE, "lbm_init has not been called");
  return LBM_OK;
}

// One eager sweep of level l.
int sweep_level(lbm_ctx* ctx, int l, hipStream_t st) {
  Level& L = ctx->lv[l];
  SweepHost h = sweep_args(ctx, l, L.cur, (uint64_t)(L.t + 1));
  hipError_t e = launch_step_kernel(ctx, h, ctx->block, st);
  if (e != hipSuccess) return hip_error(e, "sweep launch");
  L.cur ^= 1;
  L.t += 1;
  return LBM_OK;
}

// Enqueue n single-grid steps eagerly.
static int step_eager(lbm_ctx* ctx, int64_t n, hipStream_t st) {
  for (int64_t s = 0; s < n; ++s) {
    int rc = ctx->nlevels > 1 ? refined_coarse_step(ctx, st) : sweep_level(ctx, 0, st);
    if (rc != LBM_OK) return rc;
    if (ctx->nlevels == 1) ctx->t += 1;
  }
  return LBM_OK;
}

// Replaying captured step sequences: a graph holds kGraphSteps steps from a
// given buffer parity and time; inlet noise depends on the absolute time,
// so graphs are keyed by (parity, t mod period) only when no cell draws
// noise, and otherwise not used.
static constexpr int64_t kGraphSteps = 32;

static void drop_graphs(lbm_ctx* ctx) {
  for (auto& kv : ctx->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  ctx->graphs.clear();
}

static bool graphs_allowed(const lbm_ctx* ctx) {
  if (ctx->cfg.flags & LBM_NO_GRAPH) return false;
  // inlet noise depends on the absolute time, which a graph would freeze
  if (ctx->has_inlet && ctx->cfg.inlet_noise != 0.0) return false;
  return true;
}

// Refined contexts replay graphs of two coarse steps: level 0's buffer and
// the level-0 record parity flip once per coarse step and every finer level
// advances an even number of times, so after two coarse steps the whole
// schedule is back in the state it was captured from.
static constexpr int64_t kRefinedGraphSteps = 2;

static int step_graph_refined(lbm_ctx* ctx, int64_t chunks, hipStream_t st) {
  const int key = 2 + ctx->lv[0].cur;  // keys 0 / 1 are the single-level graphs
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (!ctx->capture_stream) {
      hipError_t e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_error(e, "hipStreamCreate");
    }
    // the capture runs the host side of the schedule without executing it:
    // keep its state and put it back afterwards
    int cur[kMaxLevels], prev[kMaxLevels];
    int64_t t[kMaxLevels];
    const int64_t t_ctx = ctx->t;
    for (int l = 0; l < ctx->nlevels; ++l) {
      cur[l] = ctx->lv[l].cur;
      t[l] = ctx->lv[l].t;
      prev[l] = l + 1 < ctx->nlevels ? refined_record_parity(ctx, l) : 0;
    }
    hipError_t e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    int rc = LBM_OK;
    for (int64_t s = 0; s < kRefinedGraphSteps && rc == LBM_OK; ++s)
      rc = refined_coarse_step(ctx, ctx->capture_stream);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &graph);
    for (int l = 0; l < ctx->nlevels; ++l) {
      ctx->lv[l].cur = cur[l];
      ctx->lv[l].t = t[l];
      if (l + 1 < ctx->nlevels) set_refined_record_parity(ctx, l, prev[l]);
    }
    ctx->t = t_ctx;
    if (rc != LBM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e2 != hipSuccess) return hip_error(e2, "hipStreamEndCapture");
    GraphEntry g{};
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_error(e, "hipGraphInstantiate");
    }
    it = ctx->graphs.emplace(key, g).first;
  }
  for (int64_t k = 0; k < chunks; ++k) {
    hipError_t e = hipGraphLaunch(it->second.exec, st);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  }
  // even number of coarse steps: every parity is unchanged
  for (int l = 0; l < ctx->nlevels; ++l) ctx->lv[l].t += (chunks * kRefinedGraphSteps) << l;
  ctx->t += chunks * kRefinedGraphSteps;
  return LBM_OK;
}

static int step_graph(lbm_ctx* ctx, int64_t chunks, hipStream_t st) {
  Level& L = ctx->lv[0];
  const int key = L.cur;
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (!ctx->capture_stream) {
      hipError_t e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_error(e, "hipStreamCreate");
    }
    GraphEntry g{};
    hipError_t e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    int buf = L.cur;
    for (int64_t s = 0; s < kGraphSteps; ++s) {
      SweepHost h = sweep_args(ctx, 0, buf, (uint64_t)(L.t + 1 + s));
      e = launch_step_kernel(ctx, h, ctx->block, ctx->capture_stream);
      if (e != hipSuccess) break;
      buf ^= 1;
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (e != hipSuccess) return hip_error(e, "sweep launch during capture");
    if (e2 != hipSuccess) return hip_error(e2, "hipStreamEndCapture");
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_error(e, "hipGraphInstantiate");
    }
    it = ctx->graphs.emplace(key, g).first;
  }
  for (int64_t k = 0; k < chunks; ++k) {
    hipError_t e = hipGraphLaunch(it->second.exec, st);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  }
  // kGraphSteps is even: the buffer parity is unchanged
  L.t += chunks * kGraphSteps;
  ctx->t += chunks * kGraphSteps;
  return LBM_OK;
}

int step_ctx(lbm_ctx* ctx, int64_t n, hipStream_t st) {
  if (n < 0) return set_error(LBM_EINVAL, "negative step count");
  if (n > 1 && has_halo(ctx->cfg))
    return set_error(LBM_EINVAL,
                     "a context with halo faces advances one step per call (the halos are "
                     "exchanged between steps)");
  if (graphs_allowed(ctx) && ctx->nlevels > 1 && n >= kRefinedGraphSteps) {
    const int64_t chunks = n / kRefinedGraphSteps;
    int rc = step_graph_refined(ctx, chunks, st);
    if (rc != LBM_OK) return rc;
    n -= chunks * kRefinedGraphSteps;
  } else if (graphs_allowed(ctx) && ctx->nlevels == 1 && n >= 2 * kGraphSteps) {
    const int64_t chunks = n / kGraphSteps;
    int rc = step_graph(ctx, chunks, st);
    if (rc != LBM_OK) return rc;
    n -= chunks * kGraphSteps;
  }
  return step_eager(ctx, n, st);
}

// Halo faces from the current state of level 0 outside the sweep: send
// buffers always, receive buffers with `entering` (see k_halo_pack).
static int pack_halos(lbm_ctx* ctx, bool entering) {
  const Level& L = ctx->lv[0];
  if (!L.hplane) return LBM_OK;
  HaloArgs a{};
  a.src = L.buf[L.cur];
  for (int side = 0; side < 2; ++side) {
    a.hsend[side] = L.hsend[side];
    a.hrecv[side] = L.hrecv[side];
  }
  a.nx = (uint32_t)L.nx;
  a.ny = (uint32_t)L.ny;
  a.nz = (uint32_t)L.nz;
  a.hplane = L.hplane;
  a.pstride = L.pstride;
  a.entering = entering ? 1 : 0;
  hipError_t e = launch_halo_pack(ctx->cfg.lattice, ctx->cfg.storage, a, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "halo pack launch");
  return LBM_OK;
}

}  // namespace hrlbm

extern "C" {

int lbm_init(lbm_ctx* ctx, int level, const double* rho, const double* u,
             const double* pi_neq, const uint8_t* mask) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  if (level < 0 || level >= ctx->nlevels)
    return set_error(LBM_EINVAL, "level %d of %d", level, ctx->nlevels);
  if (mask && moment_storage(ctx->cfg.storage))
    return set_error(LBM_EINVAL, "moment storage has no cell mask (every cell FLUID)");
  int rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  rc = ensure_memory(ctx);
  if (rc != LBM_OK) return rc;
  Level& L = ctx->lv[level];
  hipError_t e;
  if (!ctx->status_cleared) {
    e = hipMemsetAsync(ctx->status, 0, 256, ctx->stream);
    if (e != hipSuccess) return hip_error(e, "hipMemsetAsync");
    ctx->status_cleared = true;
  }
  InitArgs a{};
  a.rho = rho;
  a.u = u;
  a.pineq = pi_neq;
  a.mask_in = mask;
  a.mask_out = L.mask;
  a.dst0 = L.buf[0];
  a.dst1 = L.buf[1];
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  a.omega1 = 1.0 - 1.0 / L.tau;
  for (int k = 0; k < 3; ++k) a.uin[k] = ctx->uin[k];
  e = moment_storage(ctx->cfg.storage)
          ? launch_minit(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, ctx->stream)
          : launch_init(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, (uint32_t)L.N, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "init launch");
  // any level that is not a fully periodic, sponge-free, unrefined grid
  // keeps a mask (all FLUID if none was given) with the flag bits
  bool general = mask != nullptr || ctx->nlevels > 1 || L.chi_max > 0 ||
                 (ctx->cfg.flags & LBM_SPONGE_FIELD);
  for (int f = 0; f < 6; ++f)
    if (L.face[f] != LBM_PERIODIC && L.face[f] != LBM_HALO) general = true;
  L.has_mask = general;
  if (ctx->nlevels > 1) {
    rc = refined_init_level(ctx, level, rho, u, pi_neq);
    if (rc != LBM_OK) return rc;
  }
  if (general) {
    FlagsArgs fa{};
    fa.mask = L.mask;
    fa.nx = (uint32_t)L.nx;
    fa.ny = (uint32_t)L.ny;
    fa.nz = (uint32_t)L.nz;
    for (int f = 0; f < 6; ++f) fa.face[f] = L.face[f];
    fa.tiles = L.tiles;
    e = launch_flags(ctx->cfg.lattice, fa, ctx->stream);
    if (e != hipSuccess) return hip_error(e, "flags launch");
  }
  if (mask) {
    // inlet cells draw noise: note whether any exist (host scan of a copy)
    std::vector<uint8_t> hm((size_t)L.N);
    e = hipMemcpyAsync(hm.data(), mask, (size_t)L.N, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_error(e, "mask copy");
    for (uint8_t m : hm)
      if (m == LBM_INLET) {
        ctx->has_inlet = true;
        break;
      }
    for (uint8_t m : hm)
      if (m > LBM_INLET) return set_error(LBM_EINVAL, "mask value %u", (unsigned)m);
    // a link across a halo face never meets a wall: the face planes of both
    // subdomains hold no SOLID cell (each side checks its own)
    for (int side = 0; side < 2; ++side) {
      if (!L.hsend[side]) continue;
      const int64_t nl = ctx->cfg.lattice == LBM_D2Q9 ? L.ny : L.nz;
      const size_t c0 = (size_t)(side ? nl - 1 : 0) * L.hplane;
      for (size_t pc = 0; pc < L.hplane; ++pc)
        if (hm[c0 + pc] == LBM_SOLID)
          return set_error(LBM_EINVAL, "SOLID cell on the plane of halo face %d",
                           halo_face(ctx->cfg.lattice, side));
    }
  }
  L.cur = 0;
  L.t = 0;
  L.field_sponge = false;
  L.initialised = true;
  rc = pack_halos(ctx, true);
  if (rc != LBM_OK) return rc;
  if (ctx->cfg.block == 0) {
    const int tb = tuned_block(ctx);
    if (tb > 0) ctx->block = tb;
  }
  ctx->t = 0;
  for (int l = 0; l < ctx->nlevels; ++l) ctx->lv[l].t = 0;
  drop_graphs(ctx);
  bool all = true;
  for (int l = 0; l < ctx->nlevels; ++l) all = all && ctx->lv[l].initialised;
  ctx->initialised = all;
  if (all && ctx->nlevels > 1) return refined_after_init(ctx);
  return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int64_t n) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  return step_ctx(ctx, n, ctx->stream);
}

int lbm_sync(lbm_ctx* ctx) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  int rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  if (!ctx->mem) return LBM_OK;
  int flag = 0;
  e = hipMemcpy(&flag, ctx->status, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "status copy");
  if (flag) ctx->unstable = true;
  if (ctx->unstable)
    return set_error(LBM_EUNSTABLE, "non-finite or non-positive density seen");
  return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* ctx) { return ctx ? ctx->t : -1; }

int lbm_set_time(lbm_ctx* ctx, int64_t t) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (t < 0 || t > (INT64_MAX >> kMaxLevels))
    return set_error(LBM_EINVAL, "time index %lld out of range", (long long)t);
  ctx->t = t;
  for (int l = 0; l < ctx->nlevels; ++l) ctx->lv[l].t = t << l;
  return LBM_OK;
}

int64_t lbm_updates_per_step(const lbm_ctx* ctx) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  return ctx->nlevels > 1 ? refined_updates_per_step(ctx) : ctx->lv[0].N;
}

int lbm_level_shape(const lbm_ctx* ctx, int level, int64_t* nx, int64_t* ny,
                    int64_t* nz) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  if (level < 0 || level >= ctx->nlevels)
    return set_error(LBM_EINVAL, "level %d of %d", level, ctx->nlevels);
  const Level& L = ctx->lv[level];
  if (nx) *nx = L.nx;
  if (ny) *ny = L.ny;
  if (nz) *nz = L.nz;
  return LBM_OK;
}

int lbm_moments(lbm_ctx* ctx, int level, double* rho_out, double* u_out) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels)
    return set_error(LBM_EINVAL, "level %d of %d", level, ctx->nlevels);
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  const Level& L = ctx->lv[level];
  MomentArgs a{};
  a.src = L.buf[L.cur];
  a.mask = L.has_mask ? L.mask : nullptr;
  a.rho_out = rho_out;
  a.u_out = u_out;
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  hipError_t e = moment_storage(ctx->cfg.storage)
                     ? launch_mmoments(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, ctx->stream)
                     : launch_moments(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)L.N,
                                      ctx->stream);
  if (e != hipSuccess) return hip_error(e, "moments launch");
  if (ctx->unstable) return set_error(LBM_EUNSTABLE, "non-finite or non-positive density seen");
  return LBM_OK;
}

int lbm_probe(lbm_ctx* ctx, int level, const int64_t* cells, int n, double* rho_out) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels)
    return set_error(LBM_EINVAL, "level %d of %d", level, ctx->nlevels);
  if (n < 0 || (n > 0 && (!cells || !rho_out)))
    return set_error(LBM_EINVAL, "probe arguments");
  if (n == 0) return LBM_OK;
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  const Level& L = ctx->lv[level];
  ProbeArgs a{};
  a.src = L.buf[L.cur];
  a.mask = L.has_mask ? L.mask : nullptr;
  a.cells = cells;
  a.rho_out = rho_out;
  a.n = n;
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  hipError_t e = moment_storage(ctx->cfg.storage)
                     ? launch_mprobe(ctx->cfg.storage, a, ctx->stream)
                     : launch_probe(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)n, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "probe launch");
  return LBM_OK;
}

int lbm_accumulate(lbm_ctx* ctx, int level, double* sum1, double* sum2) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels)
    return set_error(LBM_EINVAL, "level %d of %d", level, ctx->nlevels);
  if (!sum1 && !sum2) return LBM_OK;
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  const Level& L = ctx->lv[level];
  AccumArgs a{};
  a.src = L.buf[L.cur];
  a.mask = L.has_mask ? L.mask : nullptr;
  a.sum1 = sum1;
  a.sum2 = sum2;
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  hipError_t e = moment_storage(ctx->cfg.storage)
                     ? launch_maccum(ctx->cfg.storage, a, ctx->stream)
                     : launch_accum(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)L.N, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "accumulate launch");
  return LBM_OK;
}

int lbm_set_sponge(lbm_ctx* ctx, int level, const double* chi, const double* rho_ref,
                   const double* u_ref) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels || !chi)
    return set_error(LBM_EINVAL, "level %d / chi", level);
  if (!(ctx->cfg.flags & LBM_SPONGE_FIELD))
    return set_error(LBM_ESTATE, "create the context with LBM_SPONGE_FIELD");
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  Level& L = ctx->lv[level];
  // Sec. II.C: 0 <= chi < 4 tau of the level (checked on a host copy)
  std::vector<double> hc((size_t)L.N);
  hipError_t e = hipMemcpyAsync(hc.data(), chi, (size_t)L.N * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(e, "sponge copy");
  for (double v : hc)
    if (!(v >= 0.0) || !(v < 4.0 * L.tau))
      return set_error(LBM_EINVAL, "sponge chi = %g outside [0, 4 tau = %g)", v, 4.0 * L.tau);
  SpongeArgs a{};
  a.chi = chi;
  a.rho_ref = rho_ref;
  a.u_ref = u_ref;
  a.rho_ref0 = ctx->cfg.rho_ref;
  for (int k = 0; k < 3; ++k)
    a.u_ref0[k] = ctx->cfg.lattice == LBM_D2Q9 && k == 2 ? 0.0 : ctx->cfg.u_ref[k];
  a.sp = L.sp;
  a.mask = L.mask;
  a.n = (uint32_t)L.N;
  e = launch_set_sponge(ctx->cfg.storage, a, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "sponge launch");
  FlagsArgs fa{};
  fa.mask = L.mask;
  fa.tiles = L.tiles;
  fa.nx = (uint32_t)L.nx;
  fa.ny = (uint32_t)L.ny;
  fa.nz = (uint32_t)L.nz;
  e = launch_tiles(fa, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "tiles launch");
  L.field_sponge = true;
  drop_graphs(ctx);
  return LBM_OK;
}

static int reduce_level(lbm_ctx* ctx, int level, double* out, bool totals) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels || !out)
    return set_error(LBM_EINVAL, "level %d / output", level);
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  const Level& L = ctx->lv[level];
  ReduceArgs a{};
  a.src = L.buf[L.cur];
  a.mask = L.has_mask ? L.mask : nullptr;
  a.partial = ctx->reduce;
  a.out = out;
  a.nx = (uint32_t)L.nx;
  a.ny = (uint32_t)L.ny;
  a.nz = (uint32_t)L.nz;
  a.pstride = L.pstride;
  for (int f = 0; f < 6; ++f) a.face[f] = L.face[f];
  a.rho0 = ctx->cfg.rho0;
  hipError_t e;
  if (moment_storage(ctx->cfg.storage))
    e = totals ? launch_mtotals(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, ctx->stream)
               : launch_mforce(a, ctx->stream);
  else
    e = totals ? launch_totals(ctx->cfg.lattice, ctx->cfg.storage, a, ctx->stream)
               : launch_force(ctx->cfg.lattice, ctx->cfg.storage, a, ctx->stream);
  if (e != hipSuccess) return hip_error(e, totals ? "totals launch" : "force launch");
  return LBM_OK;
}

int lbm_force(lbm_ctx* ctx, int level, double* out) {
  return reduce_level(ctx, level, out, false);
}

int lbm_totals(lbm_ctx* ctx, int level, double* out) {
  int rc = reduce_level(ctx, level, out, true);
  if (rc != LBM_OK) return rc;
  if (ctx->unstable) return set_error(LBM_EUNSTABLE, "non-finite or non-positive density seen");
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx* ctx, int level, double* out) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels || !out)
    return set_error(LBM_EINVAL, "level %d / output", level);
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  const Level& L = ctx->lv[level];
  PopArgs a{};
  a.native = L.buf[L.cur];
  a.canon = out;
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  hipError_t e = moment_storage(ctx->cfg.storage)
                     ? launch_mget_pop(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, ctx->stream)
                     : launch_get_pop(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)L.N,
                                      ctx->stream);
  if (e != hipSuccess) return hip_error(e, "get_populations launch");
  return LBM_OK;
}

int lbm_set_populations(lbm_ctx* ctx, int level, const double* in) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level >= ctx->nlevels || !in)
    return set_error(LBM_EINVAL, "level %d / input", level);
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  Level& L = ctx->lv[level];
  PopArgs a{};
  a.native = L.buf[L.cur];
  // SOLID cells are never written by the sweep; keep both buffers equal
  a.native2 = L.buf[L.cur ^ 1];
  a.canon = const_cast<double*>(in);
  a.ncell = (uint32_t)L.N;
  a.pstride = L.pstride;
  a.rho0 = ctx->cfg.rho0;
  hipError_t e = moment_storage(ctx->cfg.storage)
                     ? launch_mset_pop(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, ctx->stream)
                     : launch_set_pop(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)L.N,
                                      ctx->stream);
  if (e != hipSuccess) return hip_error(e, "set_populations launch");
  if (ctx->nlevels > 1) return refined_after_set(ctx, level);
  return pack_halos(ctx, false);
}

size_t lbm_interface_bytes(const lbm_ctx* ctx, int level) {
  if (!ctx || level < 0 || level + 1 >= ctx->nlevels) {
    (void)set_error(LBM_EINVAL, "no refinement interface below level %d", level);
    return 0;
  }
  return refined_interface_bytes(ctx, level);
}

static int interface_io(lbm_ctx* ctx, int level, void* out, const void* in) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (level < 0 || level + 1 >= ctx->nlevels)
    return set_error(LBM_EINVAL, "no refinement interface below level %d", level);
  if (!out && !in) return set_error(LBM_EINVAL, "interface buffer is NULL");
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  return refined_copy_interface(ctx, level, out, in);
}

int lbm_get_interface(lbm_ctx* ctx, int level, void* out) {
  if (!out) return set_error(LBM_EINVAL, "interface output is NULL");
  return interface_io(ctx, level, out, nullptr);
}

int lbm_set_interface(lbm_ctx* ctx, int level, const void* in) {
  if (!in) return set_error(LBM_EINVAL, "interface input is NULL");
  return interface_io(ctx, level, nullptr, in);
}

int lbm_halo_buffers(lbm_ctx* ctx, int side, void** send, void** recv, size_t* bytes) {
  if (!ctx) return set_error(LBM_EINVAL, "ctx is NULL");
  if (side != 0 && side != 1) return set_error(LBM_EINVAL, "side %d: 0 (low) or 1 (high)", side);
  const Level& L = ctx->lv[0];
  if (ctx->cfg.face_bc[halo_face(ctx->cfg.lattice, side)] != LBM_HALO)
    return set_error(LBM_EINVAL, "face %d is not LBM_HALO", halo_face(ctx->cfg.lattice, side));
  if (!ctx->mem) return set_error(LBM_ESTATE, "no device memory yet (call lbm_init)");
  if (send) *send = L.hsend[side];
  if (recv) *recv = L.hrecv[side];
  if (bytes)
    *bytes = (size_t)halo_count_of(ctx->cfg.lattice) * L.hplane * storage_bytes(ctx->cfg.storage);
  return LBM_OK;
}

int lbm_halo_exchange(lbm_ctx* const* ctxs, int n, int periodic) {
  if (n < 1 || !ctxs) return set_error(LBM_EINVAL, "exchange arguments");
  for (int k = 0; k < n; ++k) {
    int rc = check_ready(ctxs[k]);
    if (rc != LBM_OK) return rc;
    const lbm_config &c = ctxs[k]->cfg, &c0 = ctxs[0]->cfg;
    if (ctxs[k]->device != ctxs[0]->device || ctxs[k]->stream != ctxs[0]->stream)
      return set_error(LBM_EINVAL, "exchanged contexts must share device and stream");
    if (c.lattice != c0.lattice || c.storage != c0.storage || c.nx != c0.nx ||
        (c.lattice != LBM_D2Q9 && c.ny != c0.ny) || c.rho0 != c0.rho0)
      return set_error(LBM_EINVAL, "context %d: lattice, storage, rho0 or face plane differs", k);
    const bool lo_needed = k > 0 || periodic, hi_needed = k < n - 1 || periodic;
    if ((lo_needed && !ctxs[k]->lv[0].hrecv[0]) || (hi_needed && !ctxs[k]->lv[0].hrecv[1]))
      return set_error(LBM_EINVAL, "context %d lacks a halo face the chain needs", k);
  }
  int rc = ensure_device(ctxs[0]);
  if (rc != LBM_OK) return rc;
  size_t bytes = 0;
  rc = lbm_halo_buffers(ctxs[0], ctxs[0]->lv[0].hrecv[0] ? 0 : 1, nullptr, nullptr, &bytes);
  if (rc != LBM_OK) return rc;
  // subdomain k + 1 lies above k; with `periodic` subdomain 0 lies above n - 1
  const int pairs = periodic ? n : n - 1;
  for (int k = 0; k < pairs; ++k) {
    const Level& below = ctxs[k]->lv[0];
    const Level& above = ctxs[(k + 1) % n]->lv[0];
    hipError_t e = hipMemcpyAsync(above.hrecv[0], below.hsend[1], bytes,
                                  hipMemcpyDeviceToDevice, ctxs[0]->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(below.hrecv[1], above.hsend[0], bytes, hipMemcpyDeviceToDevice,
                         ctxs[0]->stream);
    if (e != hipSuccess) return hip_error(e, "halo copy");
  }
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  if (ensure_device(ctx) == LBM_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->owns_mem && ctx->mem) (void)hipFree(ctx->mem);
  }
  delete ctx;
}

int lbm_lattice_table(int lattice, int32_t* xi, double* w) {
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q27)
    return set_error(LBM_EINVAL, "unknown lattice %d", lattice);
  for (int i = 0; i < lattice; ++i) {
    Dir d{};
    double wi = 0;
    switch (lattice) {
      case 9: d = Lattice<9>::dir(i); wi = Lattice<9>::w(i); break;
      case 19: d = Lattice<19>::dir(i); wi = Lattice<19>::w(i); break;
      default: d = Lattice<27>::dir(i); wi = Lattice<27>::w(i); break;
    }
    if (xi) {
      xi[3 * i] = d.x;
      xi[3 * i + 1] = d.y;
      xi[3 * i + 2] = d.z;
    }
    if (w) w[i] = wi;
  }
  return lattice;
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
