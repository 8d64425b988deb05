// Two-level 2:1 multi-domain grid refinement (Sec. II.B): configuration
// checks, the fine level, interface buffers and the per-coarse-step schedule.
//
// Layout: the fine level covers the closed coarse-node box [lo, hi] with
// half the spacing (fine node k at coarse coordinate lo + k/2), so an axis
// has 2 (hi - lo) + 1 fine nodes.  Its outer shell (RING) is rebuilt from
// coarse moments; coarse nodes on the shell of [lo+1, hi-1] (IMPORT) are
// rebuilt from fine moments; coarse nodes deeper inside are COVERED and not
// updated.  tau_f = (4 tau_c - 1) / 2 keeps the physical viscosity.
//
// One coarse step (fine time 2t -> 2t+2):
//   1. coarse sweep; records coarse pre-collision moments M(t+1) on the
//      patch boundary planes;
//   2. fine sweep;  3. RING <- M(t + 1/2) = (M(t) + M(t+1)) / 2;
//   4. fine sweep;  5. RING <- M(t+1);
//   6. IMPORT <- fine moments (pulled from the fine state of step 2).
#include <hip/hip_runtime.h>

#include <vector>

#include "runtime.hpp"

lbm_ctx::~lbm_ctx() { hrlbm::free_refinement(this); }

namespace hrlbm {

struct Refinement {
  int dim = 3;
  int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int32_t rec_off[3] = {0, 0, 0};
  uint32_t rec_dim[3] = {1, 1, 1};
  uint32_t rec_n = 0;
  size_t rec_bytes = 0;  // one record buffer (10 components)
  size_t off_rec[2] = {0, 0}, off_ring = 0, off_import = 0;
  void* rec[2] = {nullptr, nullptr};
  int prev = 0;  // rec[prev] = M(t), rec[prev ^ 1] = M(t+1)
  std::vector<uint32_t> ring, import_;
  uint32_t* d_ring = nullptr;
  uint32_t* d_import = nullptr;
  bool lists_uploaded = false;
  int64_t n_normal = 0, n_fine_active = 0;
};

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

int validate_refinement(const lbm_config& c) {
  const int d = lattice_dim(c.lattice);
  const int64_t n[3] = {c.nx, c.ny, c.nz};
  if (d == 2 && (c.refine_lo[2] != 0 || c.refine_hi[2] != 0))
    return set_error(LBM_EINVAL, "D2Q9 refinement box must have z range [0, 0]");
  int64_t fcells = 1;
  for (int a = 0; a < d; ++a) {
    const int64_t lo = c.refine_lo[a], hi = c.refine_hi[a];
    if (hi - lo < 4)
      return set_error(LBM_EINVAL, "refinement box axis %d: [%lld, %lld] spans < 4 cells", a,
                       (long long)lo, (long long)hi);
    // interpolation stencils and the coarse pull need 4 coarse nodes of
    // margin on every side
    if (lo < 4 || hi > n[a] - 5)
      return set_error(LBM_EINVAL,
                       "refinement box axis %d: [%lld, %lld] must lie in [4, %lld]", a,
                       (long long)lo, (long long)hi, (long long)(n[a] - 5));
    const int32_t wl = c.sponge_width[2 * a], wh = c.sponge_width[2 * a + 1];
    if ((wl > 0 && lo < wl) || (wh > 0 && hi > n[a] - wh - 1))
      return set_error(LBM_EINVAL, "refinement box axis %d overlaps an absorbing layer", a);
    fcells *= 2 * (hi - lo) + 1;
  }
  if (fcells > 2147483647LL ||
      (double)pop_stride((uint64_t)fcells) * (double)storage_bytes(c.storage) > 4294967040.0)
    return set_error(LBM_EINVAL, "fine level has %lld cells: above the per-level limit",
                     (long long)fcells);
  return LBM_OK;
}

int make_fine_level(lbm_ctx* ctx) {
  const lbm_config& c = ctx->cfg;
  const int d = lattice_dim(c.lattice);
  Refinement* R = ctx->ref ? ctx->ref : new Refinement();
  ctx->ref = R;
  R->dim = d;
  Level& F = ctx->lv[1];
  int64_t fn[3] = {1, 1, 1};
  for (int a = 0; a < 3; ++a) {
    R->lo[a] = (int32_t)c.refine_lo[a];
    R->hi[a] = (int32_t)c.refine_hi[a];
    if (a < d) {
      fn[a] = 2 * (c.refine_hi[a] - c.refine_lo[a]) + 1;
      R->rec_off[a] = R->lo[a] - 1;
      R->rec_dim[a] = (uint32_t)(R->hi[a] - R->lo[a] + 3);
    } else {
      R->rec_off[a] = 0;
      R->rec_dim[a] = 1;
    }
  }
  R->rec_n = R->rec_dim[0] * R->rec_dim[1] * R->rec_dim[2];
  F.nx = fn[0];
  F.ny = fn[1];
  F.nz = fn[2];
  F.N = fn[0] * fn[1] * fn[2];
  F.tau = (4.0 * c.tau - 1.0) / 2.0;
  F.level = 1;
  F.chi_max = 0.0;
  for (int f = 0; f < 6; ++f) {
    // RING nodes shield the fine faces; the rule is never exercised
    F.face[f] = (d == 2 && f >= 4) ? LBM_PERIODIC : LBM_OUTFLOW;
    F.sponge[f] = 0;
  }
  ctx->nlevels = 2;
  // index lists
  R->ring.clear();
  R->import_.clear();
  for (int64_t z = 0; z < F.nz; ++z)
    for (int64_t y = 0; y < F.ny; ++y)
      for (int64_t x = 0; x < F.nx; ++x) {
        bool ring = x == 0 || x == F.nx - 1 || y == 0 || y == F.ny - 1;
        if (d == 3) ring = ring || z == 0 || z == F.nz - 1;
        if (ring) R->ring.push_back((uint32_t)((z * F.ny + y) * F.nx + x));
      }
  const Level& C = ctx->lv[0];
  int64_t covered = 0;
  for (int64_t z = 0; z < C.nz; ++z)
    for (int64_t y = 0; y < C.ny; ++y)
      for (int64_t x = 0; x < C.nx; ++x) {
        const int64_t p[3] = {x, y, z};
        bool inside = true, deep = true;
        for (int a = 0; a < d; ++a) {
          if (p[a] < R->lo[a] + 1 || p[a] > R->hi[a] - 1) inside = false;
          if (p[a] < R->lo[a] + 2 || p[a] > R->hi[a] - 2) deep = false;
        }
        if (inside && !deep) R->import_.push_back((uint32_t)((z * C.ny + y) * C.nx + x));
        if (inside && deep) ++covered;
      }
  R->n_normal = C.N - covered - (int64_t)R->import_.size();
  R->n_fine_active = F.N - (int64_t)R->ring.size();
  return LBM_OK;
}

size_t plan_interface_layout(lbm_ctx* ctx, size_t off) {
  Refinement* R = ctx->ref;
  if (!R || ctx->nlevels < 2) return off;
  const size_t rsz = ctx->cfg.storage == LBM_F64 ? 8 : 4;
  R->rec_bytes = align256((size_t)R->rec_n * 10 * rsz);
  R->off_rec[0] = off;
  R->off_rec[1] = off + R->rec_bytes;
  off += 2 * R->rec_bytes;
  R->off_ring = off;
  off += align256(R->ring.size() * sizeof(uint32_t));
  R->off_import = off;
  off += align256(R->import_.size() * sizeof(uint32_t));
  ctx->ref_off = R->off_rec[0];
  ctx->ref_bytes = off - R->off_rec[0];
  return off;
}

void assign_interface_pointers(lbm_ctx* ctx) {
  Refinement* R = ctx->ref;
  if (!R || ctx->nlevels < 2) return;
  R->rec[0] = ctx->mem + R->off_rec[0];
  R->rec[1] = ctx->mem + R->off_rec[1];
  R->d_ring = (uint32_t*)(ctx->mem + R->off_ring);
  R->d_import = (uint32_t*)(ctx->mem + R->off_import);
  R->lists_uploaded = false;
}

static int upload_lists(lbm_ctx* ctx) {
  Refinement* R = ctx->ref;
  if (R->lists_uploaded) return LBM_OK;
  hipError_t e = hipMemcpyAsync(R->d_ring, R->ring.data(), R->ring.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(R->d_import, R->import_.data(), R->import_.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(e, "refinement index upload");
  R->lists_uploaded = true;
  return LBM_OK;
}

// Called by lbm_init for one level of a refined context, after the
// population initialisation: marks roles in the mask and, on the coarse
// level, records M(0) from the initial fields.
int refined_init_level(lbm_ctx* ctx, int level, const double* rho, const double* u,
                       const double* pineq) {
  Refinement* R = ctx->ref;
  int rc = upload_lists(ctx);
  if (rc != LBM_OK) return rc;
  Level& L = ctx->lv[level];
  RolesArgs ra{};
  ra.mask = L.mask;
  ra.nx = (uint32_t)L.nx;
  ra.ny = (uint32_t)L.ny;
  ra.nz = (uint32_t)L.nz;
  ra.level = level;
  ra.dim = R->dim;
  for (int a = 0; a < 3; ++a) {
    ra.lo[a] = R->lo[a];
    ra.hi[a] = R->hi[a];
  }
  hipError_t e = launch_roles(ra, (uint32_t)L.N, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "roles launch");
  L.has_mask = true;
  if (level == 0) {
    RecordFieldsArgs a{};
    a.rho = rho;
    a.u = u;
    a.pineq = pineq;
    a.rec_a = R->rec[0];
    a.rec_b = R->rec[1];
    a.nx = (uint32_t)L.nx;
    a.ny = (uint32_t)L.ny;
    a.nz = (uint32_t)L.nz;
    for (int k = 0; k < 3; ++k) {
      a.rec_off[k] = R->rec_off[k];
      a.rec_dim[k] = R->rec_dim[k];
      a.box_lo[k] = R->lo[k];
      a.box_hi[k] = R->hi[k];
      a.uin[k] = ctx->uin[k];
    }
    a.rec_n = R->rec_n;
    a.rho0 = ctx->cfg.rho0;
    e = launch_record_fields(ctx->cfg.lattice, ctx->cfg.storage, a, (uint32_t)L.N, ctx->stream);
    if (e != hipSuccess) return hip_error(e, "record launch");
    R->prev = 0;
  }
  return LBM_OK;
}

static int fill_ring(lbm_ctx* ctx, const void* Ma, double wa, const void* Mb, double wb,
                     hipStream_t st) {
  Refinement* R = ctx->ref;
  const Level& F = ctx->lv[1];
  RingArgs a{};
  a.list = R->d_ring;
  a.n = (uint32_t)R->ring.size();
  a.fnx = (uint32_t)F.nx;
  a.fny = (uint32_t)F.ny;
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = R->lo[k];
    a.rec_off[k] = R->rec_off[k];
    a.rec_dim[k] = R->rec_dim[k];
  }
  a.Ma = Ma;
  a.Mb = Mb;
  a.wa = wa;
  a.wb = wb;
  a.rec_n = R->rec_n;
  a.alpha = F.tau / (2.0 * ctx->lv[0].tau);
  a.omega1 = 1.0 - 1.0 / F.tau;
  a.rho0 = ctx->cfg.rho0;
  a.dst = F.buf[F.cur];
  a.pstride = F.pstride;
  hipError_t e = launch_ring(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, a.n, st);
  if (e != hipSuccess) return hip_error(e, "ring launch");
  return LBM_OK;
}

int refined_after_init(lbm_ctx* ctx) {
  Refinement* R = ctx->ref;
  return fill_ring(ctx, R->rec[R->prev], 1.0, R->rec[R->prev], 0.0, ctx->stream);
}

int refined_after_set(lbm_ctx*, int) { return LBM_OK; }

int refined_coarse_step(lbm_ctx* ctx, hipStream_t st) {
  Refinement* R = ctx->ref;
  Level& C = ctx->lv[0];
  Level& F = ctx->lv[1];
  const int next = R->prev ^ 1;
  // 1. coarse sweep recording M(t+1)
  SweepHost h = sweep_args(ctx, 0, C.cur, (uint64_t)(C.t + 1));
  h.rec = R->rec[next];
  for (int k = 0; k < 3; ++k) {
    h.rec_off[k] = R->rec_off[k];
    h.rec_dim[k] = R->rec_dim[k];
    h.box_lo[k] = R->lo[k];
    h.box_hi[k] = R->hi[k];
  }
  h.rec_n = R->rec_n;
  hipError_t e = launch_sweep(kernel_lattice(ctx->cfg), ctx->cfg.storage, h, ctx->block, st);
  if (e != hipSuccess) return hip_error(e, "coarse sweep launch");
  C.cur ^= 1;
  C.t += 1;
  // 2. fine sweep 2t -> 2t+1
  int rc = sweep_level(ctx, 1, st);
  if (rc != LBM_OK) return rc;
  // 3. RING at t + 1/2
  rc = fill_ring(ctx, R->rec[R->prev], 0.5, R->rec[next], 0.5, st);
  if (rc != LBM_OK) return rc;
  // 4. fine sweep 2t+1 -> 2t+2
  rc = sweep_level(ctx, 1, st);
  if (rc != LBM_OK) return rc;
  // 5. RING at t + 1
  rc = fill_ring(ctx, R->rec[next], 1.0, R->rec[next], 0.0, st);
  if (rc != LBM_OK) return rc;
  // 6. IMPORT from the fine pre-collision moments at 2t+2, pulled from the
  //    fine state at 2t+1 (the buffer the second fine sweep read)
  ImportArgs ia{};
  ia.list = R->d_import;
  ia.n = (uint32_t)R->import_.size();
  ia.cnx = (uint32_t)C.nx;
  ia.cny = (uint32_t)C.ny;
  for (int k = 0; k < 3; ++k) ia.lo[k] = R->lo[k];
  ia.fine = sweep_args(ctx, 1, F.cur ^ 1, (uint64_t)F.t);
  ia.alpha = 2.0 * C.tau / F.tau;
  ia.omega1 = 1.0 - 1.0 / C.tau;
  ia.rho0 = ctx->cfg.rho0;
  ia.dst = C.buf[C.cur];
  ia.pstride = C.pstride;
  e = launch_import(kernel_lattice(ctx->cfg), ctx->cfg.storage, ia, ia.n, st);
  if (e != hipSuccess) return hip_error(e, "import launch");
  R->prev = next;
  ctx->t += 1;
  return LBM_OK;
}

int64_t refined_updates_per_step(const lbm_ctx* ctx) {
  const Refinement* R = ctx->ref;
  return R ? R->n_normal + 2 * R->n_fine_active : ctx->lv[0].N;
}

void free_refinement(lbm_ctx* ctx) {
  delete ctx->ref;
  ctx->ref = nullptr;
}

}  // namespace hrlbm
