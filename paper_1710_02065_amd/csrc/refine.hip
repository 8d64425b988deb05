// Nested 2:1 multi-domain grid refinement (Sec. II.B): configuration
// checks, the refined levels, interface buffers and the recursive schedule.
//
// Layout: level l + 1 covers the closed node box [lo, hi] of level l with
// half the spacing (its node k at level-l coordinate lo + k/2), so an axis
// has 2 (hi - lo) + 1 nodes.  Its outer shell (RING) is rebuilt from level-l
// moments; level-l nodes on the shell of [lo+1, hi-1] (IMPORT) are rebuilt
// from level-(l+1) moments; level-l nodes deeper inside are COVERED and not
// updated.  tau_(l+1) = (4 tau_l - 1) / 2 keeps the physical viscosity.
// The paper's setups nest four and five levels this way.
//
// One step of level l (level-l time t -> t+1), recursively:
//   1. sweep level l; it records its pre-collision moments M_l(t+1) on the
//      boundary planes of its child's box;
//   2. if level l has a child: step the child, whose sweep sets its RING
//      to M_l(t + 1/2) = (M_l(t) + M_l(t+1)) / 2; step the child again, its
//      sweep recording its pre-collision moments in the import band and
//      setting the RING to M_l(t+1); IMPORT <- filtered child moments.
//      (The RING nodes are read only by the child's next sweep, so writing
//      them in the sweep that produces that state equals filling them after
//      it.)
#include <hip/hip_runtime.h>

#include <vector>

#include "runtime.hpp"

lbm_ctx::~lbm_ctx() { hrlbm::free_refinement(this); }

namespace hrlbm {

// Coupling between level l (parent) and level l + 1 (child).
struct Refinement {
  int dim = 3;
  int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // child box, parent coordinates
  // parent-side record of M_l on the box boundary planes
  int32_t rec_off[3] = {0, 0, 0};
  uint32_t rec_dim[3] = {1, 1, 1};
  uint32_t rec_n = 0;
  size_t rec_bytes = 0;  // one record buffer (10 components)
  size_t off_rec[2] = {0, 0}, off_ring = 0, off_import = 0, off_recf = 0;
  void* rec[2] = {nullptr, nullptr};
  int prev = 0;  // rec[prev] = M_l(t), rec[prev ^ 1] = M_l(t+1)
  // child-side record of the import band (10 components over every child node)
  size_t recf_bytes = 0;
  void* recf = nullptr;
  std::vector<uint32_t> ring, import_;
  uint32_t* d_ring = nullptr;
  uint32_t* d_import = nullptr;
  int64_t n_covered = 0;
};

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// box k of the chain: k = 0 is refine_lo/hi (in level-0 coordinates),
// k >= 1 is nest k - 1 (in level-k coordinates)
static void box_of(const lbm_config& c, int k, int64_t lo[3], int64_t hi[3]) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = k == 0 ? c.refine_lo[a] : c.nest_lo[k - 1][a];
    hi[a] = k == 0 ? c.refine_hi[a] : c.nest_hi[k - 1][a];
  }
}

int validate_refinement(const lbm_config& c) {
  const int d = lattice_dim(c.lattice);
  int64_t n[3] = {c.nx, c.ny, c.nz};  // dimensions of the current parent level
  for (int k = 0; k <= c.nest_count; ++k) {
    int64_t blo[3], bhi[3];
    box_of(c, k, blo, bhi);
    if (d == 2 && (blo[2] != 0 || bhi[2] != 0))
      return set_error(LBM_EINVAL, "D2Q9 refinement box %d must have z range [0, 0]", k);
    int64_t fcells = 1, fn[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
      const int64_t lo = blo[a], hi = bhi[a];
      if (hi - lo < 4)
        return set_error(LBM_EINVAL, "refinement box %d axis %d: [%lld, %lld] spans < 4 cells",
                         k, a, (long long)lo, (long long)hi);
      // interpolation stencils, the parent's pull and the band the child's
      // own IMPORT nodes need: 4 nodes of margin on every side
      if (lo < 4 || hi > n[a] - 5)
        return set_error(LBM_EINVAL,
                         "refinement box %d axis %d: [%lld, %lld] must lie in [4, %lld]", k, a,
                         (long long)lo, (long long)hi, (long long)(n[a] - 5));
      if (k == 0) {
        const int32_t wl = c.sponge_width[2 * a], wh = c.sponge_width[2 * a + 1];
        if ((wl > 0 && lo < wl) || (wh > 0 && hi > n[a] - wh - 1))
          return set_error(LBM_EINVAL, "refinement box axis %d overlaps an absorbing layer", a);
      }
      fn[a] = 2 * (hi - lo) + 1;
      fcells *= fn[a];
    }
    if (fcells > 2147483647LL ||
        (double)pop_stride((uint64_t)fcells) * (double)storage_bytes(c.storage) > 4294967040.0)
      return set_error(LBM_EINVAL, "level %d has %lld cells: above the per-level limit", k + 1,
                       (long long)fcells);
    for (int a = 0; a < 3; ++a) n[a] = fn[a];
  }
  return LBM_OK;
}

int make_levels_refined(lbm_ctx* ctx) {
  const lbm_config& c = ctx->cfg;
  const int d = lattice_dim(c.lattice);
  ctx->nlevels = 2 + c.nest_count;
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    Refinement* R = ctx->ref[l] ? ctx->ref[l] : new Refinement();
    ctx->ref[l] = R;
    R->dim = d;
    const Level& P = ctx->lv[l];
    Level& F = ctx->lv[l + 1];
    int64_t blo[3], bhi[3], fn[3] = {1, 1, 1};
    box_of(c, l, blo, bhi);
    for (int a = 0; a < 3; ++a) {
      R->lo[a] = (int32_t)blo[a];
      R->hi[a] = (int32_t)bhi[a];
      if (a < d) {
        fn[a] = 2 * (bhi[a] - blo[a]) + 1;
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
    F.tau = (4.0 * P.tau - 1.0) / 2.0;
    F.level = l + 1;
    F.chi_max = 0.0;
    for (int f = 0; f < 6; ++f) {
      // RING nodes shield the child's faces; the rule is never exercised
      F.face[f] = (d == 2 && f >= 4) ? LBM_PERIODIC : LBM_OUTFLOW;
      F.sponge[f] = 0;
    }
    // index lists: RING of the child, IMPORT of the parent
    R->ring.clear();
    R->import_.clear();
    for (int64_t z = 0; z < F.nz; ++z)
      for (int64_t y = 0; y < F.ny; ++y)
        for (int64_t x = 0; x < F.nx; ++x) {
          bool ring = x == 0 || x == F.nx - 1 || y == 0 || y == F.ny - 1;
          if (d == 3) ring = ring || z == 0 || z == F.nz - 1;
          if (ring) R->ring.push_back((uint32_t)((z * F.ny + y) * F.nx + x));
        }
    int64_t covered = 0;
    for (int64_t z = 0; z < P.nz; ++z)
      for (int64_t y = 0; y < P.ny; ++y)
        for (int64_t x = 0; x < P.nx; ++x) {
          const int64_t p[3] = {x, y, z};
          bool inside = true, deep = true;
          for (int a = 0; a < d; ++a) {
            if (p[a] < R->lo[a] + 1 || p[a] > R->hi[a] - 1) inside = false;
            if (p[a] < R->lo[a] + 2 || p[a] > R->hi[a] - 2) deep = false;
          }
          if (inside && !deep) R->import_.push_back((uint32_t)((z * P.ny + y) * P.nx + x));
          if (inside && deep) ++covered;
        }
    R->n_covered = covered;
  }
  return LBM_OK;
}

size_t plan_interface_layout(lbm_ctx* ctx, size_t off) {
  const size_t rsz = ctx->cfg.storage == LBM_F64 ? 8 : 4;
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    Refinement* R = ctx->ref[l];
    R->rec_bytes = align256((size_t)R->rec_n * 10 * rsz);
    R->off_rec[0] = off;
    R->off_rec[1] = off + R->rec_bytes;
    off += 2 * R->rec_bytes;
    R->off_ring = off;
    off += align256(R->ring.size() * sizeof(uint32_t));
    R->off_import = off;
    off += align256(R->import_.size() * sizeof(uint32_t));
    R->recf_bytes = align256((size_t)ctx->lv[l + 1].N * 10 * rsz);
    R->off_recf = off;
    off += R->recf_bytes;
  }
  return off;
}

void assign_interface_pointers(lbm_ctx* ctx) {
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    Refinement* R = ctx->ref[l];
    R->rec[0] = ctx->mem + R->off_rec[0];
    R->rec[1] = ctx->mem + R->off_rec[1];
    R->d_ring = (uint32_t*)(ctx->mem + R->off_ring);
    R->d_import = (uint32_t*)(ctx->mem + R->off_import);
    R->recf = ctx->mem + R->off_recf;
  }
}

// Index lists to the device and the band record cleared (the oracle's
// record starts at zero too); when the parent level is initialised.
static int upload_interface(lbm_ctx* ctx, int l) {
  Refinement* R = ctx->ref[l];
  hipError_t e = hipMemcpyAsync(R->d_ring, R->ring.data(), R->ring.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(R->d_import, R->import_.data(), R->import_.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(R->recf, 0, R->recf_bytes, ctx->stream);
  // the host vectors are read by the copies: wait before returning
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(e, "refinement interface upload");
  return LBM_OK;
}

// Called by lbm_init for one level of a refined context, after the
// population initialisation: marks roles in the mask and, on a level with a
// child, records M(0) from the initial fields.
int refined_init_level(lbm_ctx* ctx, int level, const double* rho, const double* u,
                       const double* pineq) {
  Level& L = ctx->lv[level];
  const bool has_child = level + 1 < ctx->nlevels;
  RolesArgs ra{};
  ra.mask = L.mask;
  ra.nx = (uint32_t)L.nx;
  ra.ny = (uint32_t)L.ny;
  ra.nz = (uint32_t)L.nz;
  ra.ring = level > 0;
  ra.child = has_child;
  ra.dim = lattice_dim(ctx->cfg.lattice);
  if (has_child)
    for (int a = 0; a < 3; ++a) {
      ra.lo[a] = ctx->ref[level]->lo[a];
      ra.hi[a] = ctx->ref[level]->hi[a];
    }
  hipError_t e = launch_roles(ra, (uint32_t)L.N, ctx->stream);
  if (e != hipSuccess) return hip_error(e, "roles launch");
  L.has_mask = true;
  if (has_child) {
    Refinement* R = ctx->ref[level];
    int rc = upload_interface(ctx, level);
    if (rc != LBM_OK) return rc;
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

// RING of level l + 1 from level-l moments wa Ma + wb Mb.
static int fill_ring(lbm_ctx* ctx, int l, const void* Ma, double wa, const void* Mb, double wb,
                     hipStream_t st) {
  Refinement* R = ctx->ref[l];
  const Level& F = ctx->lv[l + 1];
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
  a.alpha = F.tau / (2.0 * ctx->lv[l].tau);
  a.omega1 = 1.0 - 1.0 / F.tau;
  a.rho0 = ctx->cfg.rho0;
  a.dst = F.buf[F.cur];
  a.pstride = F.pstride;
  hipError_t e = launch_ring(kernel_lattice(ctx->cfg), ctx->cfg.storage, a, a.n, st);
  if (e != hipSuccess) return hip_error(e, "ring launch");
  return LBM_OK;
}

int refined_after_init(lbm_ctx* ctx) {
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    Refinement* R = ctx->ref[l];
    int rc = fill_ring(ctx, l, R->rec[R->prev], 1.0, R->rec[R->prev], 0.0, ctx->stream);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int refined_after_set(lbm_ctx*, int) { return LBM_OK; }

// The RING state a child sweep writes: wa * Ma + wb * Mb of its parent's
// recorded moments.
struct RingSource {
  const void* Ma;
  const void* Mb;
  double wa, wb;
};

// One step of level l and, recursively, two of each finer level.
// record_band: this is the second step of level l within its parent's
// step, whose pre-collision moments the parent's IMPORT nodes filter.
// ring: the time blend of the parent's records the sweep of level l writes
// into its RING nodes for the state it produces (nullptr on level 0).
static int advance(lbm_ctx* ctx, int l, bool record_band, const RingSource* ring,
                   hipStream_t st) {
  Level& L = ctx->lv[l];
  const bool has_child = l + 1 < ctx->nlevels;
  Refinement* R = has_child ? ctx->ref[l] : nullptr;
  const int next = R ? R->prev ^ 1 : 0;
  // 1. sweep of level l (its RING nodes rebuilt by the same sweep)
  SweepHost h = sweep_args(ctx, l, L.cur, (uint64_t)(L.t + 1));
  if (ring) {
    const Refinement* P = ctx->ref[l - 1];
    h.ring_Ma = ring->Ma;
    h.ring_Mb = ring->Mb;
    h.ring_wa = ring->wa;
    h.ring_wb = ring->wb;
    h.ring_alpha = L.tau / (2.0 * ctx->lv[l - 1].tau);
    for (int k = 0; k < 3; ++k) {
      h.ring_lo[k] = P->lo[k];
      h.ring_off[k] = P->rec_off[k];
      h.ring_dim[k] = P->rec_dim[k];
    }
  }
  if (R) {
    h.rec = R->rec[next];
    for (int k = 0; k < 3; ++k) {
      h.rec_off[k] = R->rec_off[k];
      h.rec_dim[k] = R->rec_dim[k];
      h.box_lo[k] = R->lo[k];
      h.box_hi[k] = R->hi[k];
    }
    h.rec_n = R->rec_n;
  }
  if (record_band) h.recf = ctx->ref[l - 1]->recf;
  hipError_t e = launch_sweep(sweep_lattice(ctx->cfg), ctx->cfg.storage, h, ctx->block, st);
  if (e != hipSuccess) return hip_error(e, "sweep launch");
  L.cur ^= 1;
  L.t += 1;
  if (!R) return LBM_OK;
  // 2. two child steps; their sweeps set the RING at t + 1/2 and t + 1
  //    (the parent's record of M_l(t + 1) is complete: step 1 wrote it)
  const RingSource half{R->rec[R->prev], R->rec[next], 0.5, 0.5};
  const RingSource full{R->rec[next], R->rec[next], 1.0, 0.0};
  int rc = advance(ctx, l + 1, false, &half, st);
  if (rc != LBM_OK) return rc;
  rc = advance(ctx, l + 1, true, &full, st);
  if (rc != LBM_OK) return rc;
  //    IMPORT from the child's pre-collision moments at the common time
  const Level& F = ctx->lv[l + 1];
  ImportArgs ia{};
  ia.list = R->d_import;
  ia.n = (uint32_t)R->import_.size();
  ia.cnx = (uint32_t)L.nx;
  ia.cny = (uint32_t)L.ny;
  for (int k = 0; k < 3; ++k) ia.lo[k] = R->lo[k];
  ia.recf = R->recf;
  ia.fnx = (uint32_t)F.nx;
  ia.fny = (uint32_t)F.ny;
  ia.fnz = (uint32_t)F.nz;
  ia.alpha = 2.0 * L.tau / F.tau;
  ia.omega1 = 1.0 - 1.0 / L.tau;
  ia.rho0 = ctx->cfg.rho0;
  ia.dst = L.buf[L.cur];
  ia.pstride = L.pstride;
  e = launch_import(kernel_lattice(ctx->cfg), ctx->cfg.storage, ia, ia.n, st);
  if (e != hipSuccess) return hip_error(e, "import launch");
  R->prev = next;
  return LBM_OK;
}

// Interface state between coarse steps: the two parent-side records
// (M_l(t) first, then the other one), each rec_n nodes x 10 components of
// the record type.  The band record is not state: the child's second sweep
// rewrites every entry the IMPORT filter reads before the filter runs.
static size_t interface_record_bytes(const lbm_ctx* ctx, const Refinement* R) {
  return (size_t)R->rec_n * 10 * (ctx->cfg.storage == LBM_F64 ? 8 : 4);
}

size_t refined_interface_bytes(const lbm_ctx* ctx, int l) {
  return 2 * interface_record_bytes(ctx, ctx->ref[l]);
}

int refined_copy_interface(lbm_ctx* ctx, int l, void* out, const void* in) {
  Refinement* R = ctx->ref[l];
  const size_t b = interface_record_bytes(ctx, R);
  for (int k = 0; k < 2; ++k) {
    void* rec = R->rec[R->prev ^ k];
    hipError_t e = out ? hipMemcpyAsync((char*)out + k * b, rec, b, hipMemcpyDeviceToDevice,
                                        ctx->stream)
                       : hipMemcpyAsync(rec, (const char*)in + k * b, b,
                                        hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return hip_error(e, "interface record copy");
  }
  return LBM_OK;
}

int refined_record_parity(const lbm_ctx* ctx, int l) { return ctx->ref[l]->prev; }

void set_refined_record_parity(lbm_ctx* ctx, int l, int parity) { ctx->ref[l]->prev = parity; }

int refined_coarse_step(lbm_ctx* ctx, hipStream_t st) {
  int rc = advance(ctx, 0, false, nullptr, st);
  if (rc != LBM_OK) return rc;
  ctx->t += 1;
  return LBM_OK;
}

int64_t refined_updates_per_step(const lbm_ctx* ctx) {
  int64_t total = 0;
  for (int l = 0; l < ctx->nlevels; ++l) {
    int64_t swept = ctx->lv[l].N;
    if (l > 0) swept -= (int64_t)ctx->ref[l - 1]->ring.size();
    if (l + 1 < ctx->nlevels)
      swept -= ctx->ref[l]->n_covered + (int64_t)ctx->ref[l]->import_.size();
    total += swept << l;
  }
  return total;
}

void free_refinement(lbm_ctx* ctx) {
  for (int l = 0; l + 1 < kMaxLevels; ++l) {
    delete ctx->ref[l];
    ctx->ref[l] = nullptr;
  }
}

}  // namespace hrlbm
