/*
 * lbm.h -- C ABI of the MI355X (gfx950) Hermite-regularized lattice Boltzmann
 * library.
 *
 * The method is the recursive-regularized BGK scheme ("rrBGK") of Brogi,
 * Malaspinas, Chopard & Bonadonna, "Hermite regularization of the Lattice
 * Boltzmann Method for open source computational aeroacoustics"
 * (arXiv:1710.02065), Sec. II:
 *   - Sec. II.A, eq. (optimizedLB): each step streams the populations and
 *     replaces them by f^{eqH}(rho, u) + (1 - 1/tau) f^{neqH}, both rebuilt
 *     from rho, u and the non-equilibrium second moment a2_neq through the
 *     Hermite recursions eqs. (recursive1), (recursive2), up to third order;
 *   - Sec. II.C, eqs. (spongeLB), (dampingLBM), (modifiedMoments): an
 *     absorbing layer that adds chi (f^{eqH}(rho_ref, u_ref) - f^{eqH}(rho*, u*))
 *     with the polynomial profile sigma(x) printed at the end of Sec. II.C;
 *   - Sec. II.B: 2:1 multi-domain grid refinement (two levels).
 * Boundary rules (Sec. III and IV setups): halfway bounce-back walls,
 * free-slip faces, zero-gradient outflow faces, equilibrium inlet cells.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1 on the coarsest level, cs^2 = 1/3.
 *   - Cells are indexed c = (z*ny + y)*nx + x, x fastest; nz = 1 in 2D.
 *   - Direction order (documented contract; lbm_lattice_table returns it):
 *       0: rest; then opposite pairs (2k-1, 2k):
 *       1,2 = (+-1,0,0)  3,4 = (0,+-1,0)  5,6 = (0,0,+-1)         [D3Qx]
 *       D2Q9 after the four axes: 5,6 = +-(1,1)  7,8 = +-(1,-1)
 *       D3Q19/27 edges: 7,8 = +-(1,1,0)  9,10 = +-(1,-1,0)
 *                       11,12 = +-(1,0,1)  13,14 = +-(1,0,-1)
 *                       15,16 = +-(0,1,1)  17,18 = +-(0,1,-1)
 *       D3Q27 corners: 19,20 = +-(1,1,1)  21,22 = +-(1,1,-1)
 *                      23,24 = +-(1,-1,1)  25,26 = +-(-1,1,1)
 *   - State: the library stores post-collision populations f*(x, t); one
 *     step pulls f(x, t+1) = f*(x - xi_i, t) and collides it.
 *   - Every pointer argument documented as "device" must be memory of the
 *     context's device (for example a torch CUDA tensor's data_ptr()); the
 *     call only enqueues work on the context's stream and returns.  Host
 *     pointers are read before the call returns.
 *   - No call throws.  Every int-returning call returns LBM_OK or a negative
 *     status; lbm_last_error() gives a thread-local message.  A context is
 *     not thread-safe; distinct contexts are independent.
 */
#ifndef HRLBM_LBM_H
#define HRLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 1

/* lattices (Sec. II.A Gauss-Hermite quadratures) */
enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19, LBM_D3Q27 = 27 };

/* state storage.  F64: FP64 storage and FP64 arithmetic (verification
 * build).  F32: FP32 storage of f.  F32S / F16S: FP32 / IEEE binary16
 * storage of the shifted value f_i - w_i rho0 (round to nearest even).
 * Every non-F64 format computes in FP32 on the deviation from rest.
 * M64 / M32 (FP64 / FP32 storage and arithmetic): instead of the q
 * populations, the moments of the post-collision state, rho - rho0, u and
 * a2* = Pi* - rho cs^2 I - rho u u (10 values per cell, 6 on D2Q9), from
 * which the regularized post-collision populations are rebuilt exactly
 * (eqs. eqH, neqH, recursive1, recursive2: every Hermite coefficient is a
 * function of rho, u and the non-equilibrium stress).  Only for fully
 * periodic, unrefined grids without absorbing layer, mask or comparator
 * collision (LBM_EINVAL otherwise); not batchable (lbm_step_batch:
 * LBM_EUNSUPPORTED).  lbm_get_populations rebuilds the populations;
 * lbm_set_populations keeps a regularized state exactly and projects any
 * other onto (rho, u, a2*); lbm_force is zero (no SOLID cells). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F32S = 2, LBM_F16S = 3, LBM_M64 = 4, LBM_M32 = 5 };

/* face rules, per face in the order x-, x+, y-, y+, z-, z+.  Both faces of
 * an axis are periodic or neither is.
 *   PERIODIC: wrap-around.
 *   FREESLIP: specular reflection, wall half a cell outside the face row.
 *   OUTFLOW:  zero gradient, a population entering through the face is
 *             copied from the face row.
 *   HALO:     a cut of a domain split into slabs along its last axis (z in
 *             3D, y on D2Q9; the other faces of that axis only): each
 *             population entering through the face is the post-collision
 *             value of the neighbouring subdomain's face-plane cell it
 *             streams from (that cell found by the rules of the other
 *             axes), read from this context's receive buffer; each step
 *             writes the populations leaving through the face into the send
 *             buffer (lbm_halo_buffers, lbm_halo_exchange).  The stepping
 *             is that of the undivided grid, bitwise when both run the same
 *             sweep path (a subdomain whose other faces are periodic or
 *             cuts, without mask or layer, takes the periodic path; give it
 *             an all-FLUID mask to match an undivided grid on the general
 *             path).  Conditions: no refinement, no absorbing-layer width
 *             on the face, no SOLID cell in the face plane (both subdomains'
 *             face planes, each checked by its own lbm_init), one step per
 *             lbm_step call.  Inlet noise is drawn from the subdomain's own
 *             cell numbering. */
enum { LBM_PERIODIC = 0, LBM_FREESLIP = 1, LBM_OUTFLOW = 2, LBM_HALO = 3 };

/* cell kinds in the mask.
 *   FLUID: streamed and collided.
 *   SOLID: never updated; links from a fluid cell into a solid cell are
 *          bounced back halfway (wall at rest).
 *   INLET: holds f^{eqH}(rho0, U u_dir (1 + inlet_noise r)) with r uniform
 *          in [-1, 1) per component, r = (z >> 40) * 2^-23 - 1 where z is the
 *          k-th SplitMix64 output for `seed` (Steele, Lea & Flood 2014),
 *          k = ((t*M + level)*N_level + cell)*3 + component, t = time index
 *          (on that level) of the state being produced, M = the number of
 *          levels of the context, at least 2. */
enum { LBM_FLUID = 0, LBM_SOLID = 1, LBM_INLET = 2 };

/* status codes */
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument or configuration */
  LBM_ENOMEM = -2,      /* device allocation failed / bound buffer too small */
  LBM_EDEVICE = -3,     /* HIP runtime error */
  LBM_EUNSTABLE = -4,   /* a non-finite or non-positive density was seen */
  LBM_ESTATE = -5,      /* call out of order (e.g. step before init) */
  LBM_EUNSUPPORTED = -6 /* valid request the library does not implement */
};

/* levels of a refined context: level 0 plus up to four nested 2:1 boxes
 * (the paper's setups use four and five levels, Sec. III and IV) */
#define LBM_MAX_LEVELS 5

/* flags */
#define LBM_ALLOW_HIGH_MA 0x1u /* accept Ma > 0.6 (beyond the stable range
                                  reported in the paper's conclusions) */
#define LBM_NO_GRAPH 0x2u      /* never replay step sequences as hipGraphs */
#define LBM_SPONGE_FIELD 0x8u  /* reserve per-cell absorbing-layer storage
                                  (lbm_set_sponge) on every level */
#define LBM_BGK 0x10u          /* comparator collision (Sec. II.A): LBM-BGK,
                                  eq. (standardLB) with the second-order
                                  equilibrium, same sponge force; FLUID cells
                                  only (initial and inlet states stay the
                                  regularized ones); no refinement */
#define LBM_MRT 0x20u          /* comparator collision: D2Q9 LBM-MRT of
                                  Lallemand & Luo (2000) with rates 1.64,
                                  1.54, 1.9 and 1/tau; no sponge, no
                                  refinement */
#define LBM_FULL_ORDER 0x4u    /* full recursive regularization (Sec. II.A,
                                  order n > 2): every Hermite polynomial the
                                  lattice resolves, up to fourth order on
                                  D2Q9 and sixth on D3Q27, with coefficients
                                  from eqs. (recursive1) and (recursive2);
                                  without it, third order.  D2Q9 and D3Q27
                                  only (the lattices with the property the
                                  paper relies on); EINVAL on D3Q19. */

typedef struct lbm_config {
  uint32_t struct_size;  /* sizeof(lbm_config); set by lbm_config_init */
  int32_t lattice;       /* LBM_D2Q9, LBM_D3Q19, LBM_D3Q27 */
  int32_t storage;       /* LBM_F64, LBM_F32, LBM_F32S, LBM_F16S */
  int32_t device;        /* HIP device ordinal */
  int64_t nx, ny, nz;    /* coarse grid; nz must be 1 for D2Q9 */
  double tau;            /* coarse relaxation time; nu = cs^2 (tau - 1/2) */
  double rho0;           /* rest density (also the storage shift) */
  double ma;             /* inlet Mach number: U = ma * cs along u_dir */
  double u_dir[3];       /* inlet direction (need not be normalised) */
  int32_t face_bc[6];    /* LBM_PERIODIC / LBM_FREESLIP / LBM_OUTFLOW /
                            LBM_HALO */
  int32_t sponge_width[6]; /* absorbing-layer width in coarse cells, per face */
  double chi_max;        /* sponge strength maximum, 0 <= chi_max < 4 tau */
  double rho_ref;        /* sponge reference density */
  double u_ref[3];       /* sponge reference velocity */
  int64_t refine_lo[3];  /* box [lo, hi] of level 1 in level-0 node       */
  int64_t refine_hi[3];  /*   coordinates; lo == hi == 0 on every axis: no
                            refinement */
  uint64_t seed;         /* inlet noise seed */
  double inlet_noise;    /* relative inlet velocity noise amplitude */
  void* stream;          /* hipStream_t for all work; NULL = null stream */
  uint32_t flags;        /* LBM_ALLOW_HIGH_MA | LBM_NO_GRAPH | LBM_FULL_ORDER |
                            LBM_SPONGE_FIELD | LBM_BGK | LBM_MRT */
  uint32_t block;        /* threads per workgroup for the sweep; 0 = tuned.
                            Moment storages: planes one workgroup marches
                            through = block / 16 (4 .. 64) */
  int32_t nest_count;    /* further nested boxes, 0 .. LBM_MAX_LEVELS - 2
                            (needs refine_lo/hi) */
  int32_t nest_reserved; /* 0 */
  int64_t nest_lo[LBM_MAX_LEVELS - 2][3]; /* box k: level k + 2 covers the   */
  int64_t nest_hi[LBM_MAX_LEVELS - 2][3]; /*   box [lo, hi] of level k + 1,
                                             in level k + 1 node coordinates */
} lbm_config;

typedef struct lbm_ctx lbm_ctx;

/* Fill *cfg with defaults: D3Q19, F32, device 0, 64^3 periodic, tau 0.6,
 * rho0 1, ma 0, u_dir (1,0,0), no sponge, no refinement, rho_ref 1. */
void lbm_config_init(lbm_config* cfg);

/* Device bytes lbm_create would allocate for this configuration (both
 * population buffers of every level, mask, interface buffers, halo buffers
 * of LBM_HALO faces).  0 on an invalid configuration (see lbm_last_error). */
size_t lbm_required_bytes(const lbm_config* cfg);

/* Validate the configuration and create a context.  Rejects: tau <= 1/2
 * (nu = cs^2 (tau - 1/2) must be positive, Sec. II.A); chi_max >= 4 tau on
 * any level (the stability bound of Sec. II.C); ma > 0.6 without
 * LBM_ALLOW_HIGH_MA; unknown lattice or storage; grids above 2^31 - 1 cells;
 * a refinement box that is smaller than 4 cells per axis or not at least 4
 * cells inside its parent level (inside [4, n - 5]; for level 1 this also
 * keeps it 4 cells from every face), or that overlaps an absorbing layer.
 * Each level l + 1 covers its box with half the spacing of level l
 * (2 (hi - lo) + 1 nodes per axis) and tau_(l+1) = (4 tau_l - 1) / 2, and
 * advances two steps per step of level l (Sec. II.B, eq. convective).  No device memory
 * is allocated here: the first lbm_init allocates it unless lbm_bind_memory
 * was called before.  *out receives the context. */
int lbm_create(const lbm_config* cfg, lbm_ctx** out);

/* Use a caller-owned device buffer of at least lbm_required_bytes bytes for
 * all context memory.  Must be called before lbm_init.  The library never
 * frees it; the caller keeps it alive until lbm_destroy. */
int lbm_bind_memory(lbm_ctx* ctx, void* dev_ptr, size_t bytes);

/* Write the post-collision state at t = 0 of `level` (0 = coarsest):
 *   f*_i = f^{eqH}_i(rho, u) + (1 - 1/tau) f^{neqH}_i(a2_neq = pi_neq, u)
 * (eqs. eqH, neqH).  Device pointers, FP64, structure of arrays over the
 * level's cells: rho [N], u [3][N], pi_neq [6][N] in the order
 * (xx, yy, zz, xy, xz, yz); z entries are ignored in 2D.  Any of them may be
 * NULL: rho0, the inlet velocity U u_dir, zero.  mask [N] uint8 device
 * pointer of LBM_FLUID/SOLID/INLET, NULL = all fluid; it is copied.  Resets
 * the step counter of the whole context.  Inputs may be freed once the
 * stream has passed this point. */
int lbm_init(lbm_ctx* ctx, int level, const double* rho, const double* u,
             const double* pi_neq, const uint8_t* mask);

/* Enqueue n coarse steps (level l + 1 takes two steps per step of level l
 * on a refined context; n <= 1 with LBM_HALO faces, else LBM_EINVAL).
 * Returns after enqueueing.  Kernel-side instability is recorded in a sticky
 * flag reported by lbm_sync / lbm_moments. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Wait for the context's stream; return LBM_OK or the sticky
 * LBM_EUNSTABLE / LBM_EDEVICE. */
int lbm_sync(lbm_ctx* ctx);

/* Steps completed (coarse time index). */
int64_t lbm_time(const lbm_ctx* ctx);

/* Cell updates one coarse step performs: all cells of an unrefined grid; on
 * a refined context the sum over levels l of 2^l times the cells swept on
 * level l (eq. convective).  Used to report MLUPS. */
int64_t lbm_updates_per_step(const lbm_ctx* ctx);

/* Grid shape of a level. */
int lbm_level_shape(const lbm_ctx* ctx, int level, int64_t* nx, int64_t* ny,
                    int64_t* nz);

/* Density and velocity of the current stored state of `level`:
 * rho = sum_i f*_i, u = sum_i f*_i xi_i / rho (eq. moments).  Away from the
 * sponge these equal the pre-collision moments of the same time level
 * (the collision conserves them).  SOLID cells report 0.  Device FP64
 * outputs rho_out [N] and u_out [3][N] (either may be NULL).  Returns the
 * sticky instability status as lbm_sync does, without synchronising. */
int lbm_moments(lbm_ctx* ctx, int level, double* rho_out, double* u_out);

/* Density (as lbm_moments) at n cells of `level`: cells [n] int64 device
 * pointer of cell indices, rho_out [n] FP64 device pointer. */
int lbm_probe(lbm_ctx* ctx, int level, const int64_t* cells, int n,
              double* rho_out);

/* Absorbing layer given per cell (Sec. II.C with any geometry, e.g. the
 * circular layer of the paper's cylinder setup, and spatially varying
 * reference fields such as a jet similarity profile): chi [N], rho_ref [N]
 * and u_ref [3][N] are FP64 device pointers over the level's cells (rho_ref
 * and u_ref may be NULL: the constant references of the configuration).
 * Cells with chi > 0 relax towards their own reference exactly as in the
 * face layers (eqs. spongeLB, dampingLBM, modifiedMoments); on this level
 * the face profile (sponge_width, chi_max) is no longer applied.  The
 * values are copied.  Needs LBM_SPONGE_FIELD at create; call after
 * lbm_init of the level (lbm_init clears it).  Rejects chi < 0,
 * chi >= 4 tau of the level (Sec. II.C) and non-finite values (synchronous
 * check on the host). */
int lbm_set_sponge(lbm_ctx* ctx, int level, const double* chi, const double* rho_ref,
                   const double* u_ref);

/* Running field statistics for the fluctuating pressure of Sec. III (the
 * pressure minus its temporal mean, p = cs^2 rho): adds x = rho - rho0 of
 * the current stored state to sum1[c] and x*x to sum2[c] for every cell c of
 * `level` (SOLID and COVERED cells add 0).  sum1, sum2: caller-owned FP64
 * device arrays of N entries, zeroed by the caller before the first call;
 * either may be NULL.  Enqueued on the context's stream; calls on one
 * context accumulate in order.  After n calls the temporal mean of p is
 * cs^2 (rho0 + sum1/n) and the rms of its fluctuation
 * cs^2 sqrt(sum2/n - (sum1/n)^2). */
int lbm_accumulate(lbm_ctx* ctx, int level, double* sum1, double* sum2);

/* Force on all SOLID cells of `level` by momentum exchange (Ladd 1994; Mei,
 * Yu, Shyy & Luo 2002), the body force behind the drag and lift of the
 * cylinder flow of Sec. III: on every link of a FLUID cell whose pulled
 * source (under the face rules) is SOLID, the stored post-collision
 * population f*_j moving into the wall returns reversed at the next step,
 * so the wall receives 2 f*_j xi_j.  out: FP64 device pointer to 3
 * components (x, y, z; z = 0 in 2D), written on the context's stream, in
 * lattice units per step.  Uses a reduction area inside the context's
 * memory, so two calls on one context must not overlap on different
 * streams.  The summation order is fixed: repeated calls give identical
 * bits.  A context without a mask gives 0. */
int lbm_force(lbm_ctx* ctx, int level, double* out);

/* Global totals of the stored state of `level` over its updated cells
 * (every cell but SOLID and COVERED): out[0] = sum (rho - rho0), the mass
 * relative to rest, and out[1..3] = sum of the momentum j = sum_i f_i xi_i
 * (eq. moments).  out: FP64 device pointer to 4 values, written on the
 * context's stream with the same fixed-order reduction as lbm_force (and
 * the same reduction area: calls on one context must not overlap on
 * different streams).  In a periodic domain without sponge, inlet or
 * walls both are invariants of the scheme.  Returns the sticky instability
 * status as lbm_moments does. */
int lbm_totals(lbm_ctx* ctx, int level, double* out);

/* Canonical FP64 copy of the stored populations of `level`, [q][N] in the
 * documented direction order, unshifted (device pointers).  Used for
 * checkpoint/resume and parity checks.  set also resets nothing else:
 * the step counter is kept.  On a refined context every level is stored
 * this way; a checkpoint also holds each interface (lbm_get_interface) and
 * the time (lbm_time). */
int lbm_get_populations(lbm_ctx* ctx, int level, double* out);
int lbm_set_populations(lbm_ctx* ctx, int level, const double* in);

/* Set the coarse time index of an initialised context (resume from a
 * checkpoint; call after every lbm_init of the context, which resets it):
 * level l's own time index becomes t * 2^l, which the inlet noise counter
 * of later steps follows.  t >= 0. */
int lbm_set_time(lbm_ctx* ctx, int64_t t);

/* Checkpoint of the refinement interface between level `level` and level
 * `level` + 1 (Sec. II.B): the parent's recorded pre-collision moments of
 * the current coarse time, which the next step's RING fill at t + 1/2
 * blends with the new ones (eq. convective, linear in time), and the other
 * record buffer.  Opaque bytes in the record's storage type (FP64 for
 * LBM_F64, FP32 otherwise), lbm_interface_bytes long (0 and an error if
 * there is no such interface).  get copies them to `out`, set restores them
 * from `in` (device pointers, asynchronous on the context's stream) on a
 * context of the same configuration.  With the populations of every level
 * and the time, a run of 2n steps equals n steps, save, restore into a
 * fresh context, n steps, bitwise. */
size_t lbm_interface_bytes(const lbm_ctx* ctx, int level);
int lbm_get_interface(lbm_ctx* ctx, int level, void* out);
int lbm_set_interface(lbm_ctx* ctx, int level, const void* in);

/* Serving: advance ctxs[k] by steps[k] coarse steps, k < n, sharing
 * launches between contexts: the contexts are grouped by lattice, storage,
 * sweep path (fully periodic or not) and workgroup size, and each group
 * advances through one persistent launch per step.  The first group runs
 * on the contexts' stream, the others concurrently on streams the library
 * owns, ordered after and joined back into the contexts' stream with
 * events, so work queued on that stream before the call precedes every
 * group and work queued after it follows them all.  Per device and
 * contexts' stream the library keeps, until the process ends, a job table,
 * its captured graphs and, for the groups after the first, one stream with
 * its own table each.  All contexts must be
 * unrefined, without halo faces, on one device and one stream, and
 * initialised.  Each context's
 * result is bitwise the same as lbm_step(ctxs[k], steps[k]) alone. */
int lbm_step_batch(lbm_ctx* const* ctxs, const int64_t* steps, int n);

/* Largest n lbm_step_batch_noalloc accepts. */
#define LBM_NOALLOC_MAX_JOBS 256

/* lbm_step_batch for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same contexts, the same kernels and bitwise the same results as
 * lbm_step_batch, with no hipMalloc, hipFree, host staging allocation or
 * graph instantiation.  The job tables live in a fixed device array of
 * static storage (about 130 KB: LBM_NOALLOC_MAX_JOBS batch headers and
 * jobs) that each device the library runs on holds until the process ends;
 * they are uploaded through kernel arguments and every step is its own
 * batch launch.  The caller still provides the contexts (whose memory
 * lbm_init or lbm_bind_memory set up beforehand).  Errors: LBM_EINVAL if
 * n > LBM_NOALLOC_MAX_JOBS or a step count exceeds 2^31 - 1, otherwise as
 * lbm_step_batch.  Every call on one device shares that device's tables and
 * rewrites them: calls on one stream are ordered, but calls that overlap on
 * one device (other streams or threads) race. */
int lbm_step_batch_noalloc(lbm_ctx* const* ctxs, const int64_t* steps, int n);

/* Time the sweep for each candidate workgroup size (64, 128, 256, 512,
 * 1024; for the moment storages the same values select block / 16 planes
 * per workgroup) on this context's current state (the state is restored
 * afterwards), keep the fastest, and return it (> 0) or a negative
 * status. */
int lbm_autotune(lbm_ctx* ctx, int trials);

/* Slab decomposition (face rule LBM_HALO; the streaming step of eq.
 * optimizedLB across a cut).  Library-owned device buffers of the halo face
 * on side 0 (low) or 1 (high) of the last axis, valid until lbm_destroy:
 *   send: the post-collision populations of this context's face-plane cells
 *         that leave through the face, written by every lbm_step and by
 *         lbm_init / lbm_set_populations;
 *   recv: what lbm_step reads for the populations entering through the
 *         face; before each lbm_step it must hold the neighbour's send
 *         buffer of the opposite side.  lbm_init fills it from this
 *         context's own face plane (a zero-gradient face until the first
 *         exchange).
 * Both hold *bytes bytes: [k][cell of the face plane] in the storage format
 * (stored values, shifted for F32S/F16S), k = rank, in the documented
 * direction order, among the directions with xi_last = -1 (send low, recv
 * high) or +1 (send high, recv low): 3 on D2Q9, 5 on D3Q19, 9 on D3Q27;
 * plane cells x + nx*y (3D) or x (D2Q9).  A caller on several GPUs moves
 * send to the neighbour's recv itself (e.g. grouped RCCL send/recv) after
 * lbm_init, lbm_set_populations and every lbm_step.  LBM_EINVAL if the face
 * is not LBM_HALO, LBM_ESTATE before lbm_init. */
int lbm_halo_buffers(lbm_ctx* ctx, int side, void** send, void** recv, size_t* bytes);

/* The same exchange between n initialised contexts on one device and one
 * stream, subdomain k + 1 above subdomain k along the last axis (and, with
 * periodic != 0, subdomain 0 above subdomain n - 1): asynchronous device
 * copies of each send buffer into the neighbour's receive buffer, on the
 * shared stream.  The contexts must agree on lattice, storage, rho0 and the
 * face plane, and carry every halo face the chain needs (LBM_EINVAL
 * otherwise).  With n = 1 and periodic, the context is its own neighbour. */
int lbm_halo_exchange(lbm_ctx* const* ctxs, int n, int periodic);

/* Release the context and the memory it allocated.  NULL-safe. */
void lbm_destroy(lbm_ctx* ctx);

/* Velocity table of a lattice in the documented order: xi [q][3] int32,
 * w [q] FP64 (host pointers; either may be NULL).  Returns q or LBM_EINVAL. */
int lbm_lattice_table(int lattice, int32_t* xi, double* w);

/* Thread-local description of the last error on this thread. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HRLBM_LBM_H */
