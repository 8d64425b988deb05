// Host-side argument blocks and launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hrlbm {

// Added to the lattice id (9, 27) to select the full-order regularization
// in the collision kernels' dispatch.
constexpr int kFullOrderCode = 1000;
// Added to the lattice id to select a comparator collision in the sweep
// (LBM-BGK on every lattice, LBM-MRT on D2Q9).
constexpr int kBgkCode = 2000, kMrtCode = 3000;
// Storage codes of the moment-stored state (LBM_M64, LBM_M32 in lbm.h).
constexpr int kM64 = 4, kM32 = 5;
inline bool moment_storage(int storage) { return storage == kM64 || storage == kM32; }

// One sweep of one grid: src -> dst.
struct SweepHost {
  const void* src;
  void* dst;
  const uint8_t* mask;  // nullptr = all fluid
  const uint8_t* tiles;  // per 64-cell tile: 1 = every cell plain fluid
  int* status;
  uint32_t nx, ny, nz;
  uint64_t pstride;
  double tau, rho0;
  double chi_max, rho_ref, uref[3];
  double uin[3], noise;
  int32_t face[6], sponge[6];
  uint64_t seed, t_new;
  int32_t level;
  uint32_t lstride;  // inlet-noise counter blocks per time index (>= 2)
  bool general;  // false: all periodic, no mask, no sponge
  // refinement record of coarse pre-collision moments (nullptr: off)
  void* rec;
  int32_t rec_off[3];
  uint32_t rec_dim[3];
  uint32_t rec_n;
  int32_t box_lo[3], box_hi[3];
  // child-side record of the import band (nullptr: off)
  void* recf;
  // RING nodes of this level rebuilt by the sweep from the parent's records
  // ring_wa * Ma + ring_wb * Mb (ring_Ma nullptr: RING nodes left as they
  // are); the parent-side record geometry and alpha_cf = tau / (2 tau_parent)
  const void* ring_Ma;
  const void* ring_Mb;
  double ring_wa, ring_wb, ring_alpha;
  int32_t ring_lo[3], ring_off[3];
  uint32_t ring_dim[3];
  // absorbing layer given per cell (5 x N values of the compute type)
  const void* sp;
  // halo faces of the last axis, side 0 = low, 1 = high (nullptr: none;
  // hsend nullptr: the sweep does not pack); hplane cells per face plane
  const void* hrecv[2];
  void* hsend[2];
  uint32_t hplane;
};

// Halo faces packed outside the sweep (k_halo_pack).
struct HaloArgs {
  const void* src;
  void* hsend[2];  // nullptr: side has no halo face
  void* hrecv[2];
  uint32_t nx, ny, nz, hplane;
  uint64_t pstride;
  int entering;    // also fill the receive buffers from the own face plane
};

// Absorbing layer given per cell: FP64 inputs converted into `sp`
// (chi, rho_ref, u_ref x 3, each over N cells) and the kFieldSponge flag set
// in the mask where chi > 0.
struct SpongeArgs {
  const double* chi;
  const double* rho_ref;
  const double* u_ref;
  double rho_ref0, u_ref0[3];
  void* sp;
  uint8_t* mask;
  uint32_t n;
};

// Mark the refinement roles in a level's mask: with a parent, RING on the
// outer shell; with a child covering [lo, hi], IMPORT on the shell of
// [lo+1, hi-1] and COVERED inside it.
struct RolesArgs {
  uint8_t* mask;
  uint32_t nx, ny, nz;
  int32_t ring, child, dim;
  int32_t lo[3], hi[3];
};

// Flag bits of the mask (see kernels.hpp): near a SOLID cell, on a
// non-periodic face; then the per-tile summary of the flagged mask.
struct FlagsArgs {
  uint8_t* mask;
  uint8_t* tiles;  // per 64-cell tile summary, filled after the flags
  uint32_t nx, ny, nz;
  int32_t face[6];
};

// Record box of the coarse moments filled from the initial fields.
struct RecordFieldsArgs {
  const double* rho;
  const double* u;
  const double* pineq;
  void* rec_a;
  void* rec_b;
  uint32_t nx, ny, nz;
  int32_t rec_off[3];
  uint32_t rec_dim[3];
  uint32_t rec_n;
  int32_t box_lo[3], box_hi[3];
  double rho0, uin[3];
};

// RING nodes of the fine level rebuilt from the recorded coarse moments
// blended in time (wa * Ma + wb * Mb).
struct RingArgs {
  const uint32_t* list;
  uint32_t n;
  uint32_t fnx, fny;
  int32_t lo[3];
  const void* Ma;
  const void* Mb;
  double wa, wb;
  int32_t rec_off[3];
  uint32_t rec_dim[3];
  uint32_t rec_n;
  double alpha, omega1, rho0;
  void* dst;
  uint64_t pstride;
};

// IMPORT nodes of a parent level rebuilt from the child's recorded
// pre-collision moments (band record: 10 contiguous components per child node).
struct ImportArgs {
  const uint32_t* list;
  uint32_t n;
  uint32_t cnx, cny;
  int32_t lo[3];
  const void* recf;
  uint32_t fnx, fny, fnz;
  double alpha, omega1, rho0;
  void* dst;
  uint64_t pstride;
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

struct AccumArgs {
  const void* src;
  const uint8_t* mask;
  double* sum1;
  double* sum2;
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

// Deterministic reductions over a level (momentum-exchange force, totals):
// kRedBlocks partial sums of up to kRedMax doubles each in `partial`, the
// result in out.
constexpr uint32_t kRedBlocks = 1024, kRedThreads = 256, kRedMax = 4;
struct ReduceArgs {
  const void* src;
  const uint8_t* mask;  // nullptr: all cells fluid (no SOLID cells)
  double* partial;
  double* out;
  uint32_t nx, ny, nz;
  uint64_t pstride;
  int32_t face[6];
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

// One context of a batched (serving) launch.  The job table stays in device
// memory for the whole batch; the step index s comes from BatchHeader.
struct BatchJob {
  SweepHost h;          // parameters; h.src / h.dst unused
  void* buf[2];         // the context's two population buffers
  int32_t storage;
  int32_t cur0;         // buffer holding the state at batch start
  uint64_t t0;          // time index at batch start
  int64_t steps;        // steps this job takes in the batch
  uint32_t tile_begin;  // first tile of this job in the work list
  uint32_t ntiles;
  uint32_t div_nx[3], div_ny[3];  // fast-division constants (d, m, s)
};

struct BatchHeader {
  uint32_t njobs;
  uint32_t total_tiles;
  int32_t step;  // base of the step index s within the batch (plus the launch's offset)
  int32_t pad;
};

hipError_t launch_sweep(int lattice, int storage, const SweepHost& h, int block,
                        hipStream_t st);
// persistent batched sweep: grid of `grid` workgroups of `block` threads
// variant = lattice code * 16 + storage * 2 + (general path ? 1 : 0)
// s_off: offset added to the device-side step index for this launch
hipError_t launch_batch(int variant, const BatchJob* jobs, BatchHeader* hdr, int32_t s_off,
                        int block, int grid, hipStream_t st);
// advance the device-side step index by `by`
hipError_t launch_batch_bump(BatchHeader* hdr, int32_t by, hipStream_t st);
int batch_grid(int variant, int block);  // resident workgroups on the device
void fill_fastdiv(uint32_t d, uint32_t out[3]);
hipError_t launch_init(int lattice, int storage, const InitArgs& a, uint32_t n,
                       hipStream_t st);
hipError_t launch_moments(int lattice, int storage, const MomentArgs& a,
                          uint32_t n, hipStream_t st);
hipError_t launch_accum(int lattice, int storage, const AccumArgs& a, uint32_t n,
                        hipStream_t st);
hipError_t launch_set_sponge(int storage, const SpongeArgs& a, hipStream_t st);
hipError_t launch_tiles(const FlagsArgs& a, hipStream_t st);
hipError_t launch_force(int lattice, int storage, const ReduceArgs& a, hipStream_t st);
hipError_t launch_totals(int lattice, int storage, const ReduceArgs& a, hipStream_t st);
hipError_t launch_probe(int lattice, int storage, const ProbeArgs& a,
                        uint32_t n, hipStream_t st);
hipError_t launch_get_pop(int lattice, int storage, const PopArgs& a,
                          uint32_t n, hipStream_t st);
hipError_t launch_set_pop(int lattice, int storage, const PopArgs& a,
                          uint32_t n, hipStream_t st);
hipError_t launch_roles(const RolesArgs& a, uint32_t n, hipStream_t st);
hipError_t launch_halo_pack(int lattice, int storage, const HaloArgs& a, hipStream_t st);
// directions crossing one halo face (3, 5 or 9 for lattice 9, 19, 27)
int halo_count_of(int lattice);
hipError_t launch_flags(int lattice, const FlagsArgs& a, hipStream_t st);
hipError_t launch_record_fields(int lattice, int storage, const RecordFieldsArgs& a,
                                uint32_t n, hipStream_t st);
hipError_t launch_ring(int lattice, int storage, const RingArgs& a, uint32_t n,
                       hipStream_t st);
hipError_t launch_import(int lattice, int storage, const ImportArgs& a, uint32_t n,
                         hipStream_t st);

// Moment-stored state (msweep.hip): the sweep (`block` / 16 planes per
// workgroup) and the companion kernels.
hipError_t launch_msweep(int lattice, int storage, const SweepHost& h, int block,
                         hipStream_t st);
hipError_t launch_minit(int lattice, int storage, const InitArgs& a, hipStream_t st);
hipError_t launch_mmoments(int lattice, int storage, const MomentArgs& a, hipStream_t st);
hipError_t launch_mprobe(int storage, const ProbeArgs& a, hipStream_t st);
hipError_t launch_maccum(int storage, const AccumArgs& a, hipStream_t st);
hipError_t launch_mtotals(int lattice, int storage, const ReduceArgs& a, hipStream_t st);
hipError_t launch_mforce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_mget_pop(int lattice, int storage, const PopArgs& a, hipStream_t st);
hipError_t launch_mset_pop(int lattice, int storage, const PopArgs& a, hipStream_t st);

}  // namespace hrlbm
