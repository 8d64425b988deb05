// Serving entry points: batched stepping of many resident contexts through
// the persistent batch kernel (with hipGraph replay of step sequences), its
// allocation-free variant, and the workgroup-size autotuner with its on-disk
// cache.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace hrlbm {

// Steps captured per graph: each step is one batch launch plus a one-thread
// launch that advances the device step counter.
static constexpr int kBatchGraphSteps = 16;

struct BatchRunner {
  int device = -1;
  hipStream_t stream = nullptr;
  BatchJob* d_jobs = nullptr;
  size_t cap = 0;
  BatchHeader* d_hdr = nullptr;
  BatchJob* h_jobs = nullptr;  // pinned staging
  BatchHeader* h_hdr = nullptr;
  hipEvent_t staged = nullptr;  // the last upload finished reading staging
  hipStream_t capture = nullptr;
  std::map<std::pair<int, int>, GraphEntry> graphs;  // (kernel variant, block)
  std::map<std::pair<int, int>, int> grids;
  // Lanes: the second and later groups of a batch run on runners of their
  // own with their own streams, concurrently with the first group (on the
  // caller's stream): ordered after the caller's stream by `fork`, joined
  // back into it by each lane's `done`.
  std::vector<BatchRunner*> lanes;
  hipEvent_t fork = nullptr;
  hipEvent_t done = nullptr;
};

static std::mutex g_batch_mu;

static hipError_t setup_runner(BatchRunner* r) {
  hipError_t e = hipMalloc(&r->d_hdr, sizeof(BatchHeader));
  if (e == hipSuccess) e = hipHostMalloc((void**)&r->h_hdr, sizeof(BatchHeader), 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->capture, hipStreamNonBlocking);
  return e;
}
static std::map<std::pair<int, hipStream_t>, BatchRunner*> g_runners;

static int runner_for(int device, hipStream_t st, BatchRunner** out) {
  auto key = std::make_pair(device, st);
  auto it = g_runners.find(key);
  if (it != g_runners.end()) {
    *out = it->second;
    return LBM_OK;
  }
  BatchRunner* r = new BatchRunner();
  r->device = device;
  r->stream = st;
  hipError_t e = setup_runner(r);
  if (e != hipSuccess) {
    delete r;
    return hip_error(e, "batch runner setup");
  }
  g_runners[key] = r;
  *out = r;
  return LBM_OK;
}

// Lane k of a runner (created on first use; streams at the default
// priority).
static int lane_for(BatchRunner* r, size_t k, BatchRunner** out) {
  while (r->lanes.size() <= k) {
    BatchRunner* l = new BatchRunner();
    l->device = r->device;
    hipError_t e = hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = setup_runner(l);
    if (e != hipSuccess) {
      if (l->stream) (void)hipStreamDestroy(l->stream);
      delete l;
      return hip_error(e, "batch lane setup");
    }
    r->lanes.push_back(l);
  }
  *out = r->lanes[k];
  return LBM_OK;
}

static int ensure_capacity(BatchRunner* r, size_t n) {
  if (n <= r->cap) return LBM_OK;
  hipError_t e = hipEventSynchronize(r->staged);
  if (e != hipSuccess) return hip_error(e, "batch staging wait");
  e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return hip_error(e, "batch stream wait");
  size_t cap = std::max<size_t>(64, r->cap);
  while (cap < n) cap *= 2;
  if (r->d_jobs) (void)hipFree(r->d_jobs);
  if (r->h_jobs) (void)hipHostFree(r->h_jobs);
  r->d_jobs = nullptr;
  r->h_jobs = nullptr;
  e = hipMalloc(&r->d_jobs, cap * sizeof(BatchJob));
  if (e == hipSuccess) e = hipHostMalloc((void**)&r->h_jobs, cap * sizeof(BatchJob), 0);
  if (e != hipSuccess) {
    r->cap = 0;
    return hip_error(e, "batch table allocation");
  }
  r->cap = cap;
  // graphs captured the old table pointer
  for (auto& kv : r->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  r->graphs.clear();
  return LBM_OK;
}

static int graph_for(BatchRunner* r, int variant, int block, int grid, GraphEntry** out) {
  auto key = std::make_pair(variant, block);
  auto it = r->graphs.find(key);
  if (it == r->graphs.end()) {
    GraphEntry g{};
    hipError_t e = hipStreamBeginCapture(r->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "batch capture begin");
    // steps base + 0 ... base + kBatchGraphSteps - 1, then base += kBatchGraphSteps
    for (int k = 0; k < kBatchGraphSteps && e == hipSuccess; ++k)
      e = launch_batch(variant, r->d_jobs, r->d_hdr, (int32_t)k, block, grid, r->capture);
    if (e == hipSuccess) e = launch_batch_bump(r->d_hdr, (int32_t)kBatchGraphSteps, r->capture);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(r->capture, &graph);
    if (e != hipSuccess) return hip_error(e, "batch launch during capture");
    if (e2 != hipSuccess) return hip_error(e2, "batch capture end");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_error(e, "batch graph instantiate");
    }
    g.graph = graph;
    it = r->graphs.emplace(key, g).first;
  }
  *out = &it->second;
  return LBM_OK;
}

// Batch kernel variant of a context: lattice code, storage, sweep path.
static int batch_variant(const lbm_ctx* c) {
  const SweepHost h = sweep_args(c, 0, 0, 0);
  return sweep_lattice(c->cfg) * 16 + c->cfg.storage * 2 + (h.general ? 1 : 0);
}

// One batch of contexts sharing a kernel variant and workgroup size.
static int run_group(BatchRunner* r, const std::vector<std::pair<lbm_ctx*, int64_t>>& grp) {
  lbm_ctx* c0 = grp[0].first;
  const int variant = batch_variant(c0);
  const int block = c0->block;
  int rc = ensure_capacity(r, grp.size());
  if (rc != LBM_OK) return rc;
  hipError_t e = hipEventSynchronize(r->staged);
  if (e != hipSuccess) return hip_error(e, "batch staging wait");
  uint32_t tiles = 0;
  int64_t max_steps = 0;
  for (size_t k = 0; k < grp.size(); ++k) {
    lbm_ctx* c = grp[k].first;
    const Level& L = c->lv[0];
    BatchJob& J = r->h_jobs[k];
    std::memset(&J, 0, sizeof J);
    J.h = sweep_args(c, 0, L.cur, 0);
    J.buf[0] = L.buf[0];
    J.buf[1] = L.buf[1];
    J.storage = c->cfg.storage;
    J.cur0 = L.cur;
    J.t0 = (uint64_t)L.t;
    J.steps = grp[k].second;
    J.tile_begin = tiles;
    J.ntiles = (uint32_t)((L.N + block - 1) / block);
    fill_fastdiv((uint32_t)L.nx, J.div_nx);
    fill_fastdiv((uint32_t)L.ny, J.div_ny);
    tiles += J.ntiles;
    max_steps = std::max(max_steps, grp[k].second);
  }
  if (max_steps == 0) return LBM_OK;
  r->h_hdr->njobs = (uint32_t)grp.size();
  r->h_hdr->total_tiles = tiles;
  r->h_hdr->step = 0;
  e = hipMemcpyAsync(r->d_jobs, r->h_jobs, grp.size() * sizeof(BatchJob),
                     hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->d_hdr, r->h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice,
                       r->stream);
  if (e == hipSuccess) e = hipEventRecord(r->staged, r->stream);
  if (e != hipSuccess) return hip_error(e, "batch table upload");
  auto gk = std::make_pair(variant, block);
  if (!r->grids.count(gk)) r->grids[gk] = batch_grid(variant, block);
  const int grid = r->grids[gk];
  if (grid <= 0) return set_error(LBM_EDEVICE, "batch occupancy query failed");
  int64_t done = 0;
  const bool use_graph = !(c0->cfg.flags & LBM_NO_GRAPH);
  if (use_graph && max_steps >= kBatchGraphSteps) {
    GraphEntry* g = nullptr;
    rc = graph_for(r, variant, block, grid, &g);
    if (rc != LBM_OK) return rc;
    for (; done + kBatchGraphSteps <= max_steps; done += kBatchGraphSteps) {
      e = hipGraphLaunch(g->exec, r->stream);
      if (e != hipSuccess) return hip_error(e, "batch graph launch");
    }
  }
  // the graphs advanced the device-side base to `done`: the remaining
  // steps pass their offset from it
  const int64_t base = done;
  for (; done < max_steps; ++done) {
    e = launch_batch(variant, r->d_jobs, r->d_hdr, (int32_t)(done - base), block, grid,
                     r->stream);
    if (e != hipSuccess) return hip_error(e, "batch launch");
  }
  for (auto& kv : grp) {
    lbm_ctx* c = kv.first;
    c->lv[0].t += kv.second;
    c->lv[0].cur ^= (int)(kv.second & 1);
    c->t += kv.second;
  }
  return LBM_OK;
}

// ------------------------------------------------------- allocation-free --
// lbm_step_batch_noalloc keeps its job tables in `scratch`, an array of
// static storage that every device the library runs on holds until the
// process ends: kNoAllocMaxJobs batch headers (one per group), then
// kNoAllocMaxJobs jobs.  Host code never uses the array's name as an
// address: the device address comes from hipGetSymbolAddress, once per
// device, and is what the kernels receive.
static constexpr int kNoAllocMaxJobs = LBM_NOALLOC_MAX_JOBS;
static constexpr size_t kNoAllocHdrBytes = kNoAllocMaxJobs * sizeof(BatchHeader);
static constexpr size_t kNoAllocBytes = kNoAllocHdrBytes + kNoAllocMaxJobs * sizeof(BatchJob);
static_assert(kNoAllocHdrBytes % 256 == 0, "job table alignment");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch[kScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current.
static int scratch_for(int device, unsigned char** out) {
  if (device < 0 || device >= kScratchDevices)
    return set_error(LBM_EINVAL, "device %d beyond the %d the allocation-free tables cover",
                     device, kScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "address of the allocation-free job tables");
    if (!p) return set_error(LBM_EDEVICE, "allocation-free job tables have no address");
    g_scratch[device] = (unsigned char*)p;
  }
  *out = g_scratch[device];
  return LBM_OK;
}

// Jobs written per table launch: the chunk travels as the kernel argument.
static constexpr int kTableChunk = 2;
struct TableChunk {
  BatchHeader hdr;     // the group's header, written with the first chunk
  uint32_t count;      // jobs in this chunk
  uint32_t write_hdr;
  BatchJob jobs[kTableChunk];
};

// One thread copies the chunk from its kernel argument into the tables
// (plain global stores); the batch launches that follow on the same stream
// read them.
__global__ void k_write_table(TableChunk c, BatchHeader* hdr, BatchJob* jobs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < kTableChunk; ++k)
    if ((uint32_t)k < c.count) jobs[k] = c.jobs[k];
  if (c.write_hdr) *hdr = c.hdr;
}

// The batch table entry of a context (as run_group builds it).
static void fill_job(BatchJob& J, lbm_ctx* c, int64_t steps, uint32_t tile_begin, int block) {
  const Level& L = c->lv[0];
  std::memset(&J, 0, sizeof J);
  J.h = sweep_args(c, 0, L.cur, 0);
  J.buf[0] = L.buf[0];
  J.buf[1] = L.buf[1];
  J.storage = c->cfg.storage;
  J.cur0 = L.cur;
  J.t0 = (uint64_t)L.t;
  J.steps = steps;
  J.tile_begin = tile_begin;
  J.ntiles = (uint32_t)((L.N + block - 1) / block);
  fill_fastdiv((uint32_t)L.nx, J.div_nx);
  fill_fastdiv((uint32_t)L.ny, J.div_ny);
}

// One group (contexts order[0..count) sharing kernel variant and workgroup
// size) through the tables at hdr / jobs: upload by kernel arguments, then
// one batch launch per step with the step as the launch's offset (the
// header's base stays 0).  No graphs, no host staging, no allocation.
static int run_group_noalloc(lbm_ctx* const* ctxs, const int64_t* steps, const int* order,
                             int count, BatchHeader* hdr, BatchJob* jobs) {
  lbm_ctx* c0 = ctxs[order[0]];
  const int variant = batch_variant(c0);
  const int block = c0->block;
  hipStream_t st = c0->stream;
  int64_t max_steps = 0;
  uint32_t tiles = 0;
  for (int k = 0; k < count; ++k) {
    const Level& L = ctxs[order[k]]->lv[0];
    tiles += (uint32_t)((L.N + block - 1) / block);
    max_steps = std::max(max_steps, steps[order[k]]);
  }
  if (max_steps == 0) return LBM_OK;
  TableChunk chunk;
  uint32_t tile_begin = 0;
  for (int k0 = 0; k0 < count; k0 += kTableChunk) {
    std::memset(&chunk, 0, sizeof chunk);
    chunk.count = (uint32_t)std::min(kTableChunk, count - k0);
    for (uint32_t k = 0; k < chunk.count; ++k) {
      const int j = order[k0 + (int)k];
      fill_job(chunk.jobs[k], ctxs[j], steps[j], tile_begin, block);
      tile_begin += chunk.jobs[k].ntiles;
    }
    if (k0 == 0) {
      chunk.write_hdr = 1;
      chunk.hdr.njobs = (uint32_t)count;
      chunk.hdr.total_tiles = tiles;
      chunk.hdr.step = 0;
    }
    hipLaunchKernelGGL(k_write_table, dim3(1), dim3(64), 0, st, chunk, hdr, jobs + k0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "allocation-free table upload");
  }
  const int grid = batch_grid(variant, block);
  if (grid <= 0) return set_error(LBM_EDEVICE, "batch occupancy query failed");
  for (int64_t s = 0; s < max_steps; ++s) {
    hipError_t e = launch_batch(variant, jobs, hdr, (int32_t)s, block, grid, st);
    if (e != hipSuccess) return hip_error(e, "batch launch");
  }
  for (int k = 0; k < count; ++k) {
    lbm_ctx* c = ctxs[order[k]];
    const int64_t n = steps[order[k]];
    c->lv[0].t += n;
    c->lv[0].cur ^= (int)(n & 1);
    c->t += n;
  }
  return LBM_OK;
}

// Checks shared by the batched entry points: every context initialised,
// unrefined, population-stored, without halo faces, on one device and stream,
// listed once, with a non-negative step count.
static int check_batch(lbm_ctx* const* ctxs, const int64_t* steps, int n) {
  for (int k = 0; k < n; ++k) {
    int rc = check_ready(ctxs[k]);
    if (rc != LBM_OK) return rc;
    if (steps[k] < 0) return set_error(LBM_EINVAL, "negative step count for job %d", k);
    if (ctxs[k]->nlevels > 1)
      return set_error(LBM_EUNSUPPORTED, "refined contexts cannot be batched");
    if (moment_storage(ctxs[k]->cfg.storage))
      return set_error(LBM_EUNSUPPORTED, "moment-stored contexts cannot be batched");
    if (has_halo(ctxs[k]->cfg))
      return set_error(LBM_EUNSUPPORTED, "contexts with halo faces cannot be batched");
    if (ctxs[k]->device != ctxs[0]->device || ctxs[k]->stream != ctxs[0]->stream)
      return set_error(LBM_EINVAL, "batched contexts must share device and stream");
    for (int m = 0; m < k; ++m)
      if (ctxs[m] == ctxs[k]) return set_error(LBM_EINVAL, "context %d appears twice", k);
  }
  return LBM_OK;
}

// ---------------------------------------------------------------- tuning --
static std::mutex g_tune_mu;

static std::string tune_path() {
  const char* p = std::getenv("HRLBM_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/hrlbm_tune.json";
}

// flat JSON object {"key": int, ...}
static std::map<std::string, int> read_cache() {
  std::map<std::string, int> m;
  std::ifstream f(tune_path());
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    const size_t colon = s.find(':', j);
    if (colon == std::string::npos) break;
    m[key] = std::atoi(s.c_str() + colon + 1);
    i = s.find_first_of(",}", colon);
    if (i == std::string::npos) break;
  }
  return m;
}

static void write_cache(const std::map<std::string, int>& m) {
  const std::string path = tune_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);
    for (size_t k = 1; k <= dir.size(); ++k)
      if (k == dir.size() || dir[k] == '/') {
        const std::string part = dir.substr(0, k);
        (void)::mkdir(part.c_str(), 0755);
      }
  }
  const std::string tmp = path + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{";
  bool first = true;
  for (auto& kv : m) {
    f << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "\n}\n";
  f.close();
  (void)std::rename(tmp.c_str(), path.c_str());
}

// (arch, lattice, storage, path, size class) key of the tuning cache
std::string tune_key(const lbm_ctx* ctx) {
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  const Level& L = ctx->lv[0];
  int cls = 0;
  for (int64_t n = L.N; n > 1; n >>= 2) ++cls;  // log4 of the cell count
  const SweepHost h = sweep_args(ctx, 0, 0, 0);
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s/q%d/s%d/%s/n4^%d", arch.c_str(), sweep_lattice(ctx->cfg),
                ctx->cfg.storage, h.general ? "general" : "periodic", cls);
  return buf;
}

int tuned_block(const lbm_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto m = read_cache();
  auto it = m.find(tune_key(ctx));
  if (it == m.end()) return 0;
  const int b = it->second;
  return (b >= 64 && b <= 1024 && b % 64 == 0) ? b : 0;
}

}  // namespace hrlbm

using namespace hrlbm;

extern "C" {

int lbm_step_batch(lbm_ctx* const* ctxs, const int64_t* steps, int n) {
  if (n < 0 || (n > 0 && (!ctxs || !steps))) return set_error(LBM_EINVAL, "batch arguments");
  if (n == 0) return LBM_OK;
  int rc = check_batch(ctxs, steps, n);
  if (rc != LBM_OK) return rc;
  rc = ensure_device(ctxs[0]);
  if (rc != LBM_OK) return rc;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchRunner* r = nullptr;
  rc = runner_for(ctxs[0]->device, ctxs[0]->stream, &r);
  if (rc != LBM_OK) return rc;
  // one persistent launch sequence per (kernel variant, workgroup size)
  std::map<std::pair<int, int>, std::vector<std::pair<lbm_ctx*, int64_t>>> groups;
  for (int k = 0; k < n; ++k)
    groups[std::make_pair(batch_variant(ctxs[k]), ctxs[k]->block)].push_back(
        {ctxs[k], steps[k]});
  if (groups.size() == 1) return run_group(r, groups.begin()->second);
  // groups after the first run concurrently on lanes (one stream each):
  // a small group's launches fill the device poorly on their own
  hipError_t e = hipEventRecord(r->fork, r->stream);
  if (e != hipSuccess) return hip_error(e, "batch fork");
  size_t g = 0;
  for (auto& kv : groups) {
    BatchRunner* x = r;
    if (g > 0) {
      rc = lane_for(r, g - 1, &x);
      if (rc != LBM_OK) break;
      e = hipStreamWaitEvent(x->stream, r->fork, 0);
      if (e != hipSuccess) {
        rc = hip_error(e, "batch lane wait");
        break;
      }
    }
    rc = run_group(x, kv.second);
    if (g > 0) {
      e = hipEventRecord(x->done, x->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(r->stream, x->done, 0);
      if (e != hipSuccess && rc == LBM_OK) rc = hip_error(e, "batch lane join");
    }
    if (rc != LBM_OK) break;
    ++g;
  }
  return rc;
}

int lbm_step_batch_noalloc(lbm_ctx* const* ctxs, const int64_t* steps, int n) {
  if (n < 0 || (n > 0 && (!ctxs || !steps))) return set_error(LBM_EINVAL, "batch arguments");
  if (n > kNoAllocMaxJobs)
    return set_error(LBM_EINVAL, "%d contexts; the allocation-free batch takes at most %d", n,
                     kNoAllocMaxJobs);
  if (n == 0) return LBM_OK;
  int rc = check_batch(ctxs, steps, n);
  if (rc != LBM_OK) return rc;
  for (int k = 0; k < n; ++k)
    if (steps[k] > INT32_MAX)
      return set_error(LBM_EINVAL, "step count of job %d beyond 2^31 - 1", k);
  rc = ensure_device(ctxs[0]);
  if (rc != LBM_OK) return rc;
  unsigned char* base = nullptr;
  rc = scratch_for(ctxs[0]->device, &base);
  if (rc != LBM_OK) return rc;
  BatchHeader* hdrs = (BatchHeader*)base;
  BatchJob* jobs = (BatchJob*)(base + kNoAllocHdrBytes);
  // group by (kernel variant, workgroup size), stable in the callers' order
  int var[kNoAllocMaxJobs], order[kNoAllocMaxJobs];
  for (int k = 0; k < n; ++k) {
    var[k] = batch_variant(ctxs[k]);
    order[k] = k;
  }
  auto before = [&](int a, int b) {
    if (var[a] != var[b]) return var[a] < var[b];
    if (ctxs[a]->block != ctxs[b]->block) return ctxs[a]->block < ctxs[b]->block;
    return a < b;
  };
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && before(order[j], order[j - 1]); --j) std::swap(order[j], order[j - 1]);
  int groups = 0;
  for (int g0 = 0; g0 < n;) {
    int g1 = g0 + 1;
    while (g1 < n && var[order[g1]] == var[order[g0]] &&
           ctxs[order[g1]]->block == ctxs[order[g0]]->block)
      ++g1;
    // group `groups` uses header `groups` and the jobs from position g0 on
    rc = run_group_noalloc(ctxs, steps, order + g0, g1 - g0, hdrs + groups, jobs + g0);
    if (rc != LBM_OK) return rc;
    ++groups;
    g0 = g1;
  }
  return LBM_OK;
}

int lbm_autotune(lbm_ctx* ctx, int trials) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  if (trials < 1) trials = 1;
  rc = ensure_device(ctx);
  if (rc != LBM_OK) return rc;
  // Each trial sweeps the current state into the other buffer without
  // swapping: the current state is untouched, the other buffer is scratch
  // (cells the sweep never writes keep their values).
  const Level& L = ctx->lv[0];
  const int cands[] = {64, 128, 256, 512, 1024};
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return hip_error(e, "autotune events");
  SweepHost h = sweep_args(ctx, 0, L.cur, (uint64_t)(L.t + 1));
  // the timing sweeps leave the halo send buffers as they are
  h.hsend[0] = h.hsend[1] = nullptr;
  const int reps = std::max(3, (int)std::min<int64_t>(50, (int64_t)(2e8 / (double)L.N)));
  float best_ms = 1e30f;
  int best = ctx->block;
  for (int blk : cands) {
    e = launch_step_kernel(ctx, h, blk, ctx->stream);
    if (e != hipSuccess) break;
    float tot = 0.f;
    for (int t = 0; t < trials && e == hipSuccess; ++t) {
      e = hipEventRecord(a, ctx->stream);
      for (int k = 0; k < reps && e == hipSuccess; ++k)
        e = launch_step_kernel(ctx, h, blk, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      tot += ms;
    }
    if (e != hipSuccess) break;
    if (tot < best_ms) {
      best_ms = tot;
      best = blk;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_error(e, "autotune");
  ctx->block = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto m = read_cache();
    m[tune_key(ctx)] = best;
    write_cache(m);
  }
  // graphs captured the old workgroup size
  for (auto& kv : ctx->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  ctx->graphs.clear();
  return best;
}

}  // extern "C"
