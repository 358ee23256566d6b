// Allocation-free planning call (ds_optimize_noalloc): one problem
// optimised exactly as ds_optimize_seeds does, with the optimiser state,
// the work tables and the final trajectories in a file-scope device array
// instead of the plan's arena, and the tables written on the device by a
// set-up kernel from by-value arguments.  The call allocates nothing,
// copies nothing from the host and never waits, so callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation) can use it.  Every call on a GPU shares that
// GPU's array: calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "dsopt_plan.h"

namespace {

// Layout of the array (bytes, 256-aligned parts): problem record, tile
// table, tile-queue counter, final trajectories, tile states.
constexpr size_t NA_PROB = 0;
constexpr size_t NA_TILES = 256;
constexpr size_t NA_COUNTER =
    NA_TILES + ((size_t)DS_NOALLOC_MAX_SEEDS * sizeof(TileDev) + 255) / 256 * 256;
constexpr size_t NA_FINAL = NA_COUNTER + 256;
constexpr size_t NA_STATE =
    NA_FINAL + ((size_t)DS_NOALLOC_MAX_SEEDS * DS_MAX_T * NJ * sizeof(float) + 255) / 256 * 256;
constexpr size_t NA_BYTES = NA_STATE + (size_t)DS_NOALLOC_MAX_SEEDS * ST_BYTES;
static_assert(sizeof(ProbDev) <= NA_TILES, "problem record exceeds its slot");

static __device__ __align__(256) uint8_t scratch[NA_BYTES];

// The array's device address on each GPU (host code must not use the
// symbol itself as an address).
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
uint8_t* g_ptr[MAX_DEVICES] = {};

// Problem record, tile table (one tile per seed), fresh tile states (the
// iteration counter, so the optimiser starts from the seed), zeroed
// per-seed results (their counters accumulate) and an empty tile queue.
// One workgroup of one wavefront per tile.
__global__ void __launch_bounds__(64) k_noalloc_setup(ProbDev pd, uint8_t* base) {
  const int k = blockIdx.x;
  TileDev* tiles = reinterpret_cast<TileDev*>(base + NA_TILES);
  float* state = reinterpret_cast<float*>(base + NA_STATE + (size_t)k * ST_BYTES);
  if (threadIdx.x == 0) {
    TileDev t;
    t.prob = 0;
    t.seed0 = k;
    t.nseed = 1;
    t.G = pd.G;
    t.state = state;
    tiles[k] = t;
    if (k == 0) {
      *reinterpret_cast<ProbDev*>(base + NA_PROB) = pd;
      *reinterpret_cast<int*>(base + NA_COUNTER) = 0;
    }
  }
  reinterpret_cast<int*>(state)[ST_ITER + threadIdx.x] = 0;
  reinterpret_cast<int*>(state)[ST_EVG + threadIdx.x] = 0;
  constexpr int W = (int)(sizeof(ds_seed_result) / sizeof(int));
  if (threadIdx.x < W) reinterpret_cast<int*>(pd.seed_res + k)[threadIdx.x] = 0;
}

}  // namespace

namespace dsk {

// Resolve the array's address on the current device once (called by
// ds_plan_create with the plan's device current).
int noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return dsh::fail(DS_ERR_HIP, "device %d", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return DS_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return dsh::fail(DS_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_ptr[device] = static_cast<uint8_t*>(p);
  return DS_OK;
}

}  // namespace dsk

extern "C" int ds_optimize_noalloc(ds_plan* p, const ds_problem* prob,
                                   ds_seed_result* seed_results, ds_result* result,
                                   float* best_traj, void* stream) {
  using namespace dsh;
  if (!p || !prob || !seed_results || !result || !best_traj)
    return fail(DS_ERR_INVALID, "NULL argument");
  if (int rc = validate_problem(p, *prob, true)) return rc;
  if (prob->n_seeds > DS_NOALLOC_MAX_SEEDS)
    return fail(DS_ERR_INVALID, "n_seeds %d exceeds the allocation-free maximum %d",
                prob->n_seeds, DS_NOALLOC_MAX_SEEDS);
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (p->device >= 0 && p->device < MAX_DEVICES) base = g_ptr[p->device];
  }
  if (!base) return fail(DS_ERR_STATE, "allocation-free scratch not set up on device %d", p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProbDev pd = make_probdev(p, *prob);
  pd.final_traj = reinterpret_cast<float*>(base + NA_FINAL);
  pd.seed_res = seed_results;
  pd.result = result;
  pd.best_traj = best_traj;
  const int S = prob->n_seeds;
  hipLaunchKernelGGL(k_noalloc_setup, dim3(S), dim3(64), 0, s, pd, base);
  HIP_TRY(hipGetLastError());
  const ProbDev* pd_dev = reinterpret_cast<const ProbDev*>(base + NA_PROB);
  const TileDev* td_dev = reinterpret_cast<const TileDev*>(base + NA_TILES);
  int* counter = reinterpret_cast<int*>(base + NA_COUNTER);
  const int W = p->params.waves;
  const int per_block = W > 1 ? 1 : WAVES_PER_BLOCK;
  int blocks = (S + per_block - 1) / per_block;
  blocks = std::max(1, std::min(blocks, p->cu_count * p->blocks_per_cu));
  HIP_TRY(launch_optimize(p->robot_dev, p->params_dev, pd_dev, td_dev, S, counter, blocks,
                          p->params.n_iters, W, params_ext(p->params), s));
  HIP_TRY(launch_best(pd_dev, 1, nullptr, s));
  return DS_OK;
}
