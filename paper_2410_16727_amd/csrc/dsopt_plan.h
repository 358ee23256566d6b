// Host-side plan state shared by the dsopt translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "dsopt.h"
#include "dsopt_internal.h"

using namespace dsk;

namespace dsh {

int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(DS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

// ------------------------------------------------------------------ arena --
// First-fit sub-allocator over the caller's device buffer (bookkeeping on
// the host only; 256-byte alignment; neighbours coalesce on free).
class Arena {
 public:
  void init(uint8_t* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  // returns offset or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        live_[off] = bytes;
        used_ += bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t len = it->second;
    live_.erase(it);
    used_ -= len;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + len == nx->first) {
      len += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  uint8_t* ptr(size_t off) const { return base_ + off; }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  uint8_t* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_, live_;
};

struct SceneRec {
  size_t off = SIZE_MAX;
  SceneDev dev{};
};

// One launch of ds_optimize_seeds / traced: its tables live until every
// problem in it is released.
struct LaunchRec {
  size_t tab_off = SIZE_MAX;   // ProbDev[n] + TileDev[nt] + counter + landing [n]
  size_t land_off = SIZE_MAX;  // the launch's block in the plan's pinned landing pool
  hipEvent_t done = nullptr;
  int refs = 0;
};

struct ProblemRec {
  int32_t tag;
  int S, T;
  size_t state_off = SIZE_MAX;   // tile states
  size_t out_off = SIZE_MAX;     // seed results + result + final trajectories
  ds_seed_result* seed_res = nullptr;
  ds_result* result = nullptr;
  float* best_traj = nullptr;
  float* final_traj = nullptr;
  const uint8_t* land = nullptr;   // pinned copy of result + best trajectory, or null
  std::shared_ptr<LaunchRec> launch;
};

}  // namespace dsh

struct ds_plan {
  using Arena = dsh::Arena;
  using SceneRec = dsh::SceneRec;
  using ProblemRec = dsh::ProblemRec;
  int device = 0;
  Arena arena;
  size_t robot_off = SIZE_MAX, params_off = SIZE_MAX;
  RobotDev robot{};
  ParamsDev params{};
  const RobotDev* robot_dev = nullptr;
  const ParamsDev* params_dev = nullptr;
  std::map<int32_t, SceneRec> scenes;
  std::map<int32_t, ProblemRec> problems;
  // deferred arena frees, each guarded by an event
  std::vector<std::pair<hipEvent_t, size_t>> deferred;
  std::vector<hipEvent_t> event_pool;
  // pinned landing pool: results of optimise launches arrive here with one
  // asynchronous copy per launch
  uint8_t* land_host = nullptr;
  Arena land_pool;
  // pinned staging for table uploads
  uint8_t* staging = nullptr;
  size_t staging_cap = 0, staging_pos = 0;
  std::vector<hipEvent_t> staging_events;
  int cu_count = 0, blocks_per_cu = 1;
  // optional kernel timing: (start, stop) event pairs not yet read
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
  // serving
  struct Serve* serve = nullptr;
};


namespace dsh {

// Helpers implemented in dsopt_host.cpp.
hipEvent_t get_event(ds_plan* p);
void put_event(ds_plan* p, hipEvent_t e);
void poll_deferred(ds_plan* p, bool wait);
int defer_free(ds_plan* p, size_t off, hipStream_t s);
size_t arena_alloc(ds_plan* p, size_t bytes);
int upload(ds_plan* p, void* dst, const void* src, size_t bytes, hipStream_t s);
bool finite_all(const float* v, int n);
int group_size(int T);
int tiles_for(int S, int T);
int validate_problem(ds_plan* p, const ds_problem& pr, bool need_seeds);
ProbDev make_probdev(ds_plan* p, const ds_problem& pr);
size_t out_bytes(int S, int T);
int alloc_problem_outputs(ds_plan* p, ProblemRec& rec);
double now_s();

// Launch `fn` on stream s, bracketed by timing events when enabled.
template <class Fn>
int timed_launch(ds_plan* p, hipStream_t s, Fn fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (p->timing) {
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, s));
  }
  HIP_TRY(fn());
  if (p->timing) {
    HIP_TRY(hipEventRecord(b, s));
    p->timed.emplace_back(a, b);
  }
  return DS_OK;
}

}  // namespace dsh
