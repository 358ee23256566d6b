// Serving loop of the dsopt C ABI: continuous batching of planning requests.
//
// Requests wait in a FIFO queue and are admitted into device slots while a
// slot is free and the arena can hold the request's optimiser state.  One
// step = collect the replays that have completed, admit waiting requests,
// publish the active tile list, then enqueue a replay of a captured HIP
// graph (counter reset kernel, persistent optimiser over the tile list for
// block_iters iterations, best-seed kernel over the active slots).  The
// graph is captured once with fixed arguments; membership changes only
// through the device tables the host rewrites between replays, so requests
// that arrive while others run overlap with them on the device.  Every
// tile keeps its own state and iteration count, so a request's arithmetic
// is the same as when it is optimised alone.
//
// A request's iteration count is fixed, so the host knows at enqueue time
// which replay is a request's last: it queues the copy of the result to
// pinned memory right behind that replay, frees the slot for the next
// admission and defers the release of the request's arena memory to an
// event after the copy.  Up to DEPTH replays are in flight, so the table
// uploads and the next replay sit in the stream behind the running one and
// the device does not wait for the host between blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "dsopt_plan.h"

using namespace dsh;

namespace {

constexpr int MAX_TILES_PER_REQ = 128;
constexpr int DEPTH = 2;   // replays in flight

// pinned landing area of one finishing request, laid out like the device
// outputs (result record padded to 256 bytes, best trajectory after it) so
// one copy brings both
struct Landing {
  union {
    ds_result result;
    uint8_t pad[256];
  };
  float traj[DS_MAX_T * NJ];
};
static_assert(sizeof(ds_result) <= 256, "result record exceeds its slot");

struct Finishing {
  uint64_t ticket;
  int slot;
};

struct Replay {
  hipEvent_t done = nullptr;
  int64_t seq = 0;
  std::vector<Finishing> finishing;
};

struct ServeReq {
  ds_problem prob;
  double t_submit = 0, t_done = 0;
  int slot = -1;
  int iters_left = 0;       // iterations not yet enqueued
  bool done = false;
  ds_result result{};
  std::vector<float> best;
};

struct Slot {
  uint64_t ticket = 0;       // 0 = free
  size_t state_off = SIZE_MAX, out_off = SIZE_MAX;
  ds_result* result = nullptr;
  float* best_traj = nullptr;
  int ntiles = 0;
};

}  // namespace

struct Serve {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_slots = 0, queue_cap = 0;
  size_t tab_off = SIZE_MAX;
  ProbDev* probs_dev = nullptr;
  TileDev* tiles_dev = nullptr;
  int* slot_list_dev = nullptr;   // [0] = count, then slot indices; [max_slots + 1] =
                                  // iterations of the replay
  int* tile_list_dev = nullptr;   // [0] = count, then tile indices (follows the slot list)
  size_t slot_list_bytes = 0;     // padded size of the slot list region
  bool lists_dirty = true;        // membership changed since the last upload
  int block = -1;                 // iterations of the last uploaded replay
  int* counter_dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::deque<Replay> inflight;
  Landing* landing = nullptr;    // pinned, [DEPTH][max_slots]
  std::vector<Slot> slots;
  std::deque<uint64_t> queue;
  std::map<uint64_t, ServeReq> reqs;
  uint64_t next_ticket = 1;
  // statistics
  std::vector<double> lat_ms;
  double first_submit = -1, last_done = 0;
  int64_t steps = 0;
  double active_sum = 0;
  std::vector<int> host_lists, host_slots;
};

void ds_serve_free(ds_plan* p) {
  if (!p || !p->serve) return;
  Serve* sv = p->serve;
  for (Replay& r : sv->inflight) {
    hipEventSynchronize(r.done);
    put_event(p, r.done);
  }
  sv->inflight.clear();
  for (auto& sl : sv->slots) {
    if (sl.state_off != SIZE_MAX) p->arena.release(sl.state_off);
    if (sl.out_off != SIZE_MAX) p->arena.release(sl.out_off);
  }
  if (sv->tab_off != SIZE_MAX) p->arena.release(sv->tab_off);
  if (sv->exec) hipGraphExecDestroy(sv->exec);
  if (sv->graph) hipGraphDestroy(sv->graph);
  if (sv->landing) hipHostFree(sv->landing);
  if (sv->own_stream) hipStreamDestroy(sv->stream);
  delete sv;
  p->serve = nullptr;
}

bool ds_serve_uses_scene(const ds_plan* p, int32_t scene_id) {
  if (!p || !p->serve) return false;
  const Serve* sv = p->serve;
  for (uint64_t t : sv->queue) {
    auto it = sv->reqs.find(t);
    if (it != sv->reqs.end() && it->second.prob.scene_id == scene_id) return true;
  }
  for (const Slot& sl : sv->slots) {
    if (!sl.ticket) continue;
    auto it = sv->reqs.find(sl.ticket);
    if (it != sv->reqs.end() && it->second.prob.scene_id == scene_id) return true;
  }
  return false;
}

namespace {

// Take the results of completed replays (in order).  With `block`, wait
// for the oldest replay first.
int collect(ds_plan* p, Serve* sv, bool block) {
  while (!sv->inflight.empty()) {
    Replay& rp = sv->inflight.front();
    if (block) {
      HIP_TRY(hipEventSynchronize(rp.done));
      block = false;
    } else {
      hipError_t q = hipEventQuery(rp.done);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(DS_ERR_HIP, "replay failed: %s", hipGetErrorString(q));
    }
    double t = now_s();
    const Landing* set = sv->landing + (size_t)(rp.seq % DEPTH) * sv->max_slots;
    for (const Finishing& f : rp.finishing) {
      ServeReq& r = sv->reqs[f.ticket];
      r.result = set[f.slot].result;
      r.best.assign(set[f.slot].traj, set[f.slot].traj + (size_t)r.prob.horizon * NJ);
      r.done = true;
      r.t_done = t;
      sv->lat_ms.push_back((t - r.t_submit) * 1e3);
      sv->last_done = t;
    }
    put_event(p, rp.done);
    sv->inflight.pop_front();
  }
  return DS_OK;
}

int admit(ds_plan* p, Serve* sv) {
  while (!sv->queue.empty()) {
    int slot = -1;
    for (int i = 0; i < sv->max_slots; ++i)
      if (!sv->slots[i].ticket) { slot = i; break; }
    if (slot < 0) return DS_OK;
    uint64_t ticket = sv->queue.front();
    ServeReq& r = sv->reqs[ticket];
    const ds_problem& pr = r.prob;
    int nt = tiles_for(pr.n_seeds, pr.horizon);
    ProblemRec rec;
    rec.S = pr.n_seeds;
    rec.T = pr.horizon;
    rec.state_off = p->arena.alloc((size_t)nt * ST_BYTES);
    if (rec.state_off == SIZE_MAX) return DS_OK;   // wait for memory
    if (alloc_problem_outputs(p, rec) != DS_OK) {
      p->arena.release(rec.state_off);
      return DS_OK;
    }
    if (!p->scenes.count(pr.scene_id)) {           // scene released while waiting
      p->arena.release(rec.state_off);
      p->arena.release(rec.out_off);
      r.done = true;
      r.result = ds_result{};
      r.result.best_seed = -1;
      sv->queue.pop_front();
      continue;
    }
    if (reinterpret_cast<uint8_t*>(rec.best_traj) !=
        reinterpret_cast<uint8_t*>(rec.result) + offsetof(Landing, traj))
      return fail(DS_ERR_STATE, "output layout does not match the landing area");
    ProbDev pd = make_probdev(p, pr);
    pd.final_traj = rec.final_traj;
    pd.seed_res = rec.seed_res;
    pd.result = rec.result;
    pd.best_traj = rec.best_traj;
    std::vector<TileDev> td(nt);
    for (int k = 0; k < nt; ++k) {
      td[k].prob = slot;
      td[k].seed0 = k;
      td[k].nseed = 1;
      td[k].G = pd.G;
      td[k].state = reinterpret_cast<float*>(p->arena.ptr(rec.state_off) + (size_t)k * ST_BYTES);
    }
    HIP_TRY(hipMemsetAsync(p->arena.ptr(rec.state_off), 0, (size_t)nt * ST_BYTES, sv->stream));
    HIP_TRY(hipMemsetAsync(rec.seed_res, 0, (size_t)rec.S * sizeof(ds_seed_result), sv->stream));
    if (int rc = upload(p, sv->probs_dev + slot, &pd, sizeof pd, sv->stream)) return rc;
    if (int rc = upload(p, sv->tiles_dev + (size_t)slot * MAX_TILES_PER_REQ, td.data(),
                        td.size() * sizeof(TileDev), sv->stream))
      return rc;
    Slot& sl = sv->slots[slot];
    sl.ticket = ticket;
    sl.state_off = rec.state_off;
    sl.out_off = rec.out_off;
    sl.result = rec.result;
    sl.best_traj = rec.best_traj;
    sl.ntiles = nt;
    r.slot = slot;
    sv->lists_dirty = true;
    r.iters_left = p->params.n_iters;
    sv->queue.pop_front();
  }
  return DS_OK;
}

}  // namespace

extern "C" {

int ds_serve_start(ds_plan* p, int max_slots, int queue_cap, void* stream) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  if (p->serve) return fail(DS_ERR_STATE, "serving already started");
  if (max_slots < 1 || max_slots > 256 || queue_cap < 1)
    return fail(DS_ERR_INVALID, "max_slots must be 1..256 and queue_cap >= 1");
  auto* sv = new Serve();
  sv->max_slots = max_slots;
  sv->queue_cap = queue_cap;
  sv->slots.resize(max_slots);
  sv->stream = static_cast<hipStream_t>(stream);
  if (!sv->stream) {
    if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
      delete sv;
      return fail(DS_ERR_HIP, "stream creation failed");
    }
    sv->own_stream = true;
  }
  p->serve = sv;
  size_t max_tiles = (size_t)max_slots * MAX_TILES_PER_REQ;
  size_t a = ((size_t)max_slots * sizeof(ProbDev) + 255) / 256 * 256;
  size_t b = (max_tiles * sizeof(TileDev) + 255) / 256 * 256;
  size_t c = ((max_tiles + 1) * sizeof(int) + 255) / 256 * 256;
  size_t d = (((size_t)max_slots + 2) * sizeof(int) + 255) / 256 * 256;
  sv->tab_off = arena_alloc(p, a + b + c + d + 256);
  if (sv->tab_off == SIZE_MAX) {
    ds_serve_free(p);
    return fail(DS_ERR_NOMEM, "arena full (serving tables)");
  }
  uint8_t* base = p->arena.ptr(sv->tab_off);
  sv->probs_dev = reinterpret_cast<ProbDev*>(base);
  sv->tiles_dev = reinterpret_cast<TileDev*>(base + a);
  sv->slot_list_dev = reinterpret_cast<int*>(base + a + b);
  sv->tile_list_dev = reinterpret_cast<int*>(base + a + b + d);
  sv->slot_list_bytes = d;
  sv->counter_dev = reinterpret_cast<int*>(base + a + b + c + d);
  // empty lists before the first replay
  HIP_TRY(hipMemsetAsync(base, 0, a + b + c + d + 256, sv->stream));
  if (hipHostMalloc((void**)&sv->landing, sizeof(Landing) * DEPTH * max_slots,
                    hipHostMallocDefault) != hipSuccess) {
    sv->landing = nullptr;
    ds_serve_free(p);
    return fail(DS_ERR_HIP, "pinned result area allocation failed");
  }
  // capture one iteration block over whatever the tables hold at replay time
  int grid = std::max(1, p->cu_count * p->blocks_per_cu);
  HIP_TRY(hipStreamSynchronize(sv->stream));
  HIP_TRY(hipStreamBeginCapture(sv->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = launch_zero_i32(sv->counter_dev, 1, sv->stream);
  hipError_t e2 = launch_serve_step(p->robot_dev, p->params_dev, sv->probs_dev, sv->tiles_dev,
                                    sv->tile_list_dev, sv->counter_dev, (int)max_tiles, grid,
                                    sv->slot_list_dev + max_slots + 1, p->params.waves,
                                    params_ext(p->params), sv->stream);
  hipError_t e3 = launch_best(sv->probs_dev, max_slots, sv->slot_list_dev, sv->stream);
  hipError_t e4 = hipStreamEndCapture(sv->stream, &sv->graph);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    ds_serve_free(p);
    return fail(DS_ERR_HIP, "graph capture failed: %s / %s / %s / %s", hipGetErrorString(e1),
                hipGetErrorString(e2), hipGetErrorString(e3), hipGetErrorString(e4));
  }
  if (hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0) != hipSuccess) {
    ds_serve_free(p);
    return fail(DS_ERR_HIP, "graph instantiation failed");
  }
  return DS_OK;
}

int ds_serve_submit(ds_plan* p, const ds_problem* prob, uint64_t* ticket) {
  if (!p || !prob || !ticket) return fail(DS_ERR_INVALID, "NULL argument");
  Serve* sv = p->serve;
  if (!sv) return fail(DS_ERR_STATE, "serving not started");
  if (int rc = validate_problem(p, *prob, true)) return rc;
  if (tiles_for(prob->n_seeds, prob->horizon) > MAX_TILES_PER_REQ)
    return fail(DS_ERR_INVALID, "request needs more than %d wavefront tiles", MAX_TILES_PER_REQ);
  if ((int)sv->queue.size() >= sv->queue_cap) return fail(DS_ERR_BUSY, "queue full");
  uint64_t t = sv->next_ticket++;
  ServeReq r;
  r.prob = *prob;
  r.t_submit = now_s();
  if (sv->first_submit < 0) sv->first_submit = r.t_submit;
  sv->reqs[t] = std::move(r);
  sv->queue.push_back(t);
  *ticket = t;
  return DS_OK;
}

int ds_serve_step(ds_plan* p) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  Serve* sv = p->serve;
  if (!sv) return fail(DS_ERR_STATE, "serving not started");
  if (int rc = collect(p, sv, (int)sv->inflight.size() >= DEPTH)) return rc;
  poll_deferred(p, false);
  if (int rc = admit(p, sv)) return rc;
  sv->host_slots.assign(1, 0);
  for (int i = 0; i < sv->max_slots; ++i)
    if (sv->slots[i].ticket) sv->host_slots.push_back(i);
  int active = (int)sv->host_slots.size() - 1;
  if (active == 0) return 0;
  sv->host_slots[0] = active;
  // iterations of this replay: block_iters; with serve_drain and nobody
  // waiting, the active requests run to completion in one replay
  int block = std::max(1, p->params.block_iters);
  if (p->params.drain && sv->queue.empty()) {
    for (int i = 1; i <= active; ++i)
      block = std::max(block, sv->reqs[sv->slots[sv->host_slots[i]].ticket].iters_left);
  }
  if (block != sv->block) sv->lists_dirty = true;
  if (sv->lists_dirty) {
    // slot list, then the tile list at its fixed offset: one upload, only
    // when the membership changed
    const size_t ns = sv->slot_list_bytes / sizeof(int);
    sv->host_lists.assign(ns + 1, 0);
    std::copy(sv->host_slots.begin(), sv->host_slots.end(), sv->host_lists.begin());
    sv->host_lists[sv->max_slots + 1] = block;
    for (int i = 1; i <= active; ++i) {
      const int slot = sv->host_slots[i];
      for (int k = 0; k < sv->slots[slot].ntiles; ++k)
        sv->host_lists.push_back(slot * MAX_TILES_PER_REQ + k);
    }
    sv->host_lists[ns] = (int)(sv->host_lists.size() - ns - 1);
    if (int rc = upload(p, sv->slot_list_dev, sv->host_lists.data(),
                        sv->host_lists.size() * sizeof(int), sv->stream))
      return rc;
    sv->lists_dirty = false;
    sv->block = block;
  }
  if (int rc = timed_launch(p, sv->stream, [&]() { return hipGraphLaunch(sv->exec, sv->stream); }))
    return rc;
  Replay rp;
  rp.seq = sv->steps;
  Landing* set = sv->landing + (size_t)(rp.seq % DEPTH) * sv->max_slots;
  for (int i = 1; i <= active; ++i) {
    const int slot = sv->host_slots[i];
    Slot& sl = sv->slots[slot];
    ServeReq& r = sv->reqs[sl.ticket];
    r.iters_left -= block;
    if (r.iters_left > 0) continue;
    // last block of this request: land its result behind the replay, free
    // the slot, release its memory once the copies are done
    HIP_TRY(hipMemcpyAsync(&set[slot], sl.result,
                           offsetof(Landing, traj) + (size_t)r.prob.horizon * NJ * sizeof(float),
                           hipMemcpyDeviceToHost, sv->stream));
    if (int rc = defer_free(p, sl.state_off, sv->stream)) return rc;
    if (int rc = defer_free(p, sl.out_off, sv->stream)) return rc;
    rp.finishing.push_back({sl.ticket, slot});
    sl = Slot{};
    sv->lists_dirty = true;
  }
  rp.done = get_event(p);
  if (!rp.done) return fail(DS_ERR_HIP, "event creation failed");
  HIP_TRY(hipEventRecord(rp.done, sv->stream));
  sv->inflight.push_back(std::move(rp));
  sv->steps++;
  sv->active_sum += active;
  return active;
}

int ds_serve_poll(ds_plan* p, uint64_t ticket, ds_result* out, float* traj_host) {
  if (!p || !out) return fail(DS_ERR_INVALID, "NULL argument");
  Serve* sv = p->serve;
  if (!sv) return fail(DS_ERR_STATE, "serving not started");
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(DS_ERR_NOT_FOUND, "unknown ticket");
  if (!it->second.done) {
    if (int rc = collect(p, sv, false)) return rc;
    if (!it->second.done) return DS_ERR_STATE;
  }
  *out = it->second.result;
  if (traj_host && !it->second.best.empty())
    std::memcpy(traj_host, it->second.best.data(), it->second.best.size() * sizeof(float));
  sv->reqs.erase(it);
  return DS_OK;
}

int ds_serve_stats(ds_plan* p, ds_latency_stats* out) {
  if (!p || !out) return fail(DS_ERR_INVALID, "NULL argument");
  Serve* sv = p->serve;
  if (!sv) return fail(DS_ERR_STATE, "serving not started");
  std::vector<double> v = sv->lat_ms;
  std::sort(v.begin(), v.end());
  auto q = [&](double f) {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(f * v.size()) - 1);
    return v[i];
  };
  out->completed = (int64_t)v.size();
  out->p50_ms = q(0.50);
  out->p99_ms = q(0.99);
  double s = 0;
  for (double x : v) s += x;
  out->mean_ms = v.empty() ? 0.0 : s / v.size();
  out->max_ms = v.empty() ? 0.0 : v.back();
  double span = sv->last_done - sv->first_submit;
  out->problems_per_s = (span > 0 && !v.empty()) ? v.size() / span : 0.0;
  out->steps = sv->steps;
  out->mean_active_slots = sv->steps ? sv->active_sum / sv->steps : 0.0;
  return DS_OK;
}

int ds_serve_stop(ds_plan* p) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  if (!p->serve) return fail(DS_ERR_STATE, "serving not started");
  ds_serve_free(p);
  return DS_OK;
}

}  // extern "C"
