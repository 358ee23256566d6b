// Serving loop of the dsopt C ABI: continuous batching of planning requests.
//
// Requests wait in a FIFO queue and are admitted into device slots while a
// slot is free and the arena can hold the request's optimiser state.  One
// step = retire the requests whose last iteration block has completed,
// admit waiting ones, publish the active tile list, then replay a captured
// HIP graph (counter reset kernel, persistent optimiser over the tile list
// for block_iters iterations, best-seed kernel over the active slots).  The
// graph is captured once with fixed arguments; membership changes only
// through the device tables the host rewrites between replays, so requests
// that arrive while others run overlap with them on the device.  Every
// tile keeps its own state and iteration count, so a request's arithmetic
// is the same as when it is optimised alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "dsopt_plan.h"

using namespace dsh;

namespace {

constexpr int MAX_TILES_PER_REQ = 128;

struct ServeReq {
  ds_problem prob;
  double t_submit = 0, t_done = 0;
  int slot = -1;
  int blocks_left = 0;
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
  int* tile_list_dev = nullptr;   // [0] = count, then tile indices
  int* slot_list_dev = nullptr;   // [0] = count, then slot indices
  int* counter_dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t replay_done = nullptr;
  bool in_flight = false;
  std::vector<Slot> slots;
  std::deque<uint64_t> queue;
  std::map<uint64_t, ServeReq> reqs;
  uint64_t next_ticket = 1;
  // statistics
  std::vector<double> lat_ms;
  double first_submit = -1, last_done = 0;
  int64_t steps = 0;
  double active_sum = 0;
  std::vector<int> host_tiles, host_slots;
};

void ds_serve_free(ds_plan* p) {
  if (!p || !p->serve) return;
  Serve* sv = p->serve;
  if (sv->in_flight) hipEventSynchronize(sv->replay_done);
  for (auto& sl : sv->slots) {
    if (sl.state_off != SIZE_MAX) p->arena.release(sl.state_off);
    if (sl.out_off != SIZE_MAX) p->arena.release(sl.out_off);
  }
  if (sv->tab_off != SIZE_MAX) p->arena.release(sv->tab_off);
  if (sv->exec) hipGraphExecDestroy(sv->exec);
  if (sv->graph) hipGraphDestroy(sv->graph);
  if (sv->replay_done) hipEventDestroy(sv->replay_done);
  if (sv->own_stream) hipStreamDestroy(sv->stream);
  delete sv;
  p->serve = nullptr;
}

namespace {

int retire(ds_plan* p, Serve* sv) {
  if (!sv->in_flight) return DS_OK;
  HIP_TRY(hipEventSynchronize(sv->replay_done));
  sv->in_flight = false;
  std::vector<int> finished;
  for (int i = 0; i < sv->max_slots; ++i) {
    Slot& sl = sv->slots[i];
    if (!sl.ticket) continue;
    ServeReq& r = sv->reqs[sl.ticket];
    if (--r.blocks_left <= 0) finished.push_back(i);
  }
  for (int i : finished) {
    Slot& sl = sv->slots[i];
    ServeReq& r = sv->reqs[sl.ticket];
    HIP_TRY(hipMemcpyAsync(&r.result, sl.result, sizeof(ds_result), hipMemcpyDeviceToHost,
                           sv->stream));
    r.best.resize((size_t)r.prob.horizon * NJ);
    HIP_TRY(hipMemcpyAsync(r.best.data(), sl.best_traj, r.best.size() * sizeof(float),
                           hipMemcpyDeviceToHost, sv->stream));
  }
  if (!finished.empty()) HIP_TRY(hipStreamSynchronize(sv->stream));
  double t = now_s();
  for (int i : finished) {
    Slot& sl = sv->slots[i];
    ServeReq& r = sv->reqs[sl.ticket];
    r.done = true;
    r.t_done = t;
    sv->lat_ms.push_back((t - r.t_submit) * 1e3);
    sv->last_done = t;
    p->arena.release(sl.state_off);
    p->arena.release(sl.out_off);
    sl = Slot{};
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
    int B = std::max(1, p->params.block_iters);
    r.blocks_left = std::max(1, (p->params.n_iters + B - 1) / B);
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
  size_t d = (((size_t)max_slots + 1) * sizeof(int) + 255) / 256 * 256;
  sv->tab_off = arena_alloc(p, a + b + c + d + 256);
  if (sv->tab_off == SIZE_MAX) {
    ds_serve_free(p);
    return fail(DS_ERR_NOMEM, "arena full (serving tables)");
  }
  uint8_t* base = p->arena.ptr(sv->tab_off);
  sv->probs_dev = reinterpret_cast<ProbDev*>(base);
  sv->tiles_dev = reinterpret_cast<TileDev*>(base + a);
  sv->tile_list_dev = reinterpret_cast<int*>(base + a + b);
  sv->slot_list_dev = reinterpret_cast<int*>(base + a + b + c);
  sv->counter_dev = reinterpret_cast<int*>(base + a + b + c + d);
  // empty lists before the first replay
  HIP_TRY(hipMemsetAsync(base, 0, a + b + c + d + 256, sv->stream));
  HIP_TRY(hipEventCreateWithFlags(&sv->replay_done, hipEventDisableTiming));
  // capture one iteration block over whatever the tables hold at replay time
  int grid = std::max(1, p->cu_count * p->blocks_per_cu);
  HIP_TRY(hipStreamSynchronize(sv->stream));
  HIP_TRY(hipStreamBeginCapture(sv->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = launch_zero_i32(sv->counter_dev, 1, sv->stream);
  hipError_t e2 = launch_serve_step(p->robot_dev, p->params_dev, sv->probs_dev, sv->tiles_dev,
                                    sv->tile_list_dev, sv->counter_dev, (int)max_tiles, grid,
                                    p->params.block_iters, p->params.waves,
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
  if (int rc = retire(p, sv)) return rc;
  if (int rc = admit(p, sv)) return rc;
  sv->host_tiles.assign(1, 0);
  sv->host_slots.assign(1, 0);
  for (int i = 0; i < sv->max_slots; ++i) {
    const Slot& sl = sv->slots[i];
    if (!sl.ticket) continue;
    sv->host_slots.push_back(i);
    for (int k = 0; k < sl.ntiles; ++k) sv->host_tiles.push_back(i * MAX_TILES_PER_REQ + k);
  }
  int active = (int)sv->host_slots.size() - 1;
  if (active == 0) return 0;
  sv->host_tiles[0] = (int)sv->host_tiles.size() - 1;
  sv->host_slots[0] = active;
  if (int rc = upload(p, sv->tile_list_dev, sv->host_tiles.data(),
                      sv->host_tiles.size() * sizeof(int), sv->stream))
    return rc;
  if (int rc = upload(p, sv->slot_list_dev, sv->host_slots.data(),
                      sv->host_slots.size() * sizeof(int), sv->stream))
    return rc;
  if (int rc = timed_launch(p, sv->stream, [&]() { return hipGraphLaunch(sv->exec, sv->stream); }))
    return rc;
  HIP_TRY(hipEventRecord(sv->replay_done, sv->stream));
  sv->in_flight = true;
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
  if (!it->second.done) return DS_ERR_STATE;
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
