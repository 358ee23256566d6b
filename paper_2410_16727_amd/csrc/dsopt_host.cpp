// Host side of the dsopt C ABI: plan, caller-owned device arena, resident
// scenes, problem/tile tables, launches, results and the serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "dsopt_plan.h"

namespace dsh {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

hipEvent_t get_event(ds_plan* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}
void put_event(ds_plan* p, hipEvent_t e) {
  if (e) p->event_pool.push_back(e);
}

void poll_deferred(ds_plan* p, bool wait) {
  std::vector<std::pair<hipEvent_t, size_t>> keep;
  for (auto& d : p->deferred) {
    bool done = wait ? (hipEventSynchronize(d.first) == hipSuccess)
                     : (hipEventQuery(d.first) == hipSuccess);
    if (done) {
      p->arena.release(d.second);
      put_event(p, d.first);
    } else {
      keep.push_back(d);
    }
  }
  p->deferred.swap(keep);
}

int defer_free(ds_plan* p, size_t off, hipStream_t s) {
  hipEvent_t e = get_event(p);
  if (!e) return fail(DS_ERR_HIP, "event creation failed");
  HIP_TRY(hipEventRecord(e, s));
  p->deferred.emplace_back(e, off);
  return DS_OK;
}

size_t arena_alloc(ds_plan* p, size_t bytes) {
  size_t off = p->arena.alloc(bytes);
  if (off == SIZE_MAX) {
    poll_deferred(p, true);
    off = p->arena.alloc(bytes);
  }
  return off;
}

// Copy host bytes into device memory on stream s through the pinned ring.
int upload(ds_plan* p, void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes > p->staging_cap) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DS_OK;
  }
  size_t need = (bytes + 255) / 256 * 256;
  if (p->staging_pos + need > p->staging_cap) {
    for (hipEvent_t e : p->staging_events) {
      hipEventSynchronize(e);
      put_event(p, e);
    }
    p->staging_events.clear();
    p->staging_pos = 0;
  }
  uint8_t* h = p->staging + p->staging_pos;
  p->staging_pos += need;
  std::memcpy(h, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
  hipEvent_t e = get_event(p);
  if (!e) return fail(DS_ERR_HIP, "event creation failed");
  HIP_TRY(hipEventRecord(e, s));
  p->staging_events.push_back(e);
  return DS_OK;
}

bool finite_all(const float* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int group_size(int T) { return T <= 16 ? 16 : (T <= 32 ? 32 : 64); }

int validate_problem(ds_plan* p, const ds_problem& pr, bool need_seeds) {
  if (!p->scenes.count(pr.scene_id))
    return fail(DS_ERR_NOT_FOUND, "scene %d is not resident", pr.scene_id);
  if (need_seeds) {
    if (pr.n_seeds < 1) return fail(DS_ERR_INVALID, "n_seeds must be >= 1 (got %d)", pr.n_seeds);
    if (pr.horizon < DS_MIN_T || pr.horizon > DS_MAX_T)
      return fail(DS_ERR_INVALID, "horizon %d outside [%d, %d]", pr.horizon, DS_MIN_T, DS_MAX_T);
    if (!pr.seeds) return fail(DS_ERR_INVALID, "seeds pointer is NULL");
  }
  if (!finite_all(pr.q_start, 7) || !finite_all(pr.goal, 7))
    return fail(DS_ERR_INVALID, "q_start / goal must be finite");
  double n = 0;
  for (int k = 3; k < 7; ++k) n += (double)pr.goal[k] * pr.goal[k];
  if (!(n > 1e-12)) return fail(DS_ERR_INVALID, "goal quaternion is zero");
  return DS_OK;
}

ProbDev make_probdev(ds_plan* p, const ds_problem& pr) {
  ProbDev d{};
  d.sc = p->scenes[pr.scene_id].dev;
  std::memcpy(d.qs, pr.q_start, sizeof d.qs);
  std::memcpy(d.pd, pr.goal, 3 * sizeof(float));
  std::memcpy(d.quat, pr.goal + 3, 4 * sizeof(float));
  d.S = pr.n_seeds;
  d.T = pr.horizon;
  d.G = group_size(pr.horizon);
  d.n_iters = p->params.n_iters;
  d.seeds = pr.seeds;
  d.out_traj = pr.out_traj;
  return d;
}

// Problem outputs: [seed results][result (256 B)][best trajectory (2 KiB)]
// [final trajectories S x T x 7].
size_t out_bytes(int S, int T) {
  return ((size_t)S * sizeof(ds_seed_result) + 255) / 256 * 256 + 256 + 2048 +
         (size_t)S * T * NJ * sizeof(float);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int alloc_problem_outputs(ds_plan* p, ProblemRec& rec) {
  size_t ob = out_bytes(rec.S, rec.T);
  rec.out_off = arena_alloc(p, ob);
  if (rec.out_off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full (problem outputs, %zu B)", ob);
  uint8_t* base = p->arena.ptr(rec.out_off);
  rec.seed_res = reinterpret_cast<ds_seed_result*>(base);
  size_t sr = ((size_t)rec.S * sizeof(ds_seed_result) + 255) / 256 * 256;
  rec.result = reinterpret_cast<ds_result*>(base + sr);
  rec.best_traj = reinterpret_cast<float*>(base + sr + 256);
  rec.final_traj = reinterpret_cast<float*>(base + sr + 256 + 2048);
  return DS_OK;
}

void free_problem(ds_plan* p, ProblemRec& rec) {
  if (rec.state_off != SIZE_MAX) p->arena.release(rec.state_off);
  if (rec.out_off != SIZE_MAX) p->arena.release(rec.out_off);
  rec.state_off = rec.out_off = SIZE_MAX;
  if (rec.launch) {
    if (--rec.launch->refs == 0) {
      if (rec.launch->tab_off != SIZE_MAX) p->arena.release(rec.launch->tab_off);
      if (rec.launch->land_off != SIZE_MAX) p->land_pool.release(rec.launch->land_off);
      put_event(p, rec.launch->done);
    }
    rec.launch.reset();
  }
}

// One wavefront per seed: the 64/G lanes of a waypoint split its spheres.
int tiles_for(int S, int T) {
  (void)T;
  return S;
}

// Build and launch one optimisation over problems[0..n).
int run_optimize(ds_plan* p, const ds_problem* probs, int n, hipStream_t s, float* tr_x,
                 float* tr_g, float* tr_J, float* tr_d, float* tr_a) {
  poll_deferred(p, false);
  for (int i = 0; i < n; ++i) {
    int rc = validate_problem(p, probs[i], true);
    if (rc) return rc;
    if (p->problems.count(probs[i].problem_tag))
      return fail(DS_ERR_INVALID, "problem tag %d is still live (release it first)",
                  probs[i].problem_tag);
    for (int k = 0; k < i; ++k)
      if (probs[k].problem_tag == probs[i].problem_tag)
        return fail(DS_ERR_INVALID, "duplicate problem tag %d in one call", probs[i].problem_tag);
  }
  std::vector<ProbDev> pd(n);
  std::vector<TileDev> td;
  std::vector<ProblemRec> recs(n);
  size_t state_total = 0;
  for (int i = 0; i < n; ++i) state_total += (size_t)tiles_for(probs[i].n_seeds, probs[i].horizon) * ST_BYTES;
  auto launch = std::make_shared<LaunchRec>();
  int total_tiles = 0;
  for (int i = 0; i < n; ++i) total_tiles += tiles_for(probs[i].n_seeds, probs[i].horizon);
  // tables: problems, tiles, the queue counters and bounds (256 B), the
  // ordered queues (one int per tile), landing records
  const size_t land_at = ((size_t)n * sizeof(ProbDev) + 255) / 256 * 256 +
                         ((size_t)total_tiles * sizeof(TileDev) + 255) / 256 * 256 + 256 +
                         ((size_t)total_tiles * sizeof(int) + 255) / 256 * 256;
  size_t tab_bytes = land_at + (size_t)n * LAND_BYTES;
  launch->tab_off = arena_alloc(p, tab_bytes);
  if (launch->tab_off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full (tables)");
  // results land in pinned host memory when the pool has room (else
  // ds_get_best copies them synchronously)
  launch->land_off = p->land_pool.alloc((size_t)n * LAND_BYTES);
  auto cleanup = [&]() {
    for (auto& r : recs) {
      if (r.state_off != SIZE_MAX) p->arena.release(r.state_off);
      if (r.out_off != SIZE_MAX) p->arena.release(r.out_off);
    }
    p->arena.release(launch->tab_off);
    if (launch->land_off != SIZE_MAX) p->land_pool.release(launch->land_off);
  };
  for (int i = 0; i < n; ++i) {
    const ds_problem& pr = probs[i];
    ProblemRec& rec = recs[i];
    rec.tag = pr.problem_tag;
    rec.S = pr.n_seeds;
    rec.T = pr.horizon;
    int nt = tiles_for(rec.S, rec.T);
    rec.state_off = arena_alloc(p, (size_t)nt * ST_BYTES);
    if (rec.state_off == SIZE_MAX) {
      cleanup();
      return fail(DS_ERR_NOMEM, "arena full (optimiser state, %zu B)", (size_t)nt * ST_BYTES);
    }
    if (int rc = alloc_problem_outputs(p, rec)) {
      cleanup();
      return rc;
    }
    pd[i] = make_probdev(p, pr);
    pd[i].final_traj = rec.final_traj;
    pd[i].seed_res = rec.seed_res;
    pd[i].result = rec.result;
    pd[i].best_traj = rec.best_traj;
    pd[i].landing = p->arena.ptr(launch->tab_off) + land_at + (size_t)i * LAND_BYTES;
    if (launch->land_off != SIZE_MAX)
      rec.land = p->land_host + launch->land_off + (size_t)i * LAND_BYTES;
    if (n == 1) {
      pd[i].tr_x = tr_x; pd[i].tr_g = tr_g; pd[i].tr_J = tr_J; pd[i].tr_d = tr_d; pd[i].tr_a = tr_a;
    }
    for (int k = 0; k < nt; ++k) {
      TileDev t{};
      t.prob = i;
      t.seed0 = k;
      t.nseed = 1;
      t.G = pd[i].G;
      t.state = reinterpret_cast<float*>(p->arena.ptr(rec.state_off) + (size_t)k * ST_BYTES);
      td.push_back(t);
    }
  }
  // Batched launches: one tile queue per XCD.  Problems go to the XCD with
  // the least work so far, largest first, so each problem's tiles -- and
  // the records of its scene -- stay in one XCD's L2; inside a queue the
  // longest tiles come first (a tile's time grows with its group size, and
  // the short ones then fill the tail).  A problem's work is counted as
  // S G: a seed runs at wavefront width whatever its horizon inside the
  // lane group, and counting the long, most variable 64-lane seeds at more
  // than their mean time spreads them over the XCDs.  Per-seed arithmetic
  // does not depend on the order.
  std::vector<int> xcd_ranges;
  if (n > 1) {
    constexpr int NX = N_XCD;
    std::vector<int> order(n), owner(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto work = [&](int i) { return (long long)probs[i].n_seeds * pd[i].G; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    long long load[NX] = {0};
    for (int i : order) {
      int best = 0;
      for (int x = 1; x < NX; ++x)
        if (load[x] < load[best]) best = x;
      owner[i] = best;
      load[best] += work(i);
    }
    std::stable_sort(td.begin(), td.end(), [&](const TileDev& a, const TileDev& b) {
      if (owner[a.prob] != owner[b.prob]) return owner[a.prob] < owner[b.prob];
      return a.G > b.G;
    });
    xcd_ranges.assign(NX + 1, 0);
    for (const TileDev& t : td) xcd_ranges[owner[t.prob] + 1]++;
    for (int x = 0; x < NX; ++x) xcd_ranges[x + 1] += xcd_ranges[x];
  }
  uint8_t* tab = p->arena.ptr(launch->tab_off);
  ProbDev* pd_dev = reinterpret_cast<ProbDev*>(tab);
  size_t off_t = ((size_t)n * sizeof(ProbDev) + 255) / 256 * 256;
  TileDev* td_dev = reinterpret_cast<TileDev*>(tab + off_t);
  int* counter = reinterpret_cast<int*>(tab + off_t + ((size_t)total_tiles * sizeof(TileDev) + 255) / 256 * 256);
  // the tile-queue counters (N_XCD ints) and, for a batched launch, the
  // queues' bounds after them
  const size_t off_c = off_t + ((size_t)total_tiles * sizeof(TileDev) + 255) / 256 * 256;
  const int* ranges_dev = xcd_ranges.empty() ? nullptr : counter + N_XCD;
  // problem and tile tables (and the queue bounds) in one copy: they are
  // adjacent in the arena
  {
    std::vector<uint8_t> tabh(xcd_ranges.empty() ? off_t + td.size() * sizeof(TileDev)
                                                 : off_c + N_XCD * sizeof(int) +
                                                       xcd_ranges.size() * sizeof(int),
                              0);
    std::memcpy(tabh.data(), pd.data(), n * sizeof(ProbDev));
    std::memcpy(tabh.data() + off_t, td.data(), td.size() * sizeof(TileDev));
    if (!xcd_ranges.empty())
      std::memcpy(tabh.data() + off_c + N_XCD * sizeof(int), xcd_ranges.data(),
                  xcd_ranges.size() * sizeof(int));
    if (int rc = upload(p, tab, tabh.data(), tabh.size(), s)) return rc;
  }
  // fresh tiles (iteration counters and seed results start at zero) and an
  // empty tile queue
  if (total_tiles > 0) {
    HIP_TRY(launch_tile_reset(td_dev, pd_dev, total_tiles, counter, s));
  } else {
    HIP_TRY(launch_zero_i32(counter, 1, s));
  }
  const int W = p->params.waves;
  const int per_block = W > 1 ? 1 : WAVES_PER_BLOCK;
  int blocks = (total_tiles + per_block - 1) / per_block;
  blocks = std::max(1, std::min(blocks, p->cu_count * p->blocks_per_cu));
  // A batched launch with more tiles than resident wavefronts (or teams)
  // first runs every tile's initial evaluation, then orders each queue
  // longest expected tile first (lane group, then cost at the seed) and
  // runs the iterations: the long seeds start in the first round instead
  // of the tail.  A seed resumes exactly where the initial launch left it.
  const int slots = p->cu_count * p->blocks_per_cu * per_block;
  const bool ordered = !xcd_ranges.empty() && total_tiles > slots && p->params.n_iters > 0;
  int* list_dev = counter + 64;   // after the 256-byte counter slot
  if (int rc = timed_launch(p, s, [&]() {
        if (ordered) {
          hipError_t e = launch_optimize(p->robot_dev, p->params_dev, pd_dev, td_dev, total_tiles,
                                         counter, blocks, 0, W, params_ext(p->params), s,
                                         ranges_dev);
          if (e != hipSuccess) return e;
          e = launch_queue_order(td_dev, ranges_dev, list_dev, counter, s);
          if (e != hipSuccess) return e;
        }
        return launch_optimize(p->robot_dev, p->params_dev, pd_dev, td_dev, total_tiles, counter,
                               blocks, p->params.n_iters, W, params_ext(p->params), s,
                               ranges_dev, ordered ? list_dev : nullptr);
      }))
    return rc;
  HIP_TRY(launch_best(pd_dev, n, nullptr, s));
  if (launch->land_off != SIZE_MAX)
    HIP_TRY(hipMemcpyAsync(p->land_host + launch->land_off, tab + land_at, (size_t)n * LAND_BYTES,
                           hipMemcpyDeviceToHost, s));
  launch->done = get_event(p);
  if (!launch->done) return fail(DS_ERR_HIP, "event creation failed");
  HIP_TRY(hipEventRecord(launch->done, s));
  launch->refs = n;
  for (int i = 0; i < n; ++i) {
    recs[i].launch = launch;
    p->problems[recs[i].tag] = recs[i];
  }
  return DS_OK;
}

}  // namespace dsh

using namespace dsh;

// ====================================================================== ABI ==
extern "C" {

int ds_version(void) { return DS_VERSION; }
const char* ds_last_error(void) { return g_err.c_str(); }

int ds_plan_create(const ds_robot* robot, const ds_params* prm, void* arena_dev,
                   size_t arena_bytes, ds_plan** out) {
  if (!out) return fail(DS_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!robot || !prm || !arena_dev) return fail(DS_ERR_INVALID, "robot/params/arena is NULL");
  if (arena_bytes < (1u << 20)) return fail(DS_ERR_INVALID, "arena must be >= 1 MiB");
  if (robot->n_joints != 7) return fail(DS_ERR_INVALID, "n_joints must be 7");
  if (robot->n_spheres < 1 || robot->n_spheres > DS_MAX_SPHERES || !robot->spheres)
    return fail(DS_ERR_INVALID, "n_spheres must be in [1, %d]", DS_MAX_SPHERES);
  if (!finite_all(&robot->joint_frame[0][0], 84) || !finite_all(robot->ee_frame, 12))
    return fail(DS_ERR_INVALID, "frames must be finite");
  for (int j = 0; j < 7; ++j)
    if (!(robot->q_lo[j] < robot->q_hi[j])) return fail(DS_ERR_INVALID, "q_lo must be < q_hi");
  for (int s = 0; s < robot->n_spheres; ++s) {
    const ds_sphere& sp = robot->spheres[s];
    if (sp.link < 1 || sp.link > 7) return fail(DS_ERR_INVALID, "sphere %d: link must be 1..7", s);
    if (!finite_all(sp.offset, 3) || !(sp.radius >= 0) || !std::isfinite(sp.radius))
      return fail(DS_ERR_INVALID, "sphere %d: bad offset/radius", s);
  }
  if (!std::isfinite(prm->w_self) || prm->swept_samples < 0 || prm->swept_samples > 8 ||
      !(prm->eps > 0) || prm->history < 1 || prm->history > DS_MAX_HISTORY || prm->n_ls < 1 ||
      prm->n_ls > DS_MAX_LS || prm->n_iters < 0 || prm->block_iters < 1 || !(prm->dt > 0) ||
      !(prm->delta0 > 0) || !(prm->step_max > 0) || !(prm->v_limit > 0) ||
      !(prm->a_limit > 0) || !(prm->j_limit > 0) ||
      !(prm->waves_per_seed == 1 || prm->waves_per_seed == 2 || prm->waves_per_seed == 4 ||
        prm->waves_per_seed == 8))
    return fail(DS_ERR_INVALID, "invalid parameters");

  auto p = std::make_unique<ds_plan>();
  HIP_TRY(hipGetDevice(&p->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, p->device));
  p->cu_count = prop.multiProcessorCount;
  p->arena.init(static_cast<uint8_t*>(arena_dev), arena_bytes);

  RobotDev& rb = p->robot;
  std::memcpy(rb.F, robot->joint_frame, sizeof rb.F);
  std::memcpy(rb.Fee, robot->ee_frame, sizeof rb.Fee);
  std::memcpy(rb.qlo, robot->q_lo, sizeof rb.qlo);
  std::memcpy(rb.qhi, robot->q_hi, sizeof rb.qhi);
  rb.ns = robot->n_spheres;
  std::vector<int> order(rb.ns);
  for (int s = 0; s < rb.ns; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return robot->spheres[a].link < robot->spheres[b].link;
  });
  int cur = 0;
  for (int l = 0; l <= 7; ++l) {
    while (cur < rb.ns && robot->spheres[order[cur]].link <= l) ++cur;
    rb.link_begin[l] = cur;   // spheres of link l+1 start here
  }
  rb.max_per_link = 0;
  for (int l = 0; l < 7; ++l) rb.max_per_link = std::max(rb.max_per_link, rb.link_begin[l + 1] - rb.link_begin[l]);
  rb.axis_links = 0x7F;
  for (int k = 0; k < rb.ns; ++k) {
    const ds_sphere& sp = robot->spheres[order[k]];
    rb.sph[k] = make_float4(sp.offset[0], sp.offset[1], sp.offset[2], sp.radius);
    rb.perm[k] = order[k];
    // a link whose spheres all sit on its z axis takes the short centre form
    if (sp.offset[0] != 0.f || sp.offset[1] != 0.f) rb.axis_links &= ~(1 << (sp.link - 1));
  }
  ParamsDev& P = p->params;
  P.wc = prm->w_collision;
  P.ws = prm->w_self;
  P.eps = prm->eps;
  P.inv_eps = 1.f / prm->eps;
  P.half_inv_eps = 0.5f / prm->eps;
  P.lv = prm->lambda_v; P.la = prm->lambda_a; P.lj = prm->lambda_j;
  P.wp = prm->w_pos; P.wr = prm->w_rot; P.wl = prm->w_limit;
  P.c1 = prm->c1; P.delta0 = prm->delta0; P.dmax = prm->step_max; P.dt = prm->dt;
  P.tol_pos = prm->tol_pos; P.tol_rot = prm->tol_rot;
  P.m = prm->history; P.nls = prm->n_ls; P.n_iters = prm->n_iters; P.block_iters = prm->block_iters;
  P.waves = prm->waves_per_seed;
  P.nsub = prm->swept_samples;
  // float32 trilinear blends stay within 1e-6 of their corner range for
  // distances of metres; the margin keeps the zero-hinge proof exact
  P.far = prm->eps + 1e-5f;
  P.skip = prm->exact_gathers ? 0 : 1;
  P.drain = prm->serve_drain ? 1 : 0;
  P.vlim = prm->v_limit; P.alim = prm->a_limit; P.jlim = prm->j_limit;
  p->blocks_per_cu = optimize_blocks_per_cu(P.waves, params_ext(P));
  // the allocation-free call's device array, resolved once per device
  if (int rc = noalloc_init(p->device)) return rc;

  p->robot_off = p->arena.alloc(sizeof(RobotDev));
  p->params_off = p->arena.alloc(sizeof(ParamsDev));
  p->robot_dev = reinterpret_cast<const RobotDev*>(p->arena.ptr(p->robot_off));
  p->params_dev = reinterpret_cast<const ParamsDev*>(p->arena.ptr(p->params_off));
  HIP_TRY(hipMemcpy((void*)p->robot_dev, &rb, sizeof rb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy((void*)p->params_dev, &P, sizeof P, hipMemcpyHostToDevice));
  {
    const size_t land_cap = 4u << 20;
    HIP_TRY(hipHostMalloc((void**)&p->land_host, land_cap, hipHostMallocDefault));
    p->land_pool.init(p->land_host, land_cap);
  }
  p->staging_cap = 8u << 20;
  HIP_TRY(hipHostMalloc((void**)&p->staging, p->staging_cap, hipHostMallocDefault));
  *out = p.release();
  return DS_OK;
}

void ds_plan_destroy(ds_plan* p) {
  if (!p) return;
  hipDeviceSynchronize();
  ds_serve_free(p);
  poll_deferred(p, true);
  for (auto& kv : p->problems) {
    if (kv.second.launch && kv.second.launch->refs == 1) put_event(p, kv.second.launch->done);
  }
  for (hipEvent_t e : p->staging_events) hipEventDestroy(e);
  for (hipEvent_t e : p->event_pool) hipEventDestroy(e);
  if (p->staging) hipHostFree(p->staging);
  if (p->land_host) hipHostFree(p->land_host);
  delete p;
}

int ds_esdf_upload(ds_plan* p, int32_t scene_id, const float* vals, int nx, int ny, int nz,
                   float voxel, const float origin[3], void* stream) {
  if (!p || !vals || !origin) return fail(DS_ERR_INVALID, "NULL argument");
  if (scene_id < 0) return fail(DS_ERR_INVALID, "scene id must be >= 0");
  if (nx < 2 || ny < 2 || nz < 2) return fail(DS_ERR_INVALID, "grid dims must be >= 2");
  if (!(voxel > 0) || !std::isfinite(voxel) || !finite_all(origin, 3))
    return fail(DS_ERR_INVALID, "voxel must be > 0 and origin finite");
  size_t cells = (size_t)(nx - 1) * (ny - 1) * (nz - 1);
  size_t rec_bytes = cells * 32;
  if (rec_bytes > 0x7fffffffull) return fail(DS_ERR_INVALID, "grid too large (> 2^26 cells)");
  // the kernels form a cell's record index as ix + (nx-1) * ((ny-1) * iz + iy)
  // with 24-bit multiplies: both factors of each product must stay below 2^24
  if ((size_t)(ny - 1) * (nz - 1) >= (1u << 24) || (size_t)(nx - 1) >= (1u << 24))
    return fail(DS_ERR_INVALID, "grid too flat: (ny-1)*(nz-1) must be < 2^24");
  hipStream_t s = static_cast<hipStream_t>(stream);
  poll_deferred(p, false);
  if (p->scenes.count(scene_id)) {
    if (ds_serve_uses_scene(p, scene_id))
      return fail(DS_ERR_BUSY, "scene %d is used by a serving request", scene_id);
    HIP_TRY(hipDeviceSynchronize());
    p->arena.release(p->scenes[scene_id].off);
    p->scenes.erase(scene_id);
  }
  // coarse block size: the smallest 2^s (s >= 2) cells per axis whose table
  // fits COARSE_MAX blocks
  int cshift = 2, cdx, cdy, cdz;
  for (;; ++cshift) {
    const int b = 1 << cshift;
    cdx = (nx - 1 + b - 1) / b;
    cdy = (ny - 1 + b - 1) / b;
    cdz = (nz - 1 + b - 1) / b;
    if ((long long)cdx * cdy * cdz <= COARSE_MAX) break;
  }
  const size_t coarse_at = (rec_bytes + 255) / 256 * 256;
  size_t off = arena_alloc(p, coarse_at + COARSE_BYTES);
  if (off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full (scene %d, %zu B)", scene_id, rec_bytes);
  const float* src = vals;
  size_t tmp_off = SIZE_MAX;
  hipPointerAttribute_t attr;
  bool on_device = false;
  if (hipPointerGetAttributes(&attr, vals) == hipSuccess)
    on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
  (void)hipGetLastError();
  size_t nbytes = (size_t)nx * ny * nz * sizeof(float);
  if (!on_device) {
    tmp_off = arena_alloc(p, nbytes);
    if (tmp_off == SIZE_MAX) {
      p->arena.release(off);
      return fail(DS_ERR_NOMEM, "arena full (scene staging, %zu B)", nbytes);
    }
    HIP_TRY(hipMemcpyAsync(p->arena.ptr(tmp_off), vals, nbytes, hipMemcpyHostToDevice, s));
    src = reinterpret_cast<const float*>(p->arena.ptr(tmp_off));
  }
  HIP_TRY(launch_esdf_pack(src, nx, ny, nz, reinterpret_cast<float4*>(p->arena.ptr(off)), s));
  uint8_t* coarse = p->arena.ptr(off) + coarse_at;
  // one level of the coarse table: the largest sphere's skip distance
  // (radius + far) spans 8 levels, so every sphere's test fits in 15
  float rmax = 0.f;
  for (int k = 0; k < p->robot.ns; ++k) rmax = std::max(rmax, p->robot.sph[k].w);
  const float cq = (rmax + p->params.far) / 8.f;
  HIP_TRY(launch_coarse(src, nx, ny, nz, cshift, cdx, cdy, cdz, cq, coarse, s));
  if (tmp_off != SIZE_MAX)
    if (int rc = defer_free(p, tmp_off, s)) return rc;
  SceneRec rec;
  rec.off = off;
  rec.dev.rec = reinterpret_cast<const float4*>(p->arena.ptr(off));
  rec.dev.nx = nx; rec.dev.ny = ny; rec.dev.nz = nz;
  rec.dev.ox = origin[0]; rec.dev.oy = origin[1]; rec.dev.oz = origin[2];
  rec.dev.inv_h = 1.f / voxel;
  rec.dev.bytes = (uint32_t)rec_bytes;
  rec.dev.coarse = coarse;
  rec.dev.cq = cq;
  rec.dev.cshift = cshift;
  rec.dev.cdx = cdx; rec.dev.cdy = cdy; rec.dev.cdz = cdz;
  p->scenes[scene_id] = rec;
  return DS_OK;
}

int ds_esdf_from_occupancy(ds_plan* p, int32_t scene_id, const uint8_t* occ, int nx, int ny,
                           int nz, float voxel, const float origin[3], float* out_vals,
                           void* stream) {
  if (!p || !occ || !origin) return fail(DS_ERR_INVALID, "NULL argument");
  if (nx < 2 || ny < 2 || nz < 2 || nx > 1024 || ny > 1024 || nz > 1024)
    return fail(DS_ERR_INVALID, "grid dims must be in [2, 1024]");
  if (!(voxel > 0) || !std::isfinite(voxel) || !finite_all(origin, 3))
    return fail(DS_ERR_INVALID, "voxel must be > 0 and origin finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  poll_deferred(p, false);
  const size_t n = (size_t)nx * ny * nz;
  const size_t fb = n * sizeof(float);
  size_t occ_off = SIZE_MAX, work_off = arena_alloc(p, 5 * fb);
  if (work_off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full (distance transform, %zu B)", 5 * fb);
  const uint8_t* occ_dev = occ;
  hipPointerAttribute_t attr;
  bool on_device = false;
  if (hipPointerGetAttributes(&attr, occ) == hipSuccess)
    on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
  (void)hipGetLastError();
  if (!on_device) {
    occ_off = arena_alloc(p, n);
    if (occ_off == SIZE_MAX) {
      p->arena.release(work_off);
      return fail(DS_ERR_NOMEM, "arena full (occupancy staging)");
    }
    HIP_TRY(hipMemcpyAsync(p->arena.ptr(occ_off), occ, n, hipMemcpyHostToDevice, s));
    occ_dev = p->arena.ptr(occ_off);
  }
  float* w = reinterpret_cast<float*>(p->arena.ptr(work_off));
  float* dist = w + 4 * n;
  HIP_TRY(launch_esdf_from_occupancy(occ_dev, nx, ny, nz, voxel, w, w + n, w + 2 * n, w + 3 * n,
                                     dist, s));
  if (out_vals) HIP_TRY(hipMemcpyAsync(out_vals, dist, fb, hipMemcpyDeviceToDevice, s));
  int rc = ds_esdf_upload(p, scene_id, dist, nx, ny, nz, voxel, origin, stream);
  if (int r2 = defer_free(p, work_off, s)) return r2;
  if (occ_off != SIZE_MAX)
    if (int r2 = defer_free(p, occ_off, s)) return r2;
  return rc;
}

int ds_esdf_release(ds_plan* p, int32_t scene_id) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  auto it = p->scenes.find(scene_id);
  if (it == p->scenes.end()) return fail(DS_ERR_NOT_FOUND, "scene %d is not resident", scene_id);
  if (ds_serve_uses_scene(p, scene_id))
    return fail(DS_ERR_BUSY, "scene %d is used by a serving request", scene_id);
  HIP_TRY(hipDeviceSynchronize());
  p->arena.release(it->second.off);
  p->scenes.erase(it);
  return DS_OK;
}

int ds_optimize_seeds(ds_plan* p, const ds_problem* probs, int n, void* stream) {
  if (!p || !probs || n < 1) return fail(DS_ERR_INVALID, "need a plan and n >= 1 problems");
  return run_optimize(p, probs, n, static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr,
                      nullptr, nullptr);
}

int ds_optimize_traced(ds_plan* p, const ds_problem* prob, float* tr_x, float* tr_g,
                       float* tr_J, float* tr_d, float* tr_a, void* stream) {
  if (!p || !prob) return fail(DS_ERR_INVALID, "NULL argument");
  if (!tr_x || !tr_g || !tr_J || !tr_d || !tr_a) return fail(DS_ERR_INVALID, "trace buffer is NULL");
  return run_optimize(p, prob, 1, static_cast<hipStream_t>(stream), tr_x, tr_g, tr_J, tr_d, tr_a);
}

int ds_get_best(ds_plan* p, int32_t tag, float* traj_host, ds_result* out) {
  if (!p || !out) return fail(DS_ERR_INVALID, "NULL argument");
  auto it = p->problems.find(tag);
  if (it == p->problems.end()) return fail(DS_ERR_NOT_FOUND, "unknown problem tag %d", tag);
  ProblemRec& r = it->second;
  HIP_TRY(hipEventSynchronize(r.launch->done));
  if (r.land) {   // landed with the launch
    std::memcpy(out, r.land, sizeof(ds_result));
    if (traj_host && out->best_seed >= 0)
      std::memcpy(traj_host, r.land + 256, (size_t)r.T * NJ * sizeof(float));
    return DS_OK;
  }
  HIP_TRY(hipMemcpy(out, r.result, sizeof(ds_result), hipMemcpyDeviceToHost));
  if (traj_host && out->best_seed >= 0)
    HIP_TRY(hipMemcpy(traj_host, r.best_traj, (size_t)r.T * NJ * sizeof(float),
                      hipMemcpyDeviceToHost));
  return DS_OK;
}

int ds_get_seed_results(ds_plan* p, int32_t tag, ds_seed_result* out, int cap) {
  if (!p || !out || cap < 0) return fail(DS_ERR_INVALID, "bad argument");
  auto it = p->problems.find(tag);
  if (it == p->problems.end()) return fail(DS_ERR_NOT_FOUND, "unknown problem tag %d", tag);
  ProblemRec& r = it->second;
  HIP_TRY(hipEventSynchronize(r.launch->done));
  int n = std::min(cap, r.S);
  HIP_TRY(hipMemcpy(out, r.seed_res, (size_t)n * sizeof(ds_seed_result), hipMemcpyDeviceToHost));
  return DS_OK;
}

int ds_problem_release(ds_plan* p, int32_t tag) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  auto it = p->problems.find(tag);
  if (it == p->problems.end()) return fail(DS_ERR_NOT_FOUND, "unknown problem tag %d", tag);
  HIP_TRY(hipEventSynchronize(it->second.launch->done));
  free_problem(p, it->second);
  p->problems.erase(it);
  return DS_OK;
}

static int cost_common(ds_plan* p, const ds_problem* prob, const float* X, int S, int T,
                       const float* dJ, float* J_out, float* dX, int with_grad, void* stream) {
  if (!p || !prob || !X) return fail(DS_ERR_INVALID, "NULL argument");
  if (S < 1 || T < DS_MIN_T || T > DS_MAX_T) return fail(DS_ERR_INVALID, "bad S/T (%d, %d)", S, T);
  if (with_grad && !dX) return fail(DS_ERR_INVALID, "dX is NULL");
  if (!with_grad && !J_out) return fail(DS_ERR_INVALID, "J_out is NULL");
  if (int rc = validate_problem(p, *prob, false)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  poll_deferred(p, false);
  size_t off = arena_alloc(p, sizeof(ProbDev));
  if (off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full");
  ProbDev pd = make_probdev(p, *prob);
  pd.S = S;
  pd.T = T;
  ProbDev* dev = reinterpret_cast<ProbDev*>(p->arena.ptr(off));
  if (int rc = upload(p, dev, &pd, sizeof pd, s)) return rc;
  HIP_TRY(launch_cost(p->robot_dev, p->params_dev, dev, X, S, T, dJ, J_out, dX, with_grad,
                      params_ext(p->params), p->cu_count, s));
  return defer_free(p, off, s);
}

int ds_cost(ds_plan* p, const ds_problem* prob, const float* X, int S, int T, float* J_out,
            void* stream) {
  return cost_common(p, prob, X, S, T, nullptr, J_out, nullptr, 0, stream);
}

int ds_cost_grad(ds_plan* p, const ds_problem* prob, const float* X, int S, int T,
                 const float* dJ, float* J_out, float* dX, void* stream) {
  return cost_common(p, prob, X, S, T, dJ, J_out, dX, 1, stream);
}

int ds_guide(ds_plan* p, const ds_problem* prob, float* X, int S, int T, float alpha, int n_steps,
             float* J_out, void* stream) {
  if (!p || !prob || !X) return fail(DS_ERR_INVALID, "NULL argument");
  if (S < 1 || T < DS_MIN_T || T > DS_MAX_T) return fail(DS_ERR_INVALID, "bad S/T (%d, %d)", S, T);
  if (n_steps < 0 || !std::isfinite(alpha)) return fail(DS_ERR_INVALID, "bad alpha / n_steps");
  if (int rc = validate_problem(p, *prob, false)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  poll_deferred(p, false);
  size_t off = arena_alloc(p, sizeof(ProbDev));
  if (off == SIZE_MAX) return fail(DS_ERR_NOMEM, "arena full");
  ProbDev pd = make_probdev(p, *prob);
  pd.S = S;
  pd.T = T;
  ProbDev* dev = reinterpret_cast<ProbDev*>(p->arena.ptr(off));
  if (int rc = upload(p, dev, &pd, sizeof pd, s)) return rc;
  HIP_TRY(launch_guide(p->robot_dev, p->params_dev, dev, X, S, T, alpha, n_steps, J_out,
                       params_ext(p->params), p->cu_count, s));
  return defer_free(p, off, s);
}

int ds_kernel_timing(ds_plan* p, int enable) {
  if (!p) return fail(DS_ERR_INVALID, "NULL plan");
  p->timing = enable != 0;
  return DS_OK;
}

int ds_kernel_timing_read(ds_plan* p, double* total_ms, int64_t* launches) {
  if (!p || !total_ms || !launches) return fail(DS_ERR_INVALID, "NULL argument");
  double tot = 0;
  for (auto& ab : p->timed) {
    HIP_TRY(hipEventSynchronize(ab.second));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, ab.first, ab.second));
    tot += ms;
    hipEventDestroy(ab.first);
    hipEventDestroy(ab.second);
  }
  *total_ms = tot;
  *launches = (int64_t)p->timed.size();
  p->timed.clear();
  return DS_OK;
}

int ds_sphere_centres(ds_plan* p, const float* X, int S, int T, float* out, void* stream) {
  if (!p || !X || !out || S < 1 || T < 1) return fail(DS_ERR_INVALID, "bad argument");
  HIP_TRY(launch_spheres(p->robot_dev, X, S, T, out, static_cast<hipStream_t>(stream)));
  return DS_OK;
}

}  // extern "C"


