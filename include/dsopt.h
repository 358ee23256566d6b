/* dsopt: batched seeded trajectory optimisation for a 7-revolute serial arm
 * on AMD Instinct MI355X (gfx950).
 *
 * The library optimises many joint-space seed trajectories per planning
 * problem in parallel, following the problem statement of DiffusionSeeder
 * (arXiv 2410.16727, Sec. 3): a start configuration q_0, a goal end-effector
 * pose given as a translation and a quaternion, a distance field of the
 * scene (Sec. 4.4, ESDF) and seed trajectories of T waypoints x 7 joints.
 * Each seed minimises the objective of App. A.6,
 *     C_goal(X_d, FK(q_{T-1})) + C_smooth(tau) + C_world(tau)
 * subject to joint limits, for a fixed number of iterations (Sec. 4.4,
 * N_iters).  The concrete cost forms are:
 *   - C_world: smooth hinge (activation distance eps) of the trilinearly
 *     interpolated distance minus the sphere radius, summed over all
 *     collision spheres at every waypoint;
 *   - C_smooth: lambda_v |v|^2 + lambda_a |a|^2 + lambda_j |j|^2 of the
 *     first/second/third finite differences of the trajectory padded with
 *     two copies of q_0 before and two of q_{T-1} after (rest at both ends);
 *   - C_goal: w_pos |p_ee - p_d|^2 + w_rot (3 - tr(R_d^T R_ee)) / 4 at the
 *     last waypoint;
 *   - joint limits: w_limit * squared excess outside [q_lo, q_hi];
 *   - optional C_self: w_self * hinge of (|c_a - c_b| - r_a - r_b) over
 *     sphere pairs on links at least two apart.
 * The optimiser is L-BFGS (two-loop recursion) with a backtracking search
 * over step sizes 1, 1/2, ..., 2^-(n_ls-1) (largest step meeting the Armijo
 * condition, else the cheapest candidate below the current cost, else no
 * step).  Waypoint 0 stays equal to q_start.
 *
 * Conventions
 *   - Every call returns DS_OK (0) or a negative DS_ERR_* code; the message
 *     of the last failure on the calling thread is ds_last_error().
 *   - "device" pointers are HIP device memory of the current device;
 *     "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls taking a
 *     stream are asynchronous: borrowed pointers must stay valid until the
 *     stream reaches the enqueued work.
 *   - A plan is driven by one host thread at a time.
 *   - Layouts are row-major C arrays; trajectories are [S][T][7] float32.
 */
#ifndef DSOPT_H
#define DSOPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DS_VERSION 100

#define DS_OK 0
#define DS_ERR_INVALID (-1)   /* bad argument (shape, id, value) */
#define DS_ERR_NOMEM (-2)     /* the caller's arena cannot hold the request */
#define DS_ERR_BUSY (-3)      /* serving queue full, or a scene still in use */
#define DS_ERR_NOT_FOUND (-4) /* unknown scene id / problem tag / ticket */
#define DS_ERR_HIP (-5)       /* a HIP runtime call failed */
#define DS_ERR_STATE (-6)     /* call not valid in the current state */

#define DS_NJ 7            /* joints of the arm */
#define DS_MIN_T 4         /* shortest horizon */
#define DS_MAX_T 64        /* longest horizon: one waypoint per wavefront lane */
#define DS_MAX_SPHERES 128 /* collision spheres per robot */
#define DS_MAX_HISTORY 8   /* L-BFGS memory */
#define DS_MAX_LS 8        /* line-search candidates */

/* One collision sphere, fixed in the frame of link `link` (1..7; link i is
 * the frame after joint i).  Sec. 4.3 samples points on every link; the
 * optimiser uses spheres centred on such points. */
typedef struct ds_sphere {
  int32_t link;
  float offset[3]; /* metres, in the link frame */
  float radius;    /* metres */
} ds_sphere;

/* Serial 7-revolute arm.  Joint i rotates about the z axis of its frame:
 * T_i = T_{i-1} * joint_frame[i-1] * Rz(q_i), T_0 = identity (base at the
 * world origin); the end effector is T_7 * ee_frame. */
typedef struct ds_robot {
  int32_t n_joints;           /* must be 7 */
  int32_t n_spheres;          /* 1..DS_MAX_SPHERES */
  float joint_frame[7][12];   /* 3x4 row-major [R | p] */
  float ee_frame[12];         /* 3x4 row-major [R | p] */
  float q_lo[7], q_hi[7];     /* joint limits, radians, q_lo < q_hi */
  const ds_sphere* spheres;   /* host, n_spheres entries; copied by create */
} ds_robot;

/* Objective weights and optimiser settings (all copied by create). */
typedef struct ds_params {
  float w_collision;   /* C_world weight */
  float eps;           /* hinge activation distance, metres, > 0 */
  float lambda_v, lambda_a, lambda_j; /* smoothness weights (waypoint spacing folded in) */
  float w_pos, w_rot;  /* goal-pose weights */
  float w_limit;       /* joint-limit penalty weight */
  int32_t history;     /* L-BFGS memory, 1..DS_MAX_HISTORY */
  int32_t n_ls;        /* line-search candidates, 1..DS_MAX_LS */
  float c1;            /* Armijo constant */
  float delta0;        /* steepest-descent step length (infinity norm), radians */
  float step_max;      /* infinity-norm cap of a search direction, radians */
  float dt;            /* waypoint spacing in seconds (jerk reporting only) */
  float tol_pos;       /* success threshold on position error, metres (Sec. 5.1: 0.005) */
  float tol_rot;       /* success threshold on rotation error, radians (Sec. 5.1: 2.86 deg) */
  int32_t n_iters;     /* iterations per optimisation (Sec. 4.4, N_iters) */
  int32_t block_iters; /* iterations per serving step (graph replay) */
  int32_t waves_per_seed; /* 1, 2, 4 or 8 wavefronts cooperate on one seed: more
                             parallelism per seed for latency-bound launches (few
                             seeds); results depend on it only through the
                             order of floating-point sums */
  float w_self;        /* self-collision weight (App. A.6 C_self): hinge on the
                          separation of every sphere pair on links at least two
                          apart; 0 switches the term off.  When on, the reported
                          clearance and collision-free flag include these pairs. */
  int32_t swept_samples; /* 0..8 configurations per segment, linearly interpolated
                            between consecutive waypoints (the paper's trajectories
                            are interpolated linearly), add to C_world and to the
                            clearance; their gradient splits (1 - tau, tau) onto
                            the two waypoints.  0: waypoints only. */
  int32_t exact_gathers; /* 0 (default): a sphere sample whose cell lies in a block
                            of the scene's coarse minimum-distance table that
                            clears the sphere by more than eps is not gathered --
                            its hinge and gradient are exactly zero, so results
                            are the same bit for bit.  1: gather every sample
                            (for verifying that equality). */
  int32_t serve_drain;   /* 0 (default): every serving replay runs block_iters
                            iterations of each active request.  1: when no request
                            waits, a replay runs the active requests to completion
                            (lower median latency at light load; a request that
                            arrives meanwhile waits for that replay). */
  float v_limit;         /* joint velocity limit, rad/s, > 0 (App. A.7 motion time: */
  float a_limit;         /* acceleration limit, rad/s^2, > 0  the trajectory slowed */
  float j_limit;         /* jerk limit, rad/s^3, > 0          down to meet them) */
} ds_params;

/* One planning problem (Sec. 3).  `seeds` are the seed trajectories
 * (Sec. 4.3 produces N_trajs of them); row 0 of every seed is replaced by
 * q_start.  goal = [x, y, z, qw, qx, qy, qz]; the quaternion is normalised
 * by the library and must not be zero. */
typedef struct ds_problem {
  int32_t scene_id;    /* a scene uploaded with ds_esdf_upload */
  int32_t n_seeds;     /* S >= 1 */
  int32_t horizon;     /* T, DS_MIN_T..DS_MAX_T */
  int32_t problem_tag; /* caller's id for ds_get_best; unique among live problems */
  float q_start[7];
  float goal[7];
  const float* seeds;  /* device, [S][T][7], borrowed until the stream passes the call */
  float* out_traj;     /* device, [S][T][7] optimised seeds, or NULL */
} ds_problem;

/* Per-problem result (App. A.7 metrics; Sec. 5.1 success criterion). */
typedef struct ds_result {
  int32_t best_seed;       /* lowest-cost successful seed, else lowest-cost valid seed, else -1 */
  int32_t success;         /* best seed is collision free, within limits and within both thresholds */
  int32_t collision_free;  /* of the best seed */
  int32_t n_valid_seeds;   /* seeds whose final cost is finite */
  float pos_err_m;         /* |p_ee - p_d| of the best seed */
  float rot_err_rad;       /* rotation angle between achieved and goal orientation */
  float cost;              /* final objective of the best seed */
  float min_clearance_m;   /* min over waypoints and spheres of (distance - radius) */
  float max_jerk;          /* max |third difference| / dt^3 over waypoints and joints */
  int32_t n_iters;         /* iterations run */
  float max_vel;           /* max |q_{t+1} - q_t| / dt over waypoints and joints */
  float motion_time;       /* App. A.7: (T-1) dt times the smallest uniform slow-down
                              s >= 1 that meets the limits: s = max(1, v/v_limit,
                              sqrt(a/a_limit), cbrt(jerk/j_limit)) */
} ds_result;

/* Per-seed result (the fields of ds_result for every seed, plus the
 * evaluation counters). */
typedef struct ds_seed_result {
  float cost, clearance, pos_err, rot_err, max_jerk;
  int32_t collision_free, within_limits, success, valid;
  int32_t n_evals_cost;    /* cost-only evaluations run for this seed's wavefront */
  int32_t n_evals_grad;    /* cost+gradient evaluations run for this seed's wavefront */
  uint32_t n_gathers;      /* ESDF cell records (32 B each) gathered for this seed,
                              over all its wavefronts and launches; the coarse
                              table's skips are not counted */
  float max_vel;           /* max |q_{t+1} - q_t| / dt */
  float max_acc;           /* max |q_{t+2} - 2 q_{t+1} + q_t| / dt^2 */
  float motion_time;       /* as in ds_result */
  int32_t within_vel;      /* max_vel <= v_limit (reported; not part of success) */
} ds_seed_result;

typedef struct ds_plan ds_plan;

int ds_version(void);
const char* ds_last_error(void);

/* Create a plan.  `arena_dev` is caller-owned device memory of
 * `arena_bytes` (>= 1 MiB) borrowed for the plan's lifetime: every scene,
 * problem state and work table is placed in it, and no device memory is
 * allocated after create.  Fails with DS_ERR_INVALID for a malformed robot
 * or parameter set. */
int ds_plan_create(const ds_robot* robot, const ds_params* params, void* arena_dev,
                   size_t arena_bytes, ds_plan** out);

/* Wait for all work of the plan and free its host-side state (the arena
 * stays the caller's). */
void ds_plan_destroy(ds_plan* plan);

/* Copy a node-centred distance field into the arena (Sec. 4.4: the
 * optimiser reads the scene's ESDF).  `vals` (device or host) holds
 * nx*ny*nz float32 signed distances in metres, x fastest, node (i,j,k) at
 * origin + (i,j,k)*voxel; negative inside obstacles.  The library stores
 * its own gather layout (the 8 corners of every cell in one 32-byte record)
 * and keeps it resident until ds_esdf_release or destroy; re-uploading an
 * id replaces it.  Queries outside the grid are clamped to it.  Errors:
 * DS_ERR_INVALID (dims < 2, voxel <= 0, id < 0, more than 2^26 - 1 cells, or
 * (ny-1)*(nz-1) >= 2^24: cell indices are formed with 24-bit multiplies),
 * DS_ERR_NOMEM, DS_ERR_BUSY (replacing a scene that a serving request
 * still uses).  Releasing waits for all work on the device; it fails with
 * DS_ERR_BUSY while a queued or admitted serving request uses the scene. */
int ds_esdf_upload(ds_plan* plan, int32_t scene_id, const float* vals, int nx, int ny, int nz,
                   float voxel, const float origin[3], void* stream);
int ds_esdf_release(ds_plan* plan, int32_t scene_id);

/* Build a scene's distance field on the GPU from an occupancy grid (the
 * step before the optimiser: the paper builds its ESDF from depth with a
 * GPU mapping library, Sec. 4.4 / Sec. 5.1).  `occ` (device or host) holds
 * nx*ny*nz bytes, x fastest, nonzero = occupied, voxel (i,j,k) centred at
 * origin + (i,j,k)*voxel.  Signed Euclidean distance by definition: a free
 * voxel stores voxel * (distance to the nearest occupied voxel centre), an
 * occupied voxel -voxel * (distance to the nearest free voxel centre),
 * computed exactly by three separable squared-distance passes.  A grid with
 * no occupied (no free) voxel yields values >= 1e9 * voxel in magnitude.
 * The field becomes scene `scene_id` exactly as with ds_esdf_upload;
 * `out_vals` (device, nx*ny*nz floats, may be NULL) receives a copy of the
 * signed distances.  Temporary space (4 * nx*ny*nz floats) comes from the
 * arena.  Errors: DS_ERR_INVALID (dims < 2 or > 1024, voxel <= 0),
 * DS_ERR_NOMEM. */
int ds_esdf_from_occupancy(ds_plan* plan, int32_t scene_id, const uint8_t* occ, int nx, int ny,
                           int nz, float voxel, const float origin[3], float* out_vals,
                           void* stream);

/* Optimise n problems for params.n_iters iterations (Sec. 4.4).  n == 1
 * is the plain one-problem launch; n > 1 runs every seed of every problem
 * in one persistent launch over a work table, longest work first.
 * Per-seed arithmetic does not depend on n or on the batch composition.
 * Asynchronous on `stream`; results via ds_get_best.  Errors:
 * DS_ERR_INVALID (unknown scene, S < 1, T out of range, zero quaternion,
 * duplicate live tag), DS_ERR_NOMEM. */
int ds_optimize_seeds(ds_plan* plan, const ds_problem* probs, int n, void* stream);

/* Same as ds_optimize_seeds for one problem, additionally recording every
 * iteration (device buffers, all float32):
 *   trace_x, trace_g [n_iters+1][S][T][7]  iterate and gradient,
 *   trace_J          [n_iters+1][S]        cost,
 *   trace_d          [n_iters][S][T][7]    search direction,
 *   trace_alpha      [n_iters][S]          accepted step (0 = none). */
int ds_optimize_traced(ds_plan* plan, const ds_problem* prob, float* trace_x, float* trace_g,
                       float* trace_J, float* trace_d, float* trace_alpha, void* stream);

/* Block until problem `problem_tag` is finished; copy the best seed's
 * trajectory ([T][7] host floats, may be NULL) and the result. */
int ds_get_best(ds_plan* plan, int32_t problem_tag, float* traj_host, ds_result* out);

/* Block until finished; copy min(cap, S) per-seed results (host). */
int ds_get_seed_results(ds_plan* plan, int32_t problem_tag, ds_seed_result* out, int cap);

/* Return a finished problem's arena space (waits for it first). */
int ds_problem_release(ds_plan* plan, int32_t problem_tag);

/* Objective of S trajectories X (device [S][T][7], row 0 used as given)
 * for scene/goal of `prob` (its seeds/S/T fields are ignored): J_out
 * (device [S]).  Backs the forward of the autograd function. */
int ds_cost(ds_plan* plan, const ds_problem* prob, const float* X, int S, int T, float* J_out,
            void* stream);

/* Objective and its gradient: J_out (device [S], may be NULL) and
 * dX (device [S][T][7]) = dJ[s] * dJ_s/dX (dJ device [S], or NULL for ones).
 * The gradient recomputes the kinematics (no per-joint transform is
 * stored); row 0 of dX is zero because waypoint 0 is pinned. */
int ds_cost_grad(ds_plan* plan, const ds_problem* prob, const float* X, int S, int T,
                 const float* dJ, float* J_out, float* dX, void* stream);

/* Cost-gradient guidance for seed sampling (the appendix on cost-guided
 * diffusion sampling, Eq. 4: the denoiser mean is moved along the cost
 * gradient, n gradient steps per denoising step).  Runs n_steps steps
 * X <- X - alpha * dJ/dX of the objective for the scene/goal of `prob` on S
 * trajectories X (device [S][T][7], updated in place; row 0 stays fixed)
 * in one launch; J_out (device [S], may be NULL) receives the cost after the
 * last step.  Reading: a descent step (the printed sign would ascend the
 * cost).  Errors as ds_cost_grad; n_steps >= 0. */
int ds_guide(ds_plan* plan, const ds_problem* prob, float* X, int S, int T, float alpha,
             int n_steps, float* J_out, void* stream);

/* Sphere centres of X (device [S][T][7]) into out (device
 * [S][T][n_spheres][3]), in the robot's sphere order (parity checks). */
int ds_sphere_centres(ds_plan* plan, const float* X, int S, int T, float* out, void* stream);

/* Kernel timing: when enabled, every optimiser-kernel launch of the plan is
 * bracketed by HIP events on its stream; ds_kernel_timing_read waits for
 * the recorded launches and returns their summed duration (milliseconds)
 * and count since the last read.  For measurement only. */
int ds_kernel_timing(ds_plan* plan, int enable);
int ds_kernel_timing_read(ds_plan* plan, double* total_ms, int64_t* launches);

/* ---- allocation-free planning ----------------------------------------------
 * For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  ds_optimize_noalloc
 * optimises one problem exactly as ds_optimize_seeds does (the same
 * kernels and per-seed arithmetic, params.n_iters iterations,
 * params.waves_per_seed), but allocates nothing, copies nothing from the
 * host and never waits: the optimiser state, the work tables and the final
 * trajectories live in a fixed device array of the library (about 5.1 MB
 * per GPU, held until the process ends; its address is resolved once per
 * device by ds_plan_create), and the tables are written on the device.
 *   prob          as for ds_optimize_seeds (problem_tag is ignored, nothing
 *                 is registered under it); prob->out_traj, if not NULL,
 *                 receives the optimised seeds [S][T][7]
 *   seed_results  device, [S] per-seed results
 *   result        device, one ds_result (the best seed, as ds_get_best)
 *   best_traj     device, [T][7] the best seed's trajectory
 * Asynchronous on `stream`.  Every call on a GPU shares that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU
 * (two streams, two host threads) race -- order them on one stream.
 * Errors: as ds_optimize_seeds, DS_ERR_INVALID for S > DS_NOALLOC_MAX_SEEDS,
 * DS_ERR_STATE if the array's address is not set up on the plan's device. */
#define DS_NOALLOC_MAX_SEEDS 128
int ds_optimize_noalloc(ds_plan* plan, const ds_problem* prob, ds_seed_result* seed_results,
                        ds_result* result, float* best_traj, void* stream);

/* ---- serving: continuous batching of planning requests -------------------
 * Requests are admitted into device slots while memory and slots allow;
 * every step runs params.block_iters iterations of every admitted request
 * in one captured graph replay, retires finished requests and admits
 * waiting ones.  A request's result equals what ds_optimize_seeds gives for
 * it alone. */
typedef struct ds_latency_stats {
  int64_t completed;
  double p50_ms, p99_ms, mean_ms, max_ms; /* submit -> result ready */
  double problems_per_s;                  /* completed / (last done - first submit) */
  int64_t steps;                          /* graph replays */
  double mean_active_slots;
} ds_latency_stats;

/* Start serving with up to max_slots concurrent requests (1..256) and a
 * waiting queue of queue_cap requests; uses the plan's arena. */
int ds_serve_start(ds_plan* plan, int max_slots, int queue_cap, void* stream);
/* Queue a request; `prob->seeds` must stay valid until its result is
 * polled.  DS_ERR_BUSY when the queue is full. */
int ds_serve_submit(ds_plan* plan, const ds_problem* prob, uint64_t* ticket);
/* Advance the loop by one step: collect completed replays, admit waiting
 * requests, enqueue one replay (block_iters iterations of every active
 * request, or with serve_drain and nobody waiting, the rest of them).  Up to two replays are in flight; the call waits for the oldest
 * only when both are.  Returns the number of requests in the enqueued
 * replay (0: nothing to run) or an error. */
int ds_serve_step(ds_plan* plan);
/* Non-blocking (collects completed replays first): DS_OK with the result
 * when done, DS_ERR_STATE when not yet, DS_ERR_NOT_FOUND for an unknown
 * ticket.  traj_host (horizon x 7 floats) may be NULL. */
int ds_serve_poll(ds_plan* plan, uint64_t ticket, ds_result* out, float* traj_host);
int ds_serve_stats(ds_plan* plan, ds_latency_stats* out);
int ds_serve_stop(ds_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* DSOPT_H */
