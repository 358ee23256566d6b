// Device-side records shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "dsopt.h"

namespace dsk {

constexpr int NJ = 7;
constexpr int WAVE = 64;            // CDNA wavefront
constexpr int WAVES_PER_BLOCK = 4;  // independent tiles per workgroup
constexpr int N_XCD = 8;            // accelerator dies; workgroups are dealt to them in turn
constexpr int BLOCK = WAVE * WAVES_PER_BLOCK;

// Robot table, read with uniform (scalar) loads by every wavefront.
struct RobotDev {
  float F[7][12];        // fixed transform before joint i, 3x4 row-major
  float Fee[12];
  float qlo[7], qhi[7];
  int32_t ns;
  int32_t max_per_link;              // most spheres on one link
  int32_t link_begin[8];             // spheres of link l (1..7): [link_begin[l-1], link_begin[l])
  int32_t axis_links;                // bit l-1: every sphere of link l has zero x and y offsets
  float4 sph[DS_MAX_SPHERES];        // offset xyz, radius; sorted by link
  int32_t perm[DS_MAX_SPHERES];      // sorted position -> caller's sphere index
};

struct ParamsDev {
  float wc, ws, eps, inv_eps, half_inv_eps;
  float lv, la, lj, wp, wr, wl;
  float c1, delta0, dmax, dt, tol_pos, tol_rot;
  int32_t m, nls, n_iters, block_iters;
  int32_t waves;         // wavefronts per seed (1, 2, 4 or 8)
  int32_t nsub;          // swept sub-samples per segment
  float far;             // a block minimum >= radius + far proves a zero hinge
  int32_t skip;          // use the coarse table (0: gather every sample)
  int32_t drain;         // serving: run to completion when nobody waits
  float vlim, alim, jlim;   // velocity / acceleration / jerk limits (motion time)
};

// One resident scene: the 8 corners of cell (i,j,k) are the 32-byte record
// i + (nx-1)*(j + (ny-1)*k): [c000 c100 c010 c110 | c001 c101 c011 c111].
// Coarse table: for each block of 2^cshift cells per axis (x fastest, at
// most COARSE_MAX blocks), a 4-bit level L bounding the minimum node
// distance m over the block's nodes from below: the largest L <= 15 with
// L * cq <= m in float arithmetic (0 when m is negative or NaN); two blocks
// per byte, the even block in the low nibble (16 KB).
constexpr int COARSE_MAX = 32768;
constexpr int COARSE_BYTES = COARSE_MAX / 2;
constexpr int COARSE_FLOATS = COARSE_BYTES / 4;   // the table's size in 4-byte words
struct SceneDev {
  const float4* rec;
  int32_t nx, ny, nz;    // node counts
  float ox, oy, oz, inv_h;
  uint32_t bytes;        // size of the record array
  const uint8_t* coarse;    // [cdz][cdy][cdx] block levels (4 bits each)
  float cq;                 // distance of one level
  int32_t cshift, cdx, cdy, cdz;
};

struct ProbDev {
  SceneDev sc;
  float qs[7];
  float pd[3];
  float quat[4];         // goal quaternion as given (normalised in the kernel)
  int32_t S, T, G;       // seeds, horizon, lanes per seed (16, 32 or 64)
  int32_t n_iters;
  const float* seeds;    // [S][T][7]
  float* out_traj;       // [S][T][7] or null
  float* final_traj;     // arena [S][T][7]
  ds_seed_result* seed_res;   // arena [S]
  ds_result* result;          // arena
  float* best_traj;           // arena [T][7], the best seed's trajectory
  float *tr_x, *tr_g, *tr_J, *tr_d, *tr_a;   // trace buffers or null
  uint8_t* landing;           // null, or LAND_BYTES: result (256 B) then best trajectory
};

// a problem's result record and best trajectory, side by side, for one
// copy to the host
constexpr size_t LAND_BYTES = 256 + (size_t)DS_MAX_T * 7 * sizeof(float);

struct TileDev {
  int32_t prob;          // index into the problem table
  int32_t seed0;         // the tile's seed
  int32_t nseed;         // 1: one seed per wavefront
  int32_t G;             // lanes per copy of the trajectory (64/G copies split the spheres)
  float* state;          // tile state (layout below)
};

// Tile state, float offsets; one column per lane.
constexpr int ST_X = 0;                      // [7][64] iterate
constexpr int ST_G = ST_X + NJ * WAVE;       // [7][64] gradient
constexpr int ST_J = ST_G + NJ * WAVE;       // [64] cost (group-uniform)
constexpr int ST_CNT = ST_J + WAVE;          // [64] history count (int)
constexpr int ST_HEAD = ST_CNT + WAVE;       // [64] ring head (int)
constexpr int ST_ITER = ST_HEAD + WAVE;      // [64] iterations done (int)
constexpr int ST_EVC = ST_ITER + WAVE;       // [64] cost-only evaluations (int)
constexpr int ST_EVG = ST_EVC + WAVE;        // [64] cost+gradient evaluations (int)
constexpr int ST_RHO = ST_EVG + WAVE;        // [m][64] 1 / s^T y
constexpr int ST_YY = ST_RHO + DS_MAX_HISTORY * WAVE;    // [m][64] y^T y
constexpr int ST_S = ST_YY + DS_MAX_HISTORY * WAVE;      // [m][7][64]
constexpr int ST_Y = ST_S + DS_MAX_HISTORY * NJ * WAVE;  // [m][7][64]
constexpr int ST_FLOATS = ST_Y + DS_MAX_HISTORY * NJ * WAVE;
constexpr size_t ST_BYTES = ((size_t)ST_FLOATS * 4 + 255) / 256 * 256;

// Serving: one slot per admitted request.
struct SlotDev {
  int32_t active;        // 1 when the slot holds a request
  int32_t prob;          // problem-table index of the request
  int32_t tile0, ntiles; // its tiles in the tile table
};

}  // namespace dsk

// Releases the serving state of a plan (dsopt_serve.cpp).
void ds_serve_free(ds_plan* plan);
// True while a queued or admitted serving request uses the scene.
bool ds_serve_uses_scene(const ds_plan* plan, int32_t scene_id);

// Launch wrappers (dsopt_kernels.hip).  `ext` selects the kernel variants
// with the optional terms (self-collision, swept sub-samples) compiled in.
namespace dsk {
inline bool params_ext(const ParamsDev& P) { return P.ws != 0.f || P.nsub > 0; }
hipError_t launch_esdf_pack(const float* vals, int nx, int ny, int nz, float4* rec,
                            hipStream_t s);
// The coarse table of a scene into out (COARSE_BYTES, cleared here).
hipError_t launch_coarse(const float* vals, int nx, int ny, int nz, int shift, int cdx, int cdy,
                         int cdz, float cq, uint8_t* out, hipStream_t s);
// counter: N_XCD ints when xcd_ranges (N_XCD + 1 ints: the per-XCD queues'
// bounds in the tile table) is given, else one.
// tile_list (optional): the queue order, a permutation of 0..n_tiles-1.
hipError_t launch_optimize(const RobotDev* rb, const ParamsDev* pp, const ProbDev* probs,
                           const TileDev* tiles, int n_tiles, int* counter, int grid_blocks,
                           int max_iters, int waves, bool ext, hipStream_t s,
                           const int* xcd_ranges = nullptr, const int* tile_list = nullptr);
// Order each per-XCD queue (xcd_ranges: N_XCD + 1 ints) longest expected
// tile first -- larger lane groups first, then higher cost at the seed (the
// tile state's J after the initial evaluation) -- into list (a permutation
// of the tile table inside each queue's range), and empty the queue
// counters.
hipError_t launch_queue_order(const TileDev* tiles, const int* xcd_ranges, int* list,
                              int* counter, hipStream_t s);
hipError_t launch_best(const ProbDev* probs, int n_probs, const int* list, hipStream_t s);
hipError_t launch_cost(const RobotDev* rb, const ParamsDev* pp, const ProbDev* prob,
                       const float* X, int S, int T, const float* dJ, float* J_out, float* dX,
                       int with_grad, bool ext, int cu_count, hipStream_t s);
hipError_t launch_guide(const RobotDev* rb, const ParamsDev* pp, const ProbDev* prob, float* X,
                        int S, int T, float alpha, int n_steps, float* J_out, bool ext,
                        int cu_count, hipStream_t s);
hipError_t launch_spheres(const RobotDev* rb, const float* X, int S, int T, float* out,
                          hipStream_t s);
hipError_t launch_zero_i32(int* p, int n, hipStream_t s);
// Fresh tiles (iteration counters, seed results) and the tile queue
// counters (N_XCD ints; n_tiles >= 1).
hipError_t launch_tile_reset(const TileDev* tiles, const ProbDev* probs, int n_tiles, int* counter,
                             hipStream_t s);
hipError_t launch_esdf_from_occupancy(const uint8_t* occ, int nx, int ny, int nz, float voxel,
                                      float* w0, float* w1, float* w2, float* w3, float* out,
                                      hipStream_t s);
hipError_t launch_serve_step(const RobotDev* rb, const ParamsDev* pp, const ProbDev* probs,
                             const TileDev* tiles, const int* tile_list, int* counter,
                             int max_tiles, int grid_blocks, const int* max_iters_dev, int waves,
                             bool ext, hipStream_t s);
int team_block(int waves);
int optimize_blocks_per_cu(int waves, bool ext);
// Resolve the allocation-free call's device array on the current device
// (dsopt_noalloc.hip); DS_OK or a DS_ERR_* code.
int noalloc_init(int device);
}  // namespace dsk
