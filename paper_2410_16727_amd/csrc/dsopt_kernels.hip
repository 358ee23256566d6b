// gfx950 kernels of the seeded trajectory optimiser.
//
// Mapping: one wavefront (or a team of W wavefronts) owns one tile = one
// seed of one problem; lane t of each lane group holds waypoint t (group
// size G = 64, 32 or 16 >= T) and the 64 / G groups of a wavefront are
// copies of the seed that split its spheres.  Per lane the kernel runs the whole per-waypoint chain of the
// objective (App. A.6): forward kinematics (sincos + 3x4 compositions with
// the robot table read through the scalar cache), sphere centres, an ESDF
// gather of one 32-byte corner record per sphere (two 16-byte buffer
// loads), the smooth hinge, and -- for the gradient -- the joint-axis
// adjoint: sphere forces f = w_c phi'(D) grad d accumulated per link into
// a wrench and projected on every preceding joint twist, recomputing the
// kinematics instead of storing transforms.  Finite differences of the
// trajectory (smoothness) move between lanes with cross-lane shuffles;
// per-seed sums (cost, L-BFGS dot products, Armijo tests) are butterfly
// reductions inside the lane group, so every lane ends with bitwise the same
// value and the reduction order depends only on G.  Nothing here is a dense
// contraction: no MFMA.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <type_traits>

#include "dsopt_internal.h"

namespace dsk {
namespace {

constexpr unsigned RSRC_DWORD3 = 0x00020000u;   // raw buffer, gfx9 family

// Pointers read from tables are generic to the compiler; these casts state
// that they address global memory, so accesses use global (not flat)
// instructions.
#define DS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ DS_GLOBAL T* glb(T* p) {
  return (DS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const DS_GLOBAL T* glb(const T* p) {
  return (const DS_GLOBAL T*)p;
}
// ... and that a pointer into a __shared__ array addresses LDS (ds_read /
// ds_write rather than flat accesses).
#define DS_LDS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ DS_LDS T* lds(T* p) {
  return (DS_LDS T*)p;
}
#ifndef DSOPT_CH
#define DSOPT_CH 4
#endif
constexpr int CH = DSOPT_CH;                     // sphere gathers in flight per lane
// s_waitcnt operand: vector memory count 0, the export and LDS/scalar
// counts at their maxima (not waited on)
constexpr int WAIT_VMEM_ALL = 0x0F70;

// Butterfly reductions over a lane group of G = 16, 32 or 64 lanes.  The
// first four stages pair lanes inside a 16-lane row with DPP (quad
// permutations 1<->0 / 2<->0, then the half-row and row mirrors), the
// remaining ones exchange rows (lane ^ 16) and halves (lane ^ 32) with the
// permlane swaps -- VALU instructions, no LDS round trip.  Every pairing is
// an involution, so both partners add the same two numbers and every lane of
// the group ends with bitwise the same result.
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

constexpr int DPP_WAVE_SHL1 = 0x130;   // lane i reads lane i + 1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i reads lane i - 1

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// The value of lane i + 1 / lane i - 1 (one DPP move; the lane past either
// end of the wavefront reads 0).  Callers only use lanes whose neighbour is
// in the same lane group.
__device__ __forceinline__ float from_next(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), DPP_WAVE_SHL1, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_prev(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), DPP_WAVE_SHR1, 0xF, 0xF, true));
}

struct OpSum { __device__ static float f(float a, float b) { return a + b; } };
struct OpMax { __device__ static float f(float a, float b) { return fmaxf(a, b); } };
struct OpMin { __device__ static float f(float a, float b) { return fminf(a, b); } };

// v combined with lane ^ 16's v (v_permlane16_swap with v as both operands
// exchanges the odd rows of the first with the even rows of the second: in
// every lane one result is its own value and the other its partner's) and
// with lane ^ 32's (v_permlane32_swap: the upper half of the first operand
// with the lower half of the second).  The operations are commutative, so
// combining the two results needs no per-lane select.
template <class Op>
__device__ __forceinline__ float xor16_reduce(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), true,
                                                  false);
  return Op::f(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
template <class Op>
__device__ __forceinline__ float xor32_reduce(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), true,
                                                  false);
  return Op::f(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
template <class Op>
__device__ __forceinline__ float xor_reduce(float v, int off) {
  return off == 16 ? xor16_reduce<Op>(v) : xor32_reduce<Op>(v);
}

template <class Op>
__device__ __forceinline__ float grp_reduce(float v, int G) {
  v = Op::f(v, dpp<DPP_QUAD_XOR1>(v));
  v = Op::f(v, dpp<DPP_QUAD_XOR2>(v));
  v = Op::f(v, dpp<DPP_HALF_MIRROR>(v));
  v = Op::f(v, dpp<DPP_MIRROR>(v));
  if (G > 16) v = xor16_reduce<Op>(v);
  if (G > 32) v = xor32_reduce<Op>(v);
  return v;
}

__device__ __forceinline__ float grp_sum(float v, int G) { return grp_reduce<OpSum>(v, G); }
__device__ __forceinline__ float grp_max(float v, int G) { return grp_reduce<OpMax>(v, G); }
__device__ __forceinline__ float grp_min(float v, int G) { return grp_reduce<OpMin>(v, G); }
__device__ __forceinline__ float dot7(const float* a, const float* b) {
  float s = a[0] * b[0];
#pragma unroll
  for (int j = 1; j < NJ; ++j) s += a[j] * b[j];
  return s;
}

struct Goal {
  float pd[3];
  float Rd[9];
};

// Unit goal quaternion (w, x, y, z) -> rotation matrix (uniform per tile).
__device__ __forceinline__ Goal make_goal(const ProbDev& pb) {
  Goal g;
  float w = pb.quat[0], x = pb.quat[1], y = pb.quat[2], z = pb.quat[3];
  float n = sqrtf(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  g.Rd[0] = 1.f - 2.f * (y * y + z * z); g.Rd[1] = 2.f * (x * y - w * z); g.Rd[2] = 2.f * (x * z + w * y);
  g.Rd[3] = 2.f * (x * y + w * z); g.Rd[4] = 1.f - 2.f * (x * x + z * z); g.Rd[5] = 2.f * (y * z - w * x);
  g.Rd[6] = 2.f * (x * z - w * y); g.Rd[7] = 2.f * (y * z + w * x); g.Rd[8] = 1.f - 2.f * (x * x + y * y);
  g.pd[0] = pb.pd[0]; g.pd[1] = pb.pd[1]; g.pd[2] = pb.pd[2];
  return g;
}

struct Sampler {
  __amdgpu_buffer_rsrc_t rsrc;
  float ox, oy, oz, inv_h, h, nxm1, nym1, nzm1;
  float fxm2, fym2, fzm2;          // last cell index per axis, as floats
  int nxm2, nym2, nzm2, cx, cy;    // cells along x and y
  const DS_LDS uint8_t* cm;        // the scene's coarse table (4-bit levels), staged in LDS
  float cq;                        // distance of one level
  int cshift, cdx, cdy;
};

__device__ __forceinline__ Sampler make_sampler(const SceneDev& sc) {
  Sampler s;
  s.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)sc.rec, (short)0, (int)sc.bytes, RSRC_DWORD3);
  s.ox = sc.ox; s.oy = sc.oy; s.oz = sc.oz; s.inv_h = sc.inv_h; s.h = 1.f / sc.inv_h;
  s.nxm1 = (float)(sc.nx - 1); s.nym1 = (float)(sc.ny - 1); s.nzm1 = (float)(sc.nz - 1);
  s.nxm2 = sc.nx - 2; s.nym2 = sc.ny - 2; s.nzm2 = sc.nz - 2;
  s.fxm2 = (float)s.nxm2; s.fym2 = (float)s.nym2; s.fzm2 = (float)s.nzm2;
  s.cx = sc.nx - 1;
  s.cy = sc.ny - 1;
  s.cm = nullptr;
  s.cq = sc.cq;
  s.cshift = sc.cshift;
  s.cdx = sc.cdx;
  s.cdy = sc.cdy;
  return s;
}

// Copy the scene's coarse table into LDS (threads tid = 0..nth-1 of the
// group that shares it; the caller synchronises them afterwards) in
// 16-byte pieces, STAGE_UNROLL loads in flight per thread before their LDS
// stores (one load at a time made every piece a memory round trip).  The
// table's allocation and both ends are 16-byte aligned.
constexpr int STAGE_UNROLL = 4;
__device__ __forceinline__ void stage_coarse(const SceneDev& sc, DS_LDS uint8_t* dst, int tid,
                                             int nth) {
  const int n = (sc.cdx * sc.cdy * sc.cdz + 31) / 32;   // 32 levels per piece
  const DS_GLOBAL uint32_t* src = glb(reinterpret_cast<const uint32_t*>(sc.coarse));
  DS_LDS uint32_t* d = (DS_LDS uint32_t*)dst;
  for (int i0 = tid; i0 < n; i0 += STAGE_UNROLL * nth) {
    uint32_t v[STAGE_UNROLL][4];
#pragma unroll
    for (int u = 0; u < STAGE_UNROLL; ++u) {
      const int i = i0 + u * nth;
      if (i < n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[u][q] = src[4 * i + q];
      }
    }
#pragma unroll
    for (int u = 0; u < STAGE_UNROLL; ++u) {
      const int i = i0 + u * nth;
      if (i < n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) d[4 * i + q] = v[u][q];
      }
    }
  }
}

// A coarse-table entry as a distance: level * cq, at most the block's
// minimum node distance.
__device__ __forceinline__ float coarse_at(const Sampler& S, int idx) {
  const unsigned b = S.cm[idx >> 1];
  return (float)((b >> ((idx & 1) << 2)) & 15u) * S.cq;
}

// A sample's place in the grid.  u = (c - origin) / voxel is the sphere
// centre c in grid units; the sample's cell is trunc(clamp(u, 0, n-2)) per
// axis (the cell whose corners bracket the clamped point), its fractional
// position clamp(u, 0, n-1) - cell, and the gradient is zero along axes
// where u was clamped.
//
// A link frame (R, p) maps a sphere offset o to c = p + R o.  For a link
// whose spheres all lie on its z axis (o = (0, 0, oz)) the link's part is
// formed once -- u = u0 + oz az with u0 = (p - origin) / voxel and
// az = R e_z / voxel -- so a sphere costs one FMA per axis.
struct LinkGrid {
  float u0[3], az[3];
};

__device__ __forceinline__ LinkGrid link_grid(const Sampler& S, const float* R, const float* p) {
  LinkGrid g;
  g.u0[0] = (p[0] - S.ox) * S.inv_h;
  g.u0[1] = (p[1] - S.oy) * S.inv_h;
  g.u0[2] = (p[2] - S.oz) * S.inv_h;
  g.az[0] = R[2] * S.inv_h;
  g.az[1] = R[5] * S.inv_h;
  g.az[2] = R[8] * S.inv_h;
  return g;
}

// Grid position of the sphere with offset/radius sp on the link (R, p);
// `axis` (wave-uniform) says the link's spheres sit on its z axis.
__device__ __forceinline__ void grid_pos(const Sampler& S, const LinkGrid& g, bool axis,
                                         const float* R, const float* p, float4 sp, float* u) {
  if (axis) {
#pragma unroll
    for (int r = 0; r < 3; ++r) u[r] = fmaf(sp.z, g.az[r], g.u0[r]);
  } else {
    const float cx = R[0] * sp.x + R[1] * sp.y + R[2] * sp.z + p[0];
    const float cy = R[3] * sp.x + R[4] * sp.y + R[5] * sp.z + p[1];
    const float cz = R[6] * sp.x + R[7] * sp.y + R[8] * sp.z + p[2];
    u[0] = (cx - S.ox) * S.inv_h;
    u[1] = (cy - S.oy) * S.inv_h;
    u[2] = (cz - S.oz) * S.inv_h;
  }
}

// The sample's cell: trunc(clamp(u, 0, n-2)) per axis (for u >= 0,
// min(trunc(min(u, n-1)), n-2) == trunc(min(u, n-2)): one v_med3 and one
// conversion per axis).
__device__ __forceinline__ void cell_of(const Sampler& S, const float* u, int* i) {
  i[0] = (int)__builtin_amdgcn_fmed3f(u[0], 0.f, S.fxm2);
  i[1] = (int)__builtin_amdgcn_fmed3f(u[1], 0.f, S.fym2);
  i[2] = (int)__builtin_amdgcn_fmed3f(u[2], 0.f, S.fzm2);
}

// The cell's block in the coarse table and its record's byte offset.
// Every product fits 24 bits: the upload keeps (ny-1)(nz-1) below 2^24,
// and the coarse table has at most COARSE_MAX blocks (stating the bounds
// keeps both products 24-bit multiply-adds).
__device__ __forceinline__ int block_index(const Sampler& S, const int* i) {
  const unsigned crow =
      __umul24((unsigned)S.cdy, (unsigned)(i[2] >> S.cshift)) + (unsigned)(i[1] >> S.cshift);
  __builtin_assume(crow < (1u << 24));
  return (int)(__umul24((unsigned)S.cdx, crow) + (unsigned)(i[0] >> S.cshift));
}

__device__ __forceinline__ int record_offset(const Sampler& S, const int* i) {
  const unsigned row = __umul24((unsigned)S.cy, (unsigned)i[2]) + (unsigned)i[1];
  __builtin_assume(row < (1u << 24));
  return (int)((__umul24((unsigned)S.cx, row) + (unsigned)i[0]) << 5);
}

// Trilinear blend of a cell record (a: z0 corners, b: z1 corners) at the
// fractional position (fx, fy, fz): the value, and the differences its
// spatial gradient is formed from.
struct Blend {
  float d;                          // interpolated distance
  float dx00, dx10, dx01, dx11;     // x differences of the four x edges
  float dy0, dy1, dz;               // y differences at z0/z1, z difference
};

__device__ __forceinline__ Blend blend_value(float fx, float fy, float fz, float4 a, float4 b) {
  Blend r;
  r.dx00 = a.y - a.x; r.dx10 = a.w - a.z; r.dx01 = b.y - b.x; r.dx11 = b.w - b.z;
  float c00 = a.x + fx * r.dx00;
  float c10 = a.z + fx * r.dx10;
  float c01 = b.x + fx * r.dx01;
  float c11 = b.z + fx * r.dx11;
  r.dy0 = c10 - c00;
  r.dy1 = c11 - c01;
  float c0 = c00 + fy * r.dy0;
  float c1 = c01 + fy * r.dy1;
  r.dz = c1 - c0;
  r.d = c0 + fz * r.dz;
  return r;
}

// Its spatial gradient in grid units (times 1/voxel by the caller).
__device__ __forceinline__ void blend_grad(float fy, float fz, const Blend& r, float& gx,
                                           float& gy, float& gz) {
  float e0 = r.dx00 + fy * (r.dx10 - r.dx00);
  float e1 = r.dx01 + fy * (r.dx11 - r.dx01);
  gx = e0 + fz * (e1 - e0);
  gy = r.dy0 + fz * (r.dy1 - r.dy0);
  gz = r.dz;
}

__device__ __forceinline__ float4 load_rec(const Sampler& S, int off) {
  auto v = __builtin_amdgcn_raw_buffer_load_b128(S.rsrc, off, 0, 0);
  return *reinterpret_cast<float4*>(&v);
}

enum { EV_COST = 0, EV_GRAD = 1, EV_RESULT = 2 };

// The robot's sphere table (offset, radius; sorted by link) staged in LDS
// by every kernel that evaluates the objective: the sphere a lane takes
// depends on its copy index, so the reads are per-lane and would otherwise
// be vector memory round trips ahead of every record gather.
__shared__ float4 s_sph[DS_MAX_SPHERES];

// Fill s_sph; every thread of the workgroup must call it.
__device__ __forceinline__ void stage_spheres(const RobotDev* __restrict__ rb) {
  for (int i = threadIdx.x; i < rb->ns; i += blockDim.x) s_sph[i] = rb->sph[i];
  __syncthreads();
}

// Joint twists (axis z_i, origin o_i) of the swept joints, kept for the
// wrench projections of the adjoint.
struct Twists {
  float z[NJ][3], o[NJ][3];
  __device__ __forceinline__ void put(int i, const float* R, const float* p) {
    z[i][0] = R[2]; z[i][1] = R[5]; z[i][2] = R[8];
    o[i][0] = p[0]; o[i][1] = p[1]; o[i][2] = p[2];
  }
  __device__ __forceinline__ void get(int i, float* zi, float* oi) const {
    zi[0] = z[i][0]; zi[1] = z[i][1]; zi[2] = z[i][2];
    oi[0] = o[i][0]; oi[1] = o[i][1]; oi[2] = o[i][2];
  }
};

struct EvalOut {
  float cost;        // this lane's share of the seed objective (0 when inactive)
  float g[NJ];       // gradient row (EV_GRAD; zero at t = 0 and inactive lanes)
  float clr;         // min (distance - radius) at this waypoint (EV_RESULT)
  float perr, rerr;  // goal errors at this lane's waypoint (EV_RESULT)
  int ng;            // cell records this lane gathered
};

// Smoothness on the lane group: v_t = q_{t+1} - q_t (t <= T-2),
// a_t = v_t - v_{t-1} (t < T), j_t = a_{t+1} - a_t (t < T) plus
// j_{-1} = a_0 at t = 0 -- the first/second/third differences of the
// sequence padded with two copies of q_0 and of q_{T-1}.  The gradient
// applies the transposed stencils with the same lane shifts (DPP moves; the
// masks keep every read inside the lane group).
template <bool GRAD>
__device__ __forceinline__ float smoothness(const ParamsDev& P, const float* q, int t, int T,
                                            float* g) {
  float c = 0.f;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    float qn = from_next(q[j]);
    float v = (t <= T - 2) ? qn - q[j] : 0.f;
    float vp = from_prev(v);
    float a = (t < T) ? v - (t >= 1 ? vp : 0.f) : 0.f;
    float an = from_next(a);
    float jk = (t < T) ? ((t + 1 < T ? an : 0.f) - a) : 0.f;
    float jm = (t == 0) ? a : 0.f;   // j_{-1}
    c += P.lv * (v * v) + P.la * (a * a) + P.lj * (jk * jk) + P.lj * (jm * jm);
    if (GRAD) {
      float jb = 2.f * P.lj * jk;
      float jbp = from_prev(jb);
      float ab = (t < T) ? 2.f * P.la * a + ((t == 0) ? 2.f * P.lj * jm : jbp) - jb : 0.f;
      float abn = from_next(ab);
      float vb = (t <= T - 2) ? 2.f * P.lv * v + ab - abn : 0.f;
      float vbp = from_prev(vb);
      g[j] += ((t >= 1) ? vbp : 0.f) - vb;
    }
  }
  return c;
}

// A team of W wavefronts (one workgroup) optimises one seed: every
// wavefront holds the whole trajectory (one waypoint per lane group) and
// takes every (W*L)-th sphere of each link; the partial sums meet in
// double-buffered LDS with one barrier per evaluation.  W = 1: independent
// wavefronts, no barrier.
constexpr int MAX_TEAM = 8;
constexpr int PART = NJ + 2;   // partial sums per lane: hinge sum, gradient row, clearance

struct Team {
  int W, w;       // team size, this wavefront's index
  float* lds;     // [2][W][PART][64]
  int buf;
  __device__ __forceinline__ void sync() const {
    if (W > 1) __syncthreads();
  }
};

// Hinge cost of one sphere sample (grid position u, cell ci, cell record
// ra/rz, radius r) and, with GRAD, its force accumulated into the link
// wrench (F, M about the world origin).  Returns whether the force terms
// ran (some lane of the wavefront inside the hinge band).
template <int MODE>
__device__ __forceinline__ bool sphere_term(const ParamsDev& P, const Sampler& S, const float* u,
                                            const int* ci, float4 ra, float4 rz, float r,
                                            float& phisum, float& clr, float* FM) {
  constexpr bool GRAD = (MODE == EV_GRAD);
  const float cx = __builtin_amdgcn_fmed3f(u[0], 0.f, S.nxm1);
  const float cy = __builtin_amdgcn_fmed3f(u[1], 0.f, S.nym1);
  const float cz = __builtin_amdgcn_fmed3f(u[2], 0.f, S.nzm1);
  const float fy = cy - (float)ci[1], fz = cz - (float)ci[2];
  const Blend bl = blend_value(cx - (float)ci[0], fy, fz, ra, rz);
  float D = bl.d - r;
  float De = D - P.eps;
  float phi = (D < P.eps) ? De * De * P.half_inv_eps : 0.f;
  phi = (D < 0.f) ? 0.5f * P.eps - D : phi;
  phisum += phi;
  if (MODE == EV_RESULT) clr = fminf(clr, D);
  // the force is zero outside the hinge band: when no lane of the
  // wavefront has a sample inside it, the gradient and the wrench terms
  // (which would add zeros) are skipped
  const bool band = GRAD && __any(D < P.eps);
  if (band) {
    float gx, gy, gz;
    blend_grad(fy, fz, bl, gx, gy, gz);
    // world units; zero along axes where the point was clamped
    gx *= (cx == u[0]) ? S.inv_h : 0.f;
    gy *= (cy == u[1]) ? S.inv_h : 0.f;
    gz *= (cz == u[2]) ? S.inv_h : 0.f;
    float dphi = (D < P.eps) ? De * P.inv_eps : 0.f;
    dphi = (D < 0.f) ? -1.f : dphi;
    float w = P.wc * dphi;
    float fx = w * gx, fyy = w * gy, fzz = w * gz;
    // the sphere centre (the moment arm) back from its grid position
    const float px = fmaf(u[0], S.h, S.ox);
    const float py = fmaf(u[1], S.h, S.oy);
    const float pz = fmaf(u[2], S.h, S.oz);
    FM[0] += fx; FM[1] += fyy; FM[2] += fzz;
    FM[3] += py * fzz - pz * fyy;
    FM[4] += pz * fx - px * fzz;
    FM[5] += px * fyy - py * fx;
  }
  return band;
}

// Project a link wrench on the joints 0..l: g_i += z_i . (M - o_i x F).
__device__ __forceinline__ void project(const Twists& tw, int l, const float* FM, float* g) {
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    if (i > l) break;
    float zi[3], oi[3];
    tw.get(i, zi, oi);
    float tx = FM[3] - (oi[1] * FM[2] - oi[2] * FM[1]);
    float ty = FM[4] - (oi[2] * FM[0] - oi[0] * FM[2]);
    float tz = FM[5] - (oi[0] * FM[1] - oi[1] * FM[0]);
    g[i] += zi[0] * tx + zi[1] * ty + zi[2] * tz;
  }
}

// Self-collision share of this lane (App. A.6 C_self): every pair of spheres
// on links at least two apart, hinge on D = |c_a - c_b| - r_a - r_b; the
// pairs of each link pair are split over the W*L copies.  The sweep keeps
// the seven link frames; forces go into per-link wrenches that are projected
// on the joint axes at the end.
template <int MODE>
__device__ __attribute__((noinline)) void self_collision(const RobotDev* __restrict__ rb,
                                                         const ParamsDev& P, const float* q,
                                                         int cp, int LW, float& selfsum,
                                                         float& clr, float* g) {
  constexpr bool GRAD = (MODE == EV_GRAD);
  float Rf[NJ][9], pf[NJ][3];
  float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int l = 0; l < NJ; ++l) {
    const float* F = rb->F[l];
    float A[9], pa[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        A[3 * r + c] = R[3 * r] * F[c] + R[3 * r + 1] * F[4 + c] + R[3 * r + 2] * F[8 + c];
      pa[r] = R[3 * r] * F[3] + R[3 * r + 1] * F[7] + R[3 * r + 2] * F[11] + p[r];
    }
    float sn, cs;
    sincosf(q[l], &sn, &cs);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float a0 = A[3 * r], a1 = A[3 * r + 1];
      R[3 * r] = cs * a0 + sn * a1;
      R[3 * r + 1] = cs * a1 - sn * a0;
      R[3 * r + 2] = A[3 * r + 2];
      p[r] = pa[r];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) Rf[l][k] = R[k];
    pf[l][0] = p[0]; pf[l][1] = p[1]; pf[l][2] = p[2];
  }
  float FM[NJ][6];
#pragma unroll
  for (int l = 0; l < NJ; ++l)
#pragma unroll
    for (int k = 0; k < 6; ++k) FM[l][k] = 0.f;
#pragma unroll
  for (int la = 0; la < NJ; ++la) {
#pragma unroll
    for (int lb = la + 2; lb < NJ; ++lb) {
      const int a0 = rb->link_begin[la], na = rb->link_begin[la + 1] - a0;
      const int b0 = rb->link_begin[lb], nb = rb->link_begin[lb + 1] - b0;
      for (int k = cp; k < na * nb; k += LW) {
        const int ia = k / nb, ib = k - ia * nb;
        const float4 sa = s_sph[a0 + ia], sb = s_sph[b0 + ib];
        float ca[3], cb[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          ca[r] = Rf[la][3 * r] * sa.x + Rf[la][3 * r + 1] * sa.y + Rf[la][3 * r + 2] * sa.z + pf[la][r];
          cb[r] = Rf[lb][3 * r] * sb.x + Rf[lb][3 * r + 1] * sb.y + Rf[lb][3 * r + 2] * sb.z + pf[lb][r];
        }
        float dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
        float dist = sqrtf(dx * dx + dy * dy + dz * dz);
        float D = dist - sa.w - sb.w;
        float De = D - P.eps;
        float phi = (D < P.eps) ? De * De * P.half_inv_eps : 0.f;
        phi = (D < 0.f) ? 0.5f * P.eps - D : phi;
        selfsum += phi;
        if (MODE == EV_RESULT) clr = fminf(clr, D);
        if (GRAD) {
          float dphi = (D < P.eps) ? De * P.inv_eps : 0.f;
          dphi = (D < 0.f) ? -1.f : dphi;
          float w = (dist > 0.f) ? P.ws * dphi / dist : 0.f;
          float fx = w * dx, fy = w * dy, fz = w * dz;
          FM[la][0] += fx; FM[la][1] += fy; FM[la][2] += fz;
          FM[la][3] += ca[1] * fz - ca[2] * fy;
          FM[la][4] += ca[2] * fx - ca[0] * fz;
          FM[la][5] += ca[0] * fy - ca[1] * fx;
          FM[lb][0] -= fx; FM[lb][1] -= fy; FM[lb][2] -= fz;
          FM[lb][3] -= cb[1] * fz - cb[2] * fy;
          FM[lb][4] -= cb[2] * fx - cb[0] * fz;
          FM[lb][5] -= cb[0] * fy - cb[1] * fx;
        }
      }
    }
  }
  if (GRAD) {
#pragma unroll
    for (int l = 0; l < NJ; ++l) {
#pragma unroll
      for (int i = 0; i <= l; ++i) {
        const float zi[3] = {Rf[i][2], Rf[i][5], Rf[i][8]};
        const float* oi = pf[i];
        float tx = FM[l][3] - (oi[1] * FM[l][2] - oi[2] * FM[l][1]);
        float ty = FM[l][4] - (oi[2] * FM[l][0] - oi[0] * FM[l][2]);
        float tz = FM[l][5] - (oi[0] * FM[l][1] - oi[1] * FM[l][0]);
        g[i] += zi[0] * tx + zi[1] * ty + zi[2] * tz;
      }
    }
  }
}

// The sweep over the chain for one configuration q: FK, this lane's share
// of the sphere samples (hinge sum into phisum, min clearance into clr) and,
// with GRAD, the link wrenches projected on the joint axes into g.  On
// return R, p hold the frame of link 7 and tw the joint twists.
// PIPE (every lane holds at most one sphere of each link, W*L >= spheres
// per link): the sweep issues each link's record load as soon as its frame
// exists and consumes the samples afterwards, so one memory round trip
// covers the whole configuration.  Otherwise each link is processed in
// chunks of CH gathers right after its frame.
template <int MODE, bool PIPE>
__device__ __forceinline__ void sweep(const RobotDev* __restrict__ rb, const ParamsDev& P,
                                      const Sampler& S, const float* q, int cp, int LW,
                                      Twists& tw, float* R, float* p, float& phisum, float& clr,
                                      float* g, int& ng, bool active) {
  constexpr bool GRAD = (MODE == EV_GRAD);
  // the result pass gathers every sample: the clearance is a minimum over
  // all of them
  const bool SKIP = MODE != EV_RESULT && P.skip;
  R[0] = 1.f; R[1] = 0.f; R[2] = 0.f; R[3] = 0.f; R[4] = 1.f; R[5] = 0.f;
  R[6] = 0.f; R[7] = 0.f; R[8] = 1.f;
  p[0] = p[1] = p[2] = 0.f;
  // PIPE: the lane's sample of every link (grid position, radius, coarse
  // minimum, record)
  float4 pa_[PIPE ? NJ : 1], pz_[PIPE ? NJ : 1];
  float pu_[PIPE ? NJ : 1][3], pr_[PIPE ? NJ : 1], pcm_[PIPE ? NJ : 1];
  bool pv_[PIPE ? NJ : 1];
#pragma unroll
  for (int l = 0; l < NJ; ++l) {
    const float* F = rb->F[l];
    float A[9], pa[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        A[3 * r + c] = R[3 * r] * F[c] + R[3 * r + 1] * F[4 + c] + R[3 * r + 2] * F[8 + c];
      pa[r] = R[3 * r] * F[3] + R[3 * r + 1] * F[7] + R[3 * r + 2] * F[11] + p[r];
    }
    float sn, cs;
    sincosf(q[l], &sn, &cs);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float a0 = A[3 * r], a1 = A[3 * r + 1];
      R[3 * r] = cs * a0 + sn * a1;
      R[3 * r + 1] = cs * a1 - sn * a0;
      R[3 * r + 2] = A[3 * r + 2];
      p[r] = pa[r];
    }
    if (GRAD) tw.put(l, R, p);
    const int s0 = rb->link_begin[l], s1 = rb->link_begin[l + 1];
    const bool axis = (rb->axis_links >> l) & 1;   // wave-uniform
    const LinkGrid lg = link_grid(S, R, p);
    if (PIPE) {
      // copy cp takes sphere (cp - rot) mod LW of the link, rot advancing by
      // the longest link's sphere count from link to link: when there are
      // more copies than spheres, consecutive links land on different
      // copies and the samples spread evenly over the wavefronts
      int idx = cp - (l * rb->max_per_link) % LW;
      if (idx < 0) idx += LW;
      const int sk = s0 + idx;
      pv_[l] = active && sk < s1;   // lanes past the horizon gather nothing
      if (pv_[l]) {
        const float4 sp = s_sph[sk];
        grid_pos(S, lg, axis, R, p, sp, pu_[l]);
        pr_[l] = sp.w;
        // the coarse minimum is read here and tested after the chain, so
        // no link waits for its lookup before the next frame
        if (SKIP) {
          int ci[3];
          cell_of(S, pu_[l], ci);
          pcm_[l] = coarse_at(S, block_index(S, ci));
        }
      }
      continue;
    }
    float FM[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool forced = false;   // some sample of this link added a force
    // chunks of CH spheres per lane (this lane takes every (W*L)-th sphere
    // of the link): issue every record load of the chunk, then consume them
    // in sphere order -- CH gathers in flight per lane.  A sample whose
    // coarse block holds no node nearer than radius + eps (+ margin) has a
    // zero hinge (a trilinear blend stays within its corners' range): it
    // loads nothing.
    for (int s = s0; s < s1; s += LW * CH) {
      float u[CH][3], rr[CH];
      int ci[CH][3];
      float4 ra[CH], rz[CH];
      bool use[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int sk = s + k * LW + cp;
        use[k] = active && sk < s1;
        if (use[k]) {
          const float4 sp = s_sph[sk];
          grid_pos(S, lg, axis, R, p, sp, u[k]);
          cell_of(S, u[k], ci[k]);
          rr[k] = sp.w;
          if (SKIP && coarse_at(S, block_index(S, ci[k])) >= sp.w + P.far) {
            use[k] = false;   // zero hinge, zero gradient
          } else {
            const int off = record_offset(S, ci[k]);
            ra[k] = load_rec(S, off);
            rz[k] = load_rec(S, off + 16);
            ++ng;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (use[k])
          forced |= sphere_term<MODE>(P, S, u[k], ci[k], ra[k], rz[k], rr[k], phisum, clr, FM);
      }
      // every load of the chunk has been consumed: saying so keeps the
      // next chunk's loads in flight together.  (The loads and their uses
      // sit in separate wavefront-uniform branches, so without it the
      // compiler cannot tell which of them are outstanding at the loop's
      // back edge and drains them all before each sphere's loads.)
      __builtin_amdgcn_s_waitcnt(WAIT_VMEM_ALL);
    }
    // a link with no force in this wavefront has a zero wrench everywhere:
    // its projection would add zeros
    if (GRAD && __any(forced)) project(tw, l, FM, g);
  }
  if (PIPE) {
    // issue the record loads of the samples that can reach the hinge
#pragma unroll
    for (int l = 0; l < NJ; ++l) {
      if (pv_[l]) {
        if (SKIP && pcm_[l] >= pr_[l] + P.far) {
          pv_[l] = false;   // zero hinge, zero gradient: nothing to add
        } else {
          int ci[3];
          cell_of(S, pu_[l], ci);
          const int off = record_offset(S, ci);
          pa_[l] = load_rec(S, off);
          pz_[l] = load_rec(S, off + 16);
          ++ng;
        }
      }
    }
#pragma unroll
    for (int l = 0; l < NJ; ++l) {
      float FM[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bool forced = false;
      if (pv_[l]) {
        int ci[3];
        cell_of(S, pu_[l], ci);
        forced = sphere_term<MODE>(P, S, pu_[l], ci, pa_[l], pz_[l], pr_[l], phisum, clr, FM);
      }
      // a link with no force in this wavefront has a zero wrench
      // everywhere: its projection would add zeros
      if (GRAD && __any(forced)) project(tw, l, FM, g);
    }
  }
}

// One evaluation of the objective at this lane's configuration q (its
// waypoint) and, with swept sub-samples, at the configurations interpolated
// towards the next waypoint.
template <int MODE, bool PIPE, bool EXT>
__device__ __forceinline__ EvalOut evaluate(const RobotDev* __restrict__ rb,
                                            const ParamsDev& P, const Sampler& S, const Goal& goal,
                                            const float* q, int t, int T, int G, bool active,
                                            Team& tm) {
  constexpr bool GRAD = (MODE == EV_GRAD);
  // the L = 64/G lanes holding the same waypoint in each of the W
  // wavefronts split its spheres: copy index and stride
  const int L = WAVE / G;
  const int lane = threadIdx.x & (WAVE - 1);
  const int cp = tm.w * L + lane / G;
  const int LW = tm.W * L;
  EvalOut o;
  o.ng = 0;
  o.perr = o.rerr = 0.f;
#pragma unroll
  for (int j = 0; j < NJ; ++j) o.g[j] = 0.f;
  float phisum = 0.f, clr = FLT_MAX;
  if (EXT && P.nsub > 0) {
    // swept collision: q + tau (q_next - q), tau = i / (nsub + 1); the
    // gradient splits (1 - tau) here and tau onto the next waypoint
    float qn[NJ], gsh[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      qn[j] = __shfl_down(q[j], 1);
      gsh[j] = 0.f;
    }
    const bool seg = active && t <= T - 2;
    for (int i = 1; i <= P.nsub; ++i) {
      const float tau = (float)i / (float)(P.nsub + 1);
      float qi[NJ], gi[NJ], Rs[9], ps[3];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        qi[j] = q[j] + tau * (qn[j] - q[j]);
        gi[j] = 0.f;
      }
      Twists tws;
      float ph = 0.f, cl = FLT_MAX;
      sweep<MODE, PIPE>(rb, P, S, qi, cp, LW, tws, Rs, ps, ph, cl, gi, o.ng, seg);
      if (seg) {
        phisum += ph;
        clr = fminf(clr, cl);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          o.g[j] += (1.f - tau) * gi[j];
          gsh[j] += tau * gi[j];
        }
      }
    }
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        float up = __shfl_up(gsh[j], 1);
        o.g[j] += (t >= 1) ? up : 0.f;
      }
    }
  }
  float R[9], p[3];
  Twists tw;
  sweep<MODE, PIPE>(rb, P, S, q, cp, LW, tw, R, p, phisum, clr, o.g, o.ng, active);
  // collision cost share: world hinge sum, plus the self-collision pairs
  // when that term is on
  float coll = P.wc * phisum;
  if (EXT && P.ws != 0.f) {
    float selfsum = 0.f;
    self_collision<MODE>(rb, P, q, cp, LW, selfsum, clr, o.g);
    coll += P.ws * selfsum;
  }
  // goal pose, joint limits and smoothness: the same for every copy of the
  // waypoint, so one wavefront of the team computes each and only its first
  // copy adds them to its share before the sums below -- the goal on the
  // second wavefront, the limits on the third and the smoothness on the
  // fourth (off the first one's path; smaller teams fold them onto fewer
  // wavefronts), except in the result pass, whose goal errors the first
  // one writes
  const int xg = (MODE == EV_RESULT || tm.W == 1) ? 0 : 1;
  const int xl = (MODE == EV_RESULT || tm.W < 3) ? xg : 2;
  const int xs = (MODE == EV_RESULT || tm.W < 4) ? xl : 3;
  if (tm.w == xg || tm.w == xl || tm.w == xs) {
    const bool first = lane < G;
    const bool last = (t == T - 1);
    float ge[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) ge[j] = 0.f;
    float extra_g = 0.f, extra_l = 0.f;
    if (tm.w == xg) {
    // end effector and goal pose
    const float* E = rb->Fee;
    float Re[9], pe[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        Re[3 * r + c] = R[3 * r] * E[c] + R[3 * r + 1] * E[4 + c] + R[3 * r + 2] * E[8 + c];
      pe[r] = R[3 * r] * E[3] + R[3 * r + 1] * E[7] + R[3 * r + 2] * E[11] + p[r];
    }
    float ex = pe[0] - goal.pd[0], ey = pe[1] - goal.pd[1], ez = pe[2] - goal.pd[2];
    float tr = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) tr += goal.Rd[k] * Re[k];
    const float goal_cost = P.wp * (ex * ex + ey * ey + ez * ez) + P.wr * (3.f - tr) * 0.25f;
    extra_g = last ? goal_cost : 0.f;
    if (GRAD && last) {
      // force 2 w_p e at p_ee and torque -(w_r/4) w, w = vee(M - M^T), M = R_ee R_d^T
      float M[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          M[3 * a + b] = Re[3 * a] * goal.Rd[3 * b] + Re[3 * a + 1] * goal.Rd[3 * b + 1] +
                         Re[3 * a + 2] * goal.Rd[3 * b + 2];
      float wx = M[5] - M[7], wy = M[6] - M[2], wz = M[1] - M[3];
      float k2 = 2.f * P.wp, k4 = -0.25f * P.wr;
      float fx = k2 * ex, fy = k2 * ey, fz = k2 * ez;
#pragma unroll
      for (int i = 0; i < NJ; ++i) {
        float zi[3], oi[3];
        tw.get(i, zi, oi);
        float rx = pe[0] - oi[0], ry = pe[1] - oi[1], rz = pe[2] - oi[2];
        float tx = ry * fz - rz * fy + k4 * wx;
        float ty = rz * fx - rx * fz + k4 * wy;
        float tz = rx * fy - ry * fx + k4 * wz;
        ge[i] += zi[0] * tx + zi[1] * ty + zi[2] * tz;
      }
    }
    if (MODE == EV_RESULT) {
      o.perr = sqrtf(ex * ex + ey * ey + ez * ez);
      // angle of R_d^T R_ee: cos = (tr - 1) / 2, sin = |vee(R_ee R_d^T)| / 2
      float M5, M7, M6, M2, M1, M3;
      M5 = Re[3] * goal.Rd[6] + Re[4] * goal.Rd[7] + Re[5] * goal.Rd[8];
      M7 = Re[6] * goal.Rd[3] + Re[7] * goal.Rd[4] + Re[8] * goal.Rd[5];
      M6 = Re[6] * goal.Rd[0] + Re[7] * goal.Rd[1] + Re[8] * goal.Rd[2];
      M2 = Re[0] * goal.Rd[6] + Re[1] * goal.Rd[7] + Re[2] * goal.Rd[8];
      M1 = Re[0] * goal.Rd[3] + Re[1] * goal.Rd[4] + Re[2] * goal.Rd[5];
      M3 = Re[3] * goal.Rd[0] + Re[4] * goal.Rd[1] + Re[5] * goal.Rd[2];
      float wx = M5 - M7, wy = M6 - M2, wz = M1 - M3;
      o.rerr = atan2f(0.5f * sqrtf(wx * wx + wy * wy + wz * wz), 0.5f * (tr - 1.f));
    }
    }
    if (tm.w == xl) {
    // joint limits
    float lim = 0.f;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      float hi = q[j] - rb->qhi[j], lo = rb->qlo[j] - q[j];
      float hp = fmaxf(hi, 0.f), lp = fmaxf(lo, 0.f);
      lim += hp * hp + lp * lp;
      if (GRAD) ge[j] += 2.f * P.wl * (hp - lp);
    }
    extra_l = P.wl * lim;
    }
    if (tm.w == xs) extra_l += smoothness<GRAD>(P, q, t, T, ge);
    coll += first ? extra_l + extra_g : 0.f;
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) o.g[j] += first ? ge[j] : 0.f;
    }
  }
  phisum = coll;
  // a team's gradient pass sums the copies inside its reduce-scatter below
  const bool scatter = GRAD && tm.W > 1;
  // sum the shares of the L lanes of this waypoint (butterfly: every copy
  // ends with the same value)
  if (!scatter)
  for (int off = G; off < WAVE; off <<= 1) {
    phisum = xor_reduce<OpSum>(phisum, off);
    if (MODE == EV_RESULT) clr = xor_reduce<OpMin>(clr, off);
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) o.g[j] = xor_reduce<OpSum>(o.g[j], off);
    }
  }
  if (scatter) {
    // ... and of the W wavefronts, summed in wavefront order: wavefront w
    // sums the components c = w mod W of the team (into wavefront 0's row)
    // -- each copy's lanes separately, then the copies by the butterfly --
    // and every wavefront takes the sums
    constexpr int NC = NJ + 1;
    float* base = tm.lds + (tm.buf * tm.W * PART) * WAVE + lane;
    float* mine = base + tm.w * PART * WAVE;
    mine[0] = phisum;
#pragma unroll
    for (int j = 0; j < NJ; ++j) mine[(1 + j) * WAVE] = o.g[j];
    tm.sync();
    for (int cc = tm.w; cc < NC; cc += tm.W) {
      float v = base[cc * WAVE];
      for (int u = 1; u < tm.W; ++u) v += base[(u * PART + cc) * WAVE];
      for (int off = G; off < WAVE; off <<= 1) v = xor_reduce<OpSum>(v, off);
      base[cc * WAVE] = v;
    }
    tm.sync();
    phisum = base[0];
#pragma unroll
    for (int j = 0; j < NJ; ++j) o.g[j] = base[(1 + j) * WAVE];
    tm.buf ^= 1;
  } else if (tm.W > 1) {
    // (cost and result passes: every wavefront sums all shares)
    float* mine = tm.lds + ((tm.buf * tm.W + tm.w) * PART) * WAVE + lane;
    mine[0] = phisum;
    if (MODE == EV_RESULT) mine[(1 + NJ) * WAVE] = clr;
    tm.sync();
    const float* all = tm.lds + (tm.buf * tm.W * PART) * WAVE + lane;
    phisum = all[0];
    if (MODE == EV_RESULT) clr = all[(1 + NJ) * WAVE];
    for (int v = 1; v < tm.W; ++v) {
      const float* pv = all + v * PART * WAVE;
      phisum += pv[0];
      if (MODE == EV_RESULT) clr = fminf(clr, pv[(1 + NJ) * WAVE]);
    }
    tm.buf ^= 1;
  }
  if (MODE == EV_RESULT) o.clr = clr;
  o.cost = active ? phisum : 0.f;
  if (GRAD) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) o.g[j] = (active && t > 0) ? o.g[j] : 0.f;
  }
  return o;
}

// The evaluation form for this team: PIPE when every lane holds at most one
// sphere per link.
template <int MODE, bool EXT>
__device__ __forceinline__ EvalOut eval_any(bool pipe, const RobotDev* __restrict__ rb,
                                            const ParamsDev& P, const Sampler& S, const Goal& goal,
                                            const float* q, int t, int T, int G, bool active,
                                            Team& tm) {
  if (pipe) return evaluate<MODE, true, EXT>(rb, P, S, goal, q, t, T, G, active, tm);
  return evaluate<MODE, false, EXT>(rb, P, S, goal, q, t, T, G, active, tm);
}

__device__ __forceinline__ bool use_pipe(const RobotDev* __restrict__ rb, const Team& tm, int G) {
  return tm.W * (WAVE / G) >= rb->max_per_link;
}

// ------------------------------------------------------------ optimiser ----

struct TileCtx {
  const RobotDev* rb;
  ParamsDev P;
  const ProbDev* pb;
  Sampler S;
  Goal goal;
  DS_GLOBAL float* st;
  int lane, G, t, T, seed;
  bool owner;    // first copy of the waypoint: writes outputs and traces
  bool pipe;     // all-gathers-in-flight evaluation form
  bool active;   // t < T
};

__device__ __forceinline__ DS_GLOBAL float* col(DS_GLOBAL float* st, int base, int j, int lane) {
  return st + base + j * WAVE + lane;
}

// History ring (rho, y^T y, s, y per slot) of one seed, laid out like the
// tile state's history section: in the tile state (global) for single
// wavefronts, or in LDS for a team for the duration of a launch.
constexpr int H_RHO = 0, H_YY = H_RHO + DS_MAX_HISTORY * WAVE, H_S = H_YY + DS_MAX_HISTORY * WAVE,
              H_Y = H_S + DS_MAX_HISTORY * NJ * WAVE, H_FLOATS = H_Y + DS_MAX_HISTORY * NJ * WAVE;
static_assert(ST_YY - ST_RHO == H_YY && ST_S - ST_RHO == H_S && ST_Y - ST_RHO == H_Y &&
                  ST_FLOATS - ST_RHO == H_FLOATS,
              "history layout must match the tile state");

template <class Ptr>
struct Hist {
  Ptr h;      // base of the history section
  int lane;
  __device__ __forceinline__ float s(int k, int j) const { return h[H_S + (k * NJ + j) * WAVE + lane]; }
  __device__ __forceinline__ float y(int k, int j) const { return h[H_Y + (k * NJ + j) * WAVE + lane]; }
  __device__ __forceinline__ float rho(int k) const { return h[H_RHO + k * WAVE + lane]; }
  __device__ __forceinline__ float yy(int k) const { return h[H_YY + k * WAVE + lane]; }
  __device__ __forceinline__ void push(int k, const float* sv, const float* yv, float r, float q) const {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      h[H_S + (k * NJ + j) * WAVE + lane] = sv[j];
      h[H_Y + (k * NJ + j) * WAVE + lane] = yv[j];
    }
    h[H_RHO + k * WAVE + lane] = r;
    h[H_YY + k * WAVE + lane] = q;
  }
};
using LHist = Hist<float*>;

// The ring in the tile state, read and written through a buffer resource:
// the lane's column is the vector offset and slot and joint a scalar one,
// so an access needs no per-lane 64-bit address arithmetic.  Slots are
// wave-uniform (one seed per wavefront).  Only the first copy's lanes that
// hold a waypoint touch memory for s and y: the other copies read the first
// copy's column (the same bits: every copy carries the same s and y), and
// lanes past the horizon (s = y = 0 there) use an offset past the end of
// the buffer, which reads zeros and drops stores without a memory access.
// rho and y^T y, the same in every lane, are read by all lanes from column
// 0 (one broadcast access).
constexpr int HIST_OFF_NONE = 0x7FFFFF00;
struct BHist {
  __amdgpu_buffer_rsrc_t r;
  int vo;   // column * 4 for loads, or HIST_OFF_NONE
  int vw;   // column * 4 for stores (first copy only), or HIST_OFF_NONE
  __device__ __forceinline__ float ld(int idx) const {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, idx * 4, 0));
  }
  __device__ __forceinline__ float ld0(int idx) const {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, 0, idx * 4, 0));
  }
  __device__ __forceinline__ void st(int idx, float v) const {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vw, idx * 4, 0);
  }
  __device__ __forceinline__ float s(int k, int j) const { return ld(H_S + (k * NJ + j) * WAVE); }
  __device__ __forceinline__ float y(int k, int j) const { return ld(H_Y + (k * NJ + j) * WAVE); }
  __device__ __forceinline__ float rho(int k) const { return ld0(H_RHO + k * WAVE); }
  __device__ __forceinline__ float yy(int k) const { return ld0(H_YY + k * WAVE); }
  __device__ __forceinline__ void push(int k, const float* sv, const float* yv, float r, float q) const {
    k = __builtin_amdgcn_readfirstlane(k);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      st(H_S + (k * NJ + j) * WAVE, sv[j]);
      st(H_Y + (k * NJ + j) * WAVE, yv[j]);
    }
    st(H_RHO + k * WAVE, r);
    st(H_YY + k * WAVE, q);
  }
};

// Steepest-descent step scaled so that its largest entry is delta0 (the
// restart direction).
__device__ __forceinline__ void steepest(const TileCtx& c, const float* g, float* d) {
  float gmax = 0.f;
#pragma unroll
  for (int j = 0; j < NJ; ++j) gmax = fmaxf(gmax, fabsf(g[j]));
  gmax = grp_max(gmax, c.G);
  const float sc = c.P.delta0 / fmaxf(gmax, 1e-30f);
#pragma unroll
  for (int j = 0; j < NJ; ++j) d[j] = -g[j] * sc;
}

// A direction's descent test, restart and infinity-norm cap (the seed's
// values are the same in every lane, so the tests are taken wave-uniformly).
__device__ __forceinline__ void restart_and_cap(const TileCtx& c, const float* g, int& cnt,
                                                float* d) {
  const float gtd = grp_sum(dot7(g, d), c.G);
  if (!__builtin_amdgcn_readfirstlane(gtd < 0.f ? 1 : 0)) {
    cnt = 0;
    steepest(c, g, d);
  }
  float dn = 0.f;
#pragma unroll
  for (int j = 0; j < NJ; ++j) dn = fmaxf(dn, fabsf(d[j]));
  dn = grp_max(dn, c.G);
  if (dn > c.P.dmax) {
    const float f = c.P.dmax / dn;
#pragma unroll
    for (int j = 0; j < NJ; ++j) d[j] *= f;
  }
}

// Ring slot of the entry of a given age (0 = newest), 0 <= head < m and
// 0 <= age < m: one conditional wrap, no integer division.
__device__ __forceinline__ int ring_slot(int head, int age, int m) {
  const int s = head - 1 - age;
  return s < 0 ? s + m : s;
}

// L-BFGS direction (two-loop recursion over the history ring),
// steepest-descent restart and infinity-norm cap.  cnt/head are the seed's
// history count and ring head (the same in every lane of the wavefront).
template <class H>
__device__ __forceinline__ void direction(const TileCtx& c, const H& hist, const float* g, int& cnt,
                                          int head, float* d) {
  const int m = c.P.m;
  // one seed per wavefront: count and head are wave-uniform
  const int cmax = __builtin_amdgcn_readfirstlane(cnt);
  const int hd = __builtin_amdgcn_readfirstlane(head);
  // the ring's live slots are read once, all loads in flight together,
  // and both passes of the recursion run on registers
  float hs[DS_MAX_HISTORY][NJ], hy[DS_MAX_HISTORY][NJ], hr[DS_MAX_HISTORY];
  float yy_n = 0.f;
#pragma unroll
  for (int k = 0; k < DS_MAX_HISTORY; ++k) {
    if (k < cmax) {
      const int slot = ring_slot(hd, k, m);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        hs[k][j] = hist.s(slot, j);
        hy[k][j] = hist.y(slot, j);
      }
      hr[k] = hist.rho(slot);
      if (k == 0) yy_n = hist.yy(slot);
    }
  }
  float q[NJ], a[DS_MAX_HISTORY];
#pragma unroll
  for (int j = 0; j < NJ; ++j) q[j] = g[j];
#pragma unroll
  for (int k = 0; k < DS_MAX_HISTORY; ++k) {
    a[k] = 0.f;
    if (k < cmax) {
      const float ak = hr[k] * grp_sum(dot7(hs[k], q), c.G);
      a[k] = ak;
#pragma unroll
      for (int j = 0; j < NJ; ++j) q[j] -= ak * hy[k][j];
    }
  }
  if (cmax > 0) {
    const float gamma = 1.f / (hr[0] * yy_n);   // s^T y / y^T y
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] *= gamma;
  }
#pragma unroll
  for (int k = DS_MAX_HISTORY - 1; k >= 0; --k) {
    if (k < cmax) {
      const float b = hr[k] * grp_sum(dot7(hy[k], q), c.G);
#pragma unroll
      for (int j = 0; j < NJ; ++j) q[j] += hs[k][j] * (a[k] - b);
    }
  }
  if (cmax > 0) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) d[j] = -q[j];
  } else {
    steepest(c, g, d);
  }
  restart_and_cap(c, g, cnt, d);
}

// A team's direction block in LDS: the columns of d, the 2m dot products
// of the history with g, and the ring-slot matrices s_a.y_b and y_a.y_b
// (element (a, b) at a * DS_MAX_HISTORY + b).
constexpr int DL_D = 0, DL_AB = NJ * WAVE, DL_SY = DL_AB + 2 * DS_MAX_HISTORY,
              DL_YY = DL_SY + DS_MAX_HISTORY * DS_MAX_HISTORY,
              DL_FLOATS = DL_YY + DS_MAX_HISTORY * DS_MAX_HISTORY;

// The same direction for a team (W > 1), spread over its wavefronts.  The
// two-loop recursion's result written with inner products (ages k = 0
// newest .. cnt-1; a_k = s_k.g, b_k = y_k.g; SY(k,j) = s_k.y_j,
// YY(k,j) = y_k.y_j):
//   alpha_k = rho_k (a_k - sum_{j<k} alpha_j SY(k,j)),
//   beta_k  = rho_k (gamma (b_k - sum_i alpha_i YY(k,i))
//                    + sum_{j>k} (alpha_j - beta_j) SY(j,k)),
//   H g     = gamma g - sum_k gamma alpha_k y_k + sum_k (alpha_k - beta_k) s_k,
// gamma = s_0.y_0 / y_0.y_0.  Wavefront w reduces a_k, b_k of the ages
// k = w mod W; every wavefront then runs the two triangular recurrences
// (lane i < cnt holds row i) and forms the columns j = w mod W of d.  Every
// wavefront ends with bitwise the same d and cnt.
template <class H>
__device__ __forceinline__ void team_direction(const TileCtx& c, const H& hist, const Team& tm,
                                               const float* g, int& cnt, int head, float* d,
                                               DS_LDS float* dl) {
  const int m = c.P.m;
  const int cu = __builtin_amdgcn_readfirstlane(cnt);
  const int hd = __builtin_amdgcn_readfirstlane(head);

  // wavefront w: ages k = w mod W -- a_k, b_k and the newest pair's row and
  // column of the slot matrices (the same values again when nothing was
  // pushed since the last direction; older pairs were formed when the
  // newer of the two was pushed)
  const int s0 = ring_slot(hd, 0, m);
  for (int k = tm.w; k < cu; k += tm.W) {
    const int b = ring_slot(hd, k, m);
    float sv[NJ], yv[NJ], s0v[NJ], y0v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      sv[j] = hist.s(b, j);
      yv[j] = hist.y(b, j);
      s0v[j] = hist.s(s0, j);
      y0v[j] = hist.y(s0, j);
    }
    const float a = grp_sum(dot7(sv, g), c.G);
    const float bb = grp_sum(dot7(yv, g), c.G);
    const float p0b = grp_sum(dot7(s0v, yv), c.G);   // s_0 . y_k
    const float pb0 = grp_sum(dot7(sv, y0v), c.G);   // s_k . y_0
    const float q0b = grp_sum(dot7(y0v, yv), c.G);   // y_0 . y_k
    if (c.lane == 0) {
      dl[DL_AB + k] = a;
      dl[DL_AB + DS_MAX_HISTORY + k] = bb;
      dl[DL_SY + s0 * DS_MAX_HISTORY + b] = p0b;
      dl[DL_SY + b * DS_MAX_HISTORY + s0] = pb0;
      dl[DL_YY + s0 * DS_MAX_HISTORY + b] = q0b;
      dl[DL_YY + b * DS_MAX_HISTORY + s0] = q0b;
    }
  }
  tm.sync();

  // lane i < cnt holds age i: row i of SY and YY, column i of SY.  Every
  // operand is loaded unconditionally (valid LDS addresses) and entries of
  // ages >= cnt are replaced by zeros, so no stale value reaches a sum.
  const int li = c.lane < m ? c.lane : 0;
  const bool lrow = c.lane < cu;
  const int sli = ring_slot(hd, li, m);
  float syr[DS_MAX_HISTORY], syc[DS_MAX_HISTORY], yyr[DS_MAX_HISTORY], rh[DS_MAX_HISTORY];
  float al[DS_MAX_HISTORY], ee[DS_MAX_HISTORY];
  float acc = lrow ? dl[DL_AB + li] : 0.f;
  float bq = lrow ? dl[DL_AB + DS_MAX_HISTORY + li] : 0.f;
#pragma unroll
  for (int k = 0; k < DS_MAX_HISTORY; ++k) {
    const bool v = k < cu;
    const int sk = ring_slot(hd, k < m ? k : 0, m);
    const float a = dl[DL_SY + sli * DS_MAX_HISTORY + sk];
    const float b = dl[DL_SY + sk * DS_MAX_HISTORY + sli];
    const float e = dl[DL_YY + sli * DS_MAX_HISTORY + sk];
    const float r = hist.rho(sk);
    syr[k] = (v && lrow) ? a : 0.f;
    syc[k] = (v && lrow) ? b : 0.f;
    yyr[k] = (v && lrow) ? e : 0.f;
    rh[k] = v ? r : 0.f;
  }
  // alpha: forward substitution, one age per step (lane k is final at step k)
#pragma unroll
  for (int k = 0; k < DS_MAX_HISTORY; ++k) {
    al[k] = rh[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc), k));
    acc -= al[k] * syr[k];
  }
#pragma unroll
  for (int k = 0; k < DS_MAX_HISTORY; ++k) bq -= al[k] * yyr[k];
  const float gamma = cu > 0 ? 1.f / (hist.rho(s0) * hist.yy(s0)) : 0.f;
  // beta: backward substitution from the oldest age
  float acc2 = gamma * bq;
#pragma unroll
  for (int k = DS_MAX_HISTORY - 1; k >= 0; --k) {
    const float be = rh[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc2), k));
    ee[k] = al[k] - be;
    acc2 += ee[k] * syc[k];
  }
  // the columns j = w mod W of d: all operands loaded before the sums
  for (int j0 = tm.w; j0 < NJ; j0 += tm.W) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (j != j0) continue;
      float sv[DS_MAX_HISTORY], yv[DS_MAX_HISTORY];
#pragma unroll
      for (int k = 0; k < DS_MAX_HISTORY; ++k) {
        const int sk = ring_slot(hd, k < m ? k : 0, m);
        const bool v = k < cu;
        const float a = hist.s(sk, j), b = hist.y(sk, j);
        sv[k] = v ? a : 0.f;
        yv[k] = v ? b : 0.f;
      }
      float r = gamma * g[j];
#pragma unroll
      for (int k = 0; k < DS_MAX_HISTORY; ++k) {
        r += (-gamma * al[k]) * yv[k];
        r += ee[k] * sv[k];
      }
      dl[DL_D + j * WAVE + c.lane] = -r;
    }
  }
  tm.sync();
  if (cu > 0) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) d[j] = dl[DL_D + j * WAVE + c.lane];
  } else {
    steepest(c, g, d);
  }
  restart_and_cap(c, g, cnt, d);
}

// The slot matrices of the cnt valid ring entries, formed from the ring
// (a team resuming a seed in a later launch): the same grp_sum(dot7(.))
// products the direction forms, so a resumed run is bitwise the same.
template <class H>
__device__ __forceinline__ void team_rebuild_products(const TileCtx& c, const H& hist,
                                                      const Team& tm, int cnt, int head,
                                                      DS_LDS float* dl) {
  const int m = c.P.m;
  const int cu = __builtin_amdgcn_readfirstlane(cnt);
  const int hd = __builtin_amdgcn_readfirstlane(head);
  for (int ka = tm.w; ka < cu; ka += tm.W) {
    const int a = ring_slot(hd, ka, m);
    float sa[NJ], ya[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      sa[j] = hist.s(a, j);
      ya[j] = hist.y(a, j);
    }
    for (int kb = 0; kb < cu; ++kb) {
      const int b = ring_slot(hd, kb, m);
      float yb[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) yb[j] = hist.y(b, j);
      const float v = grp_sum(dot7(sa, yb), c.G);
      const float w = grp_sum(dot7(ya, yb), c.G);
      if (c.lane == 0) {
        dl[DL_SY + a * DS_MAX_HISTORY + b] = v;
        dl[DL_YY + a * DS_MAX_HISTORY + b] = w;
      }
    }
  }
}

__device__ __forceinline__ void trace_row(float* buf, const TileCtx& c, int k, const float* v) {
  if (!buf || !c.owner || c.t >= c.T) return;
  size_t base = (((size_t)k * c.pb->S + c.seed) * c.T + c.t) * NJ;
#pragma unroll
  for (int j = 0; j < NJ; ++j) glb(buf)[base + j] = v[j];
}
__device__ __forceinline__ void trace_scalar(float* buf, const TileCtx& c, int k, float v) {
  if (!buf || !c.owner || c.t != 0) return;
  glb(buf)[(size_t)k * c.pb->S + c.seed] = v;
}

// Final per-seed results and output trajectory.
template <bool EXT>
__device__ __forceinline__ int finalize(const TileCtx& c, const float* x, Team& tm) {
  EvalOut r = eval_any<EV_RESULT, EXT>(c.pipe, c.rb, c.P, c.S, c.goal, x, c.t, c.T, c.G, c.active, tm);
  float Jr = grp_sum(r.cost, c.G);
  float clr = grp_min(c.active ? r.clr : FLT_MAX, c.G);
  float perr = grp_sum((c.t == c.T - 1) ? r.perr : 0.f, c.G);
  float rerr = grp_sum((c.t == c.T - 1) ? r.rerr : 0.f, c.G);
  int inlim = 1;
#pragma unroll
  for (int j = 0; j < NJ; ++j) inlim &= (x[j] >= c.rb->qlo[j] && x[j] <= c.rb->qhi[j]) ? 1 : 0;
  float okf = grp_min((c.active && !inlim) ? 0.f : 1.f, c.G);
  // trajectory metrics: largest first, second and third differences
  float vm = 0.f, am = 0.f, jm = 0.f;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    float q1 = __shfl_down(x[j], 1), q2 = __shfl_down(x[j], 2), q3 = __shfl_down(x[j], 3);
    float v1 = q1 - x[j];
    float v2 = q2 - 2.f * q1 + x[j];
    float v3 = q3 - 3.f * q2 + 3.f * q1 - x[j];
    vm = fmaxf(vm, (c.t + 1 < c.T) ? fabsf(v1) : 0.f);
    am = fmaxf(am, (c.t + 2 < c.T) ? fabsf(v2) : 0.f);
    jm = fmaxf(jm, (c.t + 3 < c.T) ? fabsf(v3) : 0.f);
  }
  vm = grp_max(vm, c.G);
  am = grp_max(am, c.G);
  jm = grp_max(jm, c.G);
  if (c.owner && c.t < c.T) {
    DS_GLOBAL float* ft = glb(c.pb->final_traj) + ((size_t)c.seed * c.T + c.t) * NJ;
#pragma unroll
    for (int j = 0; j < NJ; ++j) ft[j] = x[j];
    if (c.pb->out_traj) {
      DS_GLOBAL float* ot = glb(c.pb->out_traj) + ((size_t)c.seed * c.T + c.t) * NJ;
#pragma unroll
      for (int j = 0; j < NJ; ++j) ot[j] = x[j];
    }
  }
  if (c.owner && c.t == 0) {
    ds_seed_result sr;
    sr.cost = Jr;
    sr.clearance = clr;
    sr.pos_err = perr;
    sr.rot_err = rerr;
    const float dt = c.P.dt;
    sr.max_jerk = jm / (dt * dt * dt);
    sr.max_vel = vm / dt;
    sr.max_acc = am / (dt * dt);
    sr.within_vel = sr.max_vel <= c.P.vlim ? 1 : 0;
    // the uniform slow-down s >= 1 that meets the velocity, acceleration and
    // jerk limits (they scale as 1/s, 1/s^2, 1/s^3)
    const float sc = fmaxf(fmaxf(1.f, sr.max_vel / c.P.vlim),
                           fmaxf(sqrtf(sr.max_acc / c.P.alim), cbrtf(sr.max_jerk / c.P.jlim)));
    sr.motion_time = sc * (float)(c.T - 1) * dt;
    sr.valid = isfinite(Jr) ? 1 : 0;
    sr.collision_free = clr > 0.f ? 1 : 0;
    sr.within_limits = okf > 0.5f ? 1 : 0;
    sr.success = (sr.valid && sr.collision_free && sr.within_limits && perr < c.P.tol_pos &&
                  rerr < c.P.tol_rot) ? 1 : 0;
    sr.n_evals_cost = ((const DS_GLOBAL int*)c.st)[ST_EVC + c.lane];
    sr.n_evals_grad = ((const DS_GLOBAL int*)c.st)[ST_EVG + c.lane];
    // field by field: the implicit struct copy has no global-address form
    DS_GLOBAL ds_seed_result* o = glb(c.pb->seed_res) + c.seed;
    o->cost = sr.cost; o->clearance = sr.clearance; o->pos_err = sr.pos_err;
    o->rot_err = sr.rot_err; o->max_jerk = sr.max_jerk;
    o->collision_free = sr.collision_free; o->within_limits = sr.within_limits;
    o->success = sr.success; o->valid = sr.valid; o->n_evals_cost = sr.n_evals_cost;
    o->n_evals_grad = sr.n_evals_grad;
    o->max_vel = sr.max_vel; o->max_acc = sr.max_acc; o->motion_time = sr.motion_time;
    o->within_vel = sr.within_vel;
  }
  return r.ng;
}

enum { PH_INIT = 0, PH_DIR = 1, PH_TRIAL = 2, PH_ACCEPT = 3 };

// Run up to max_iters iterations of one tile (state persists in the arena).
// The wavefront loops over phases around a single cost+gradient evaluation:
//   INIT   evaluate the seed (first launch of the tile only);
//   DIR    direction from the history, trial point x + d;
//   TRIAL  Armijo test of alpha = 1 (its gradient is already there); further
//          cost-only candidates while a seed of the tile has no Armijo step;
//          if a seed accepted alpha < 1, evaluate there (ACCEPT), else update;
//   ACCEPT take the accepted point's cost and gradient, update.
template <bool LDS_HIST, bool EXT>
__device__ __forceinline__ void run_tile(const RobotDev* __restrict__ rb, const ParamsDev* __restrict__ pp,
                         const ProbDev* __restrict__ probs, const TileDev& td, int max_iters,
                         Team& tm, float* hist_lds, uint8_t* coarse_lds, float* dir_lds) {
  TileCtx c;
  c.rb = rb;
  c.P = *pp;
  c.pb = probs + td.prob;
  c.S = make_sampler(c.pb->sc);
  c.goal = make_goal(*c.pb);
  c.st = glb(td.state);
  c.lane = threadIdx.x & (WAVE - 1);
  c.G = td.G;
  c.t = c.lane & (c.G - 1);
  c.T = c.pb->T;
  c.seed = td.seed0;
  c.owner = tm.w == 0 && c.lane < c.G;
  c.pipe = use_pipe(rb, tm, c.G);
  c.active = c.t < c.T;
  const bool writer = tm.w == 0;   // the team's first wavefront writes state
  const int n_iters = c.pb->n_iters;
  DS_GLOBAL int* sti = (DS_GLOBAL int*)c.st;
  const ProbDev& pb = *c.pb;
  // the trace buffers are all set or all null: one flag per tile, so the
  // iteration does not reload the pointers
  const bool tracing = pb.tr_x != nullptr;

  float x[NJ], g[NJ], d[NJ], xe[NJ], gt[NJ];
  float J = 0.f, Jt = 0.f, gtd = 0.f, alpha = 0.f;
  int cnt, head, evc, evg, chosen = 0;
  int ngath = 0;   // cell records gathered by this lane in this launch
  int iter = sti[ST_ITER + c.lane];
  int phase;
  // a tile whose initial evaluation ran in an earlier launch (iteration 0,
  // one gradient evaluation counted) resumes from its state like any other
  if (iter == 0 && sti[ST_EVG + c.lane] == 0) {
    if (c.active) {
      const DS_GLOBAL float* sp = glb(pb.seeds) + ((size_t)c.seed * c.T + c.t) * NJ;
#pragma unroll
      for (int j = 0; j < NJ; ++j) xe[j] = (c.t == 0) ? pb.qs[j] : sp[j];
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) xe[j] = 0.f;
    }
    cnt = head = evc = evg = 0;
    phase = PH_INIT;
  } else {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      x[j] = *col(c.st, ST_X, j, c.lane);
      g[j] = *col(c.st, ST_G, j, c.lane);
    }
    J = c.st[ST_J + c.lane];
    cnt = sti[ST_CNT + c.lane];
    head = sti[ST_HEAD + c.lane];
    evc = sti[ST_EVC + c.lane];
    evg = sti[ST_EVG + c.lane];
    phase = PH_DIR;
  }
  int n_left = min(max_iters, n_iters - iter);
  // the history ring: LDS copy for a team, else the tile state
  typename std::conditional<LDS_HIST, LHist, BHist>::type hist;
  // the scene's coarse table: shared by the team, else this wavefront's own
  c.S.cm = lds(coarse_lds);
  if constexpr (LDS_HIST) {
    hist.lane = c.lane;
    hist.h = hist_lds;
    if (iter > 0 && n_left > 0) {   // resume: bring the ring into LDS
      const DS_GLOBAL float* src = c.st + ST_RHO;
      for (int i = threadIdx.x; i < H_FLOATS; i += tm.W * WAVE) hist_lds[i] = src[i];
    }
    if (c.P.skip) stage_coarse(pb.sc, lds(coarse_lds), threadIdx.x, tm.W * WAVE);
    tm.sync();
    // the slot matrices of a resumed ring (read after the direction's first
    // barrier)
    if (iter > 0 && n_left > 0) team_rebuild_products(c, hist, tm, cnt, head, lds(dir_lds));
  } else {
    hist.r = __builtin_amdgcn_make_buffer_rsrc((void*)(float*)(c.st + ST_RHO), (short)0,
                                               (int)(H_FLOATS * sizeof(float)), RSRC_DWORD3);
    hist.vo = c.active ? (c.lane & (c.G - 1)) * 4 : HIST_OFF_NONE;
    hist.vw = (c.active && c.lane < c.G) ? c.lane * 4 : HIST_OFF_NONE;
    // one wavefront: its LDS accesses complete in order, no barrier needed
    if (c.P.skip) stage_coarse(pb.sc, lds(coarse_lds), c.lane, WAVE);
  }

  for (;;) {
    if (phase == PH_DIR) {
      if (n_left <= 0) break;
      if (tracing) {
        trace_row(pb.tr_x, c, iter, x);
        trace_row(pb.tr_g, c, iter, g);
        trace_scalar(pb.tr_J, c, iter, J);
      }
      if constexpr (LDS_HIST) {
        team_direction(c, hist, tm, g, cnt, head, d, lds(dir_lds));
      } else {
        direction(c, hist, g, cnt, head, d);
      }
      if (tracing) trace_row(pb.tr_d, c, iter, d);
      gtd = grp_sum(dot7(g, d), c.G);
#pragma unroll
      for (int j = 0; j < NJ; ++j) xe[j] = x[j] + d[j];
      phase = PH_TRIAL;
    }
    // the one cost+gradient evaluation of this pass
    EvalOut e = eval_any<EV_GRAD, EXT>(c.pipe, rb, c.P, c.S, c.goal, xe, c.t, c.T, c.G, c.active, tm);
    ++evg;
    ngath += e.ng;
    const float Je = grp_sum(e.cost, c.G);
    if (phase == PH_INIT) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) { x[j] = xe[j]; g[j] = e.g[j]; }
      J = Je;
      phase = PH_DIR;
      continue;
    }
    bool update_now = true;
    if (phase == PH_TRIAL) {
      Jt = Je;
#pragma unroll
      for (int j = 0; j < NJ; ++j) gt[j] = e.g[j];
      chosen = (Jt <= J + c.P.c1 * gtd) ? 0 : -1;
      float Jmin = Jt;
      int kmin = 0;
      for (int kk = 1; kk < c.P.nls; ++kk) {
        bool need = chosen < 0;
        if (!__any(need)) break;
        float al = ldexpf(1.f, -kk);
        float xk[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) xk[j] = x[j] + al * d[j];
        EvalOut ek = eval_any<EV_COST, EXT>(c.pipe, rb, c.P, c.S, c.goal, xk, c.t, c.T, c.G, c.active,
                                       tm);
        ++evc;
        ngath += ek.ng;
        float Jk = grp_sum(ek.cost, c.G);
        if (need && Jk <= J + c.P.c1 * al * gtd) chosen = kk;
        if (need && Jk < Jmin) { Jmin = Jk; kmin = kk; }
      }
      if (chosen < 0 && Jmin < J) chosen = kmin;
      alpha = chosen >= 0 ? ldexpf(1.f, -chosen) : 0.f;
      if (__any(chosen > 0)) {
        // evaluate the accepted step (seeds that took alpha = 1 recompute
        // the same point and keep their trial values)
        float al = chosen > 0 ? alpha : 1.f;
#pragma unroll
        for (int j = 0; j < NJ; ++j) xe[j] = x[j] + al * d[j];
        phase = PH_ACCEPT;
        update_now = false;
      }
    } else {   // PH_ACCEPT
      if (chosen > 0) {
        Jt = Je;
#pragma unroll
        for (int j = 0; j < NJ; ++j) gt[j] = e.g[j];
      }
    }
    if (!update_now) continue;
    // history update and step
    if (tracing) trace_scalar(pb.tr_a, c, iter, alpha);
    const bool accept = chosen >= 0;
    float s[NJ], y[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      float xn = x[j] + alpha * d[j];
      s[j] = accept ? xn - x[j] : 0.f;
      y[j] = accept ? gt[j] - g[j] : 0.f;
    }
    float sy = grp_sum(dot7(s, y), c.G);
    float ss = grp_sum(dot7(s, s), c.G);
    float yy = grp_sum(dot7(y, y), c.G);
    if (accept) {
      if (sy > 1e-10f * sqrtf(ss) * sqrtf(yy)) {
        if (writer) hist.push(head, s, y, 1.f / sy, yy);
        head = (head + 1) % c.P.m;
        cnt = min(cnt + 1, c.P.m);
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) { x[j] = x[j] + alpha * d[j]; g[j] = gt[j]; }
      J = Jt;
    } else {
      cnt = 0;
    }
    ++iter;
    --n_left;
    phase = PH_DIR;
    tm.sync();   // the writer's history is visible to the team
  }
  // persist the state (a team writes its LDS ring back for a later launch)
  if constexpr (LDS_HIST) {
    if (iter < n_iters) {
      DS_GLOBAL float* dst = c.st + ST_RHO;
      for (int i = threadIdx.x; i < H_FLOATS; i += tm.W * WAVE) dst[i] = hist_lds[i];
    }
  }
  if (writer) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      *col(c.st, ST_X, j, c.lane) = x[j];
      *col(c.st, ST_G, j, c.lane) = g[j];
    }
    c.st[ST_J + c.lane] = J;
    sti[ST_CNT + c.lane] = cnt;
    sti[ST_HEAD + c.lane] = head;
    sti[ST_ITER + c.lane] = iter;
    sti[ST_EVC + c.lane] = evc;
    sti[ST_EVG + c.lane] = evg;
  }
  if (iter == n_iters) {
    trace_row(pb.tr_x, c, iter, x);
    trace_row(pb.tr_g, c, iter, g);
    trace_scalar(pb.tr_J, c, iter, J);
    ngath += finalize<EXT>(c, x, tm);
  }
  // this launch's gathers into the seed's counter: every lane adds its own
  // count.  No lane-dependent branch here -- one at the end of the tile body
  // turns the persistent tile loop into a divergent loop, and the wavefront's
  // tile fetch below must run with the whole wavefront.
  __hip_atomic_fetch_add(&glb(pb.seed_res)[c.seed].n_gathers, (unsigned)ngath,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The next tile for this workgroup: from one atomic counter over the
// whole table, or -- with per-XCD queues (xcd_ranges[x] .. xcd_ranges[x+1]
// is queue x, counter[x] its position) -- from the queue of the XCD the
// workgroup runs on (workgroups are dispatched to the 8 XCDs in turn), so
// a problem's tiles, and its scene's records, stay in one XCD's L2; an
// exhausted queue sends the workgroup on to the others.  -1: nothing left.
__device__ __forceinline__ int next_tile(int* counter, const int* __restrict__ xcd_ranges,
                                         int nt) {
  if (!xcd_ranges) {
    const int i = atomicAdd(counter, 1);
    return i < nt ? i : -1;
  }
  const int home = (int)(blockIdx.x % N_XCD);
  for (int q = 0; q < N_XCD; ++q) {
    const int x = (home + q) % N_XCD;
    const int b = xcd_ranges[x], len = xcd_ranges[x + 1] - b;
    if (len <= 0) continue;
    const int i = atomicAdd(&counter[x], 1);
    if (i < len) return b + i;
  }
  return -1;
}

// Persistent optimiser: every team (W = 1: every wavefront) takes tiles
// (next_tile) until the table is exhausted (tile_list, if given, indirects
// the table; n_tiles_dev, if given, overrides n_tiles).  Every member of a
// team sees the same tile sequence and the same decisions, so all of them
// reach every barrier.  Variants: TEAM (W > 1, history ring in LDS) and EXT
// (self-collision and swept terms compiled in); the plain variant carries
// no code for the optional terms.
template <bool TEAM, bool EXT>
__global__ void __launch_bounds__(TEAM ? MAX_TEAM * WAVE : BLOCK, TEAM ? 1 : 2)
k_optimize(const RobotDev* __restrict__ rb, const ParamsDev* __restrict__ pp,
           const ProbDev* __restrict__ probs, const TileDev* __restrict__ tiles,
           const int* __restrict__ tile_list, const int* __restrict__ n_tiles_dev, int n_tiles,
           int* counter, int max_iters, const int* __restrict__ max_iters_dev,
           const int* __restrict__ xcd_ranges) {
  extern __shared__ float s_dyn[];
  __shared__ int s_tile;
  stage_spheres(rb);
  const int lane = threadIdx.x & (WAVE - 1);
  const int nt = n_tiles_dev ? *n_tiles_dev : n_tiles;
  if (max_iters_dev) max_iters = *max_iters_dev;   // serving: set per replay
  Team tm;
  tm.W = TEAM ? pp->waves : 1;
  // wave-uniform (scalar) index, so loops over a wavefront's share stay scalar
  tm.w = TEAM ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)) : 0;
  tm.lds = s_dyn;
  tm.buf = 0;
  for (;;) {
    int mine = 0;
    if constexpr (TEAM) {
      if (threadIdx.x == 0) s_tile = next_tile(counter, xcd_ranges, nt);
      __syncthreads();
      mine = s_tile;
      __syncthreads();
    } else {
      // one fetch per wavefront, by its first active lane, broadcast from
      // that lane (correct for any set of active lanes)
      const int first = __ffsll((long long)__ballot(1)) - 1;
      if (lane == first) mine = next_tile(counter, xcd_ranges, nt);
      mine = __builtin_amdgcn_readfirstlane(__shfl(mine, first));
    }
    if (mine < 0) break;
    const int ti = tile_list ? tile_list[mine] : mine;
    TileDev td = tiles[ti];
    if constexpr (TEAM) {
      run_tile<true, EXT>(rb, pp, probs, td, max_iters, tm, s_dyn + 2 * tm.W * PART * WAVE,
                          reinterpret_cast<uint8_t*>(s_dyn + 2 * tm.W * PART * WAVE + H_FLOATS),
                          s_dyn + 2 * tm.W * PART * WAVE + H_FLOATS + COARSE_FLOATS);
      __syncthreads();   // the LDS ring is free for the next tile
    } else {
      // this wavefront's coarse table (uniform)
      const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
      run_tile<false, EXT>(rb, pp, probs, td, max_iters, tm, nullptr,
                           reinterpret_cast<uint8_t*>(s_dyn + wv * COARSE_FLOATS), nullptr);
    }
  }
}

// Best seed per problem: lowest cost among successful seeds (ties: lowest
// index), else lowest cost among valid seeds.
__global__ void __launch_bounds__(256) k_best(const ProbDev* __restrict__ probs,
                                              const int* __restrict__ list) {
  if (list && (int)blockIdx.x >= list[0]) return;
  const ProbDev& pb = probs[list ? list[1 + blockIdx.x] : blockIdx.x];
  __shared__ int s_any;
  __shared__ unsigned long long s_key[2];
  __shared__ int s_valid;
  if (threadIdx.x == 0) { s_any = 0; s_key[0] = ~0ull; s_key[1] = ~0ull; s_valid = 0; }
  __syncthreads();
  for (int s = threadIdx.x; s < pb.S; s += blockDim.x) {
    const ds_seed_result& r = pb.seed_res[s];
    if (r.valid) {
      atomicAdd(&s_valid, 1);
      // order-preserving key of a finite float cost, then the index
      unsigned u = __float_as_uint(r.cost);
      u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      unsigned long long key = ((unsigned long long)u << 32) | (unsigned)s;
      atomicMin(&s_key[0], key);
      if (r.success) { atomicMin(&s_key[1], key); s_any = 1; }
    }
  }
  __syncthreads();
  const unsigned long long key = s_any ? s_key[1] : s_key[0];
  const int best = (key == ~0ull) ? -1 : (int)(key & 0xffffffffu);
  float* land_traj = pb.landing ? reinterpret_cast<float*>(pb.landing + 256) : nullptr;
  if (best >= 0)
    for (int e = threadIdx.x; e < pb.T * NJ; e += blockDim.x) {
      const float v = pb.final_traj[(size_t)best * pb.T * NJ + e];
      pb.best_traj[e] = v;
      if (land_traj) land_traj[e] = v;
    }
  if (threadIdx.x == 0) {
    ds_result out;
    out.best_seed = best;
    out.n_valid_seeds = s_valid;
    out.n_iters = pb.n_iters;
    if (best >= 0) {
      const ds_seed_result& r = pb.seed_res[best];
      out.success = r.success;
      out.collision_free = r.collision_free;
      out.pos_err_m = r.pos_err;
      out.rot_err_rad = r.rot_err;
      out.cost = r.cost;
      out.min_clearance_m = r.clearance;
      out.max_jerk = r.max_jerk;
      out.max_vel = r.max_vel;
      out.motion_time = r.motion_time;
    } else {
      out.success = 0;
      out.collision_free = 0;
      out.pos_err_m = out.rot_err_rad = out.cost = out.min_clearance_m = out.max_jerk = NAN;
      out.max_vel = out.motion_time = NAN;
    }
    *pb.result = out;
    if (pb.landing) *reinterpret_cast<ds_result*>(pb.landing) = out;
  }
}

// Fresh tiles: each tile's iteration counters (so the optimiser starts from
// the seed) and its seed's result record (counters accumulate over
// launches).  One workgroup of one wavefront per tile.
// Queue order of a batched launch after the tiles' initial evaluation: one
// workgroup per XCD queue sorts its tiles, longest expected first -- by
// lane group (a G = 64 tile walks twice the spheres per lane of a G = 32
// one), then by the cost at the seed (seeds far from a good trajectory
// tend to need more line-search candidates) -- with a counting sort over
// ORDER_BINS keys.  Ties land in any order: the order only decides when a
// seed runs, never what it computes.
constexpr int ORDER_BINS = 4096;
constexpr int ORDER_THREADS = 1024;
__device__ __forceinline__ int order_key(const TileDev& t) {
  const float J = t.state[ST_J];
  const int grp = t.G >= 64 ? 2 : (t.G >= 32 ? 1 : 0);
  // log2(1 + J) in 1/48 steps, 1024 per group; a NaN cost sorts last
  const float l = J > 0.f ? __log2f(1.f + J) * 48.f : 0.f;
  const int b = l >= 0.f ? (int)fminf(l, 1023.f) : 0;
  return grp * 1024 + b;
}
__global__ void __launch_bounds__(ORDER_THREADS) k_queue_order(const TileDev* __restrict__ tiles,
                                                               const int* __restrict__ ranges,
                                                               int* __restrict__ list,
                                                               int* __restrict__ counter) {
  __shared__ int bins[ORDER_BINS];
  const int x = blockIdx.x;
  const int b = ranges[x], e = ranges[x + 1];
  for (int i = threadIdx.x; i < ORDER_BINS; i += blockDim.x) bins[i] = 0;
  if (threadIdx.x == 0) counter[x] = 0;
  __syncthreads();
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) atomicAdd(&bins[order_key(tiles[i])], 1);
  __syncthreads();
  // start of each key's run, largest key first: an exclusive scan of the
  // bins in descending key order.  Thread t owns the PER keys from
  // ORDER_BINS - 1 - PER t downwards; the threads' totals are scanned per
  // wavefront (shuffles), then across the wavefronts (LDS).
  constexpr int PER = ORDER_BINS / ORDER_THREADS;
  constexpr int NW = ORDER_THREADS / WAVE;
  __shared__ int wsum[NW];
  const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
  int cnt[PER], tot = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    cnt[q] = bins[ORDER_BINS - 1 - (PER * t + q)];
    tot += cnt[q];
  }
  int inc = tot;   // inclusive scan of the totals inside the wavefront
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const int o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == WAVE - 1) wsum[wv] = inc;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wv; ++w) base += wsum[w];
  int run = base + inc - tot;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    bins[ORDER_BINS - 1 - (PER * t + q)] = run;
    run += cnt[q];
  }
  __syncthreads();
  for (int i = b + threadIdx.x; i < e; i += blockDim.x)
    list[b + atomicAdd(&bins[order_key(tiles[i])], 1)] = i;
}

__global__ void __launch_bounds__(64) k_tile_reset(const TileDev* __restrict__ tiles,
                                                   const ProbDev* __restrict__ probs,
                                                   int* __restrict__ counter) {
  if (blockIdx.x == 0 && threadIdx.x < N_XCD) counter[threadIdx.x] = 0;   // the tile queues
  const TileDev td = tiles[blockIdx.x];
  reinterpret_cast<int*>(td.state)[ST_ITER + threadIdx.x] = 0;
  reinterpret_cast<int*>(td.state)[ST_EVG + threadIdx.x] = 0;
  constexpr int W = (int)(sizeof(ds_seed_result) / sizeof(int));
  if (threadIdx.x < W)
    reinterpret_cast<int*>(probs[td.prob].seed_res + td.seed0)[threadIdx.x] = 0;
}

// Seed of this wavefront in k_cost / k_guide: W = 1, one seed per
// wavefront (WAVES_PER_BLOCK per workgroup); W > 1, one seed per workgroup
// of W wavefronts (a team, for batches too small to fill the chip).
__device__ __forceinline__ int seed_of(int W, float* team_lds, Team& tm) {
  tm.buf = 0;
  if (W > 1) {
    tm.W = W;
    tm.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    tm.lds = team_lds;
    return blockIdx.x;
  }
  tm.W = 1;
  tm.w = 0;
  tm.lds = nullptr;
  return (blockIdx.x * BLOCK + threadIdx.x) / WAVE;
}

// Objective (and gradient) of arbitrary trajectories: one wavefront (or a
// team) per seed group of G lanes (G = smallest of 16/32/64 holding T).
template <bool EXT>
__global__ void __launch_bounds__(MAX_TEAM * WAVE)
k_cost(const RobotDev* __restrict__ rb, const ParamsDev* __restrict__ pp,
       const ProbDev* __restrict__ pb, const float* __restrict__ X, int S, int T, int G,
       const float* __restrict__ dJ, float* __restrict__ J_out, float* __restrict__ dX,
       int with_grad, int W) {
  extern __shared__ float s_team[];
  __shared__ __attribute__((aligned(16))) uint8_t s_cm[COARSE_BYTES];
  if (pp->skip) stage_coarse(pb->sc, lds(s_cm), threadIdx.x, blockDim.x);
  stage_spheres(rb);
  const int lane = threadIdx.x & (WAVE - 1);
  Team tm;
  const int seed = seed_of(W, s_team, tm);
  if (seed >= S) return;   // whole wavefront (team: whole workgroup) past the end
  const int t = lane & (G - 1);
  const bool owner = tm.w == 0 && lane < G;
  const bool active = t < T;
  ParamsDev P = *pp;
  Sampler Sm = make_sampler(pb->sc);
  Sm.cm = lds(s_cm);
  Goal goal = make_goal(*pb);
  float x[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) x[j] = active ? X[((size_t)seed * T + t) * NJ + j] : 0.f;
  float J;
  if (with_grad) {
    EvalOut e = eval_any<EV_GRAD, EXT>(use_pipe(rb, tm, G), rb, P, Sm, goal, x, t, T, G, active, tm);
    J = grp_sum(e.cost, G);
    float w = dJ ? dJ[seed] : 1.f;
    if (active && owner) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) dX[((size_t)seed * T + t) * NJ + j] = w * e.g[j];
    }
  } else {
    EvalOut e = eval_any<EV_COST, EXT>(use_pipe(rb, tm, G), rb, P, Sm, goal, x, t, T, G, active, tm);
    J = grp_sum(e.cost, G);
  }
  if (J_out && tm.w == 0 && lane == 0) J_out[seed] = J;
}

// Guidance: n gradient steps x <- x - alpha * g on every trajectory, one
// wavefront (or a team) per seed (same evaluation as the optimiser).
template <bool EXT>
__global__ void __launch_bounds__(MAX_TEAM * WAVE)
k_guide(const RobotDev* __restrict__ rb, const ParamsDev* __restrict__ pp,
        const ProbDev* __restrict__ pb, float* __restrict__ X, int S, int T, int G, float alpha,
        int n_steps, float* __restrict__ J_out, int W) {
  extern __shared__ float s_team[];
  __shared__ __attribute__((aligned(16))) uint8_t s_cm[COARSE_BYTES];
  if (pp->skip) stage_coarse(pb->sc, lds(s_cm), threadIdx.x, blockDim.x);
  stage_spheres(rb);
  const int lane = threadIdx.x & (WAVE - 1);
  Team tm;
  const int seed = seed_of(W, s_team, tm);
  if (seed >= S) return;   // whole wavefront (team: whole workgroup) past the end
  const int t = lane & (G - 1);
  const bool owner = tm.w == 0 && lane < G;
  const bool active = t < T;
  ParamsDev P = *pp;
  Sampler Sm = make_sampler(pb->sc);
  Sm.cm = lds(s_cm);
  Goal goal = make_goal(*pb);
  const bool pipe = use_pipe(rb, tm, G);
  float x[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) x[j] = active ? X[((size_t)seed * T + t) * NJ + j] : 0.f;
  for (int k = 0; k < n_steps; ++k) {
    EvalOut e = eval_any<EV_GRAD, EXT>(pipe, rb, P, Sm, goal, x, t, T, G, active, tm);
#pragma unroll
    for (int j = 0; j < NJ; ++j) x[j] -= alpha * e.g[j];
  }
  if (J_out) {
    EvalOut e = eval_any<EV_COST, EXT>(pipe, rb, P, Sm, goal, x, t, T, G, active, tm);
    float J = grp_sum(e.cost, G);
    if (tm.w == 0 && lane == 0) J_out[seed] = J;
  }
  if (active && owner) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) X[((size_t)seed * T + t) * NJ + j] = x[j];
  }
}

// Sphere centres (parity dump), one thread per seed-waypoint.
__global__ void k_spheres(const RobotDev* __restrict__ rb, const float* __restrict__ X, int n,
                          float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float q[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) q[j] = X[(size_t)i * NJ + j];
  float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  float p[3] = {0.f, 0.f, 0.f};
  const int ns = rb->ns;
  for (int l = 0; l < NJ; ++l) {
    const float* F = rb->F[l];
    float A[9], pa[3];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        A[3 * r + c] = R[3 * r] * F[c] + R[3 * r + 1] * F[4 + c] + R[3 * r + 2] * F[8 + c];
      pa[r] = R[3 * r] * F[3] + R[3 * r + 1] * F[7] + R[3 * r + 2] * F[11] + p[r];
    }
    float sn, cs;
    sincosf(q[l], &sn, &cs);
    for (int r = 0; r < 3; ++r) {
      float a0 = A[3 * r], a1 = A[3 * r + 1];
      R[3 * r] = cs * a0 + sn * a1;
      R[3 * r + 1] = cs * a1 - sn * a0;
      R[3 * r + 2] = A[3 * r + 2];
      p[r] = pa[r];
    }
    for (int s = rb->link_begin[l]; s < rb->link_begin[l + 1]; ++s) {
      float4 sp = rb->sph[s];
      float* o = out + ((size_t)i * ns + rb->perm[s]) * 3;
      o[0] = R[0] * sp.x + R[1] * sp.y + R[2] * sp.z + p[0];
      o[1] = R[3] * sp.x + R[4] * sp.y + R[5] * sp.z + p[1];
      o[2] = R[6] * sp.x + R[7] * sp.y + R[8] * sp.z + p[2];
    }
  }
}

// x-fastest node values -> 8-corner cell records.
__global__ void k_esdf_pack(const float* __restrict__ v, int nx, int ny, int nz,
                            float4* __restrict__ rec) {
  const long long cx = nx - 1, cy = ny - 1, cz = nz - 1;
  const long long n = cx * cy * cz;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x) {
    long long i = r % cx, j = (r / cx) % cy, k = r / (cx * cy);
    auto at = [&](long long a, long long b, long long c) { return v[a + nx * (b + (long long)ny * c)]; };
    rec[2 * r] = make_float4(at(i, j, k), at(i + 1, j, k), at(i, j + 1, k), at(i + 1, j + 1, k));
    rec[2 * r + 1] = make_float4(at(i, j, k + 1), at(i + 1, j, k + 1), at(i, j + 1, k + 1),
                                 at(i + 1, j + 1, k + 1));
  }
}

// Coarse table: minimum node value m over each block of 2^shift cells per
// axis (the nodes of the block's cells, inclusive of the far faces), kept
// as the 4-bit level L = the largest L <= 15 with L * cq <= m (0 for a
// negative or NaN m).  One workgroup per block: its threads stride over
// the block's nodes (x runs contiguous), then a shuffle and LDS minimum;
// the level lands in its nibble of the cleared table with an atomic or.
constexpr int COARSE_THREADS = 256;

__global__ void __launch_bounds__(COARSE_THREADS)
k_coarse(const float* __restrict__ v, int nx, int ny, int nz, int shift, int cdx, int cdy,
         float cq, unsigned* __restrict__ out) {
  __shared__ float s_min[COARSE_THREADS / WAVE];
  const int b = blockIdx.x;
  const int bx = b % cdx, by = (b / cdx) % cdy, bz = b / (cdx * cdy);
  const int x0 = bx << shift, x1 = min((bx + 1) << shift, nx - 1);
  const int y0 = by << shift, y1 = min((by + 1) << shift, ny - 1);
  const int z0 = bz << shift, z1 = min((bz + 1) << shift, nz - 1);
  const int lx = x1 - x0 + 1, ly = y1 - y0 + 1, lz = z1 - z0 + 1;
  const int n = lx * ly * lz;
  float m = FLT_MAX;
  for (int e = threadIdx.x; e < n; e += COARSE_THREADS) {
    const int i = e % lx, j = (e / lx) % ly, k = e / (lx * ly);
    m = fminf(m, v[(size_t)(x0 + i) + (size_t)nx * ((y0 + j) + (size_t)ny * (z0 + k))]);
  }
  for (int off = 1; off < WAVE; off <<= 1) m = fminf(m, __shfl_xor(m, off));
  if ((threadIdx.x & (WAVE - 1)) == 0) s_min[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = s_min[0];
    for (int w = 1; w < COARSE_THREADS / WAVE; ++w) r = fminf(r, s_min[w]);
    // fminf drops NaN node values; a NaN minimum (every node NaN) or a
    // negative one gives level 0, which never proves a skip
    unsigned L = 0;
    if (r >= 0.f) {
      L = (unsigned)fminf(floorf(r / cq), 15.f);
      while (L > 0 && (float)L * cq > r) --L;   // the quotient may have rounded up
    }
    atomicOr(&out[b >> 3], L << ((b & 7) * 4));
  }
}

// ---------------------------------------------- ESDF from an occupancy grid --
// Exact squared Euclidean distance transform by separable passes: after the
// pass along x, y and z, f(v) = min over marked voxels w of |v - w|^2 (index
// units).  Every value is an integer below 2^24 (or the "none" sentinel), so
// float arithmetic is exact.
constexpr float EDT_NONE = 1e20f;

__global__ void k_edt_init(const uint8_t* __restrict__ occ, long long n, int target,
                           float* __restrict__ f) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    f[i] = ((occ[i] != 0) == (target != 0)) ? 0.f : EDT_NONE;
}

// One pass along `axis` (0 = x, 1 = y, 2 = z): one workgroup per line, the
// line staged in LDS.  Element p takes min_q (p - q)^2 + f(q) by scanning
// outward from q = p and stopping once r^2 >= the best value so far (every
// farther term is at least r^2): the same minimum as a scan of the whole
// line.  A line with no finite value stays at "none".
__global__ void __launch_bounds__(256)
k_edt_pass(const float* __restrict__ fin, float* __restrict__ fout, int nx, int ny, int nz,
           int axis) {
  extern __shared__ float line[];
  __shared__ int s_any;
  const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
  const long long stride = axis == 0 ? 1 : (axis == 1 ? (long long)nx : (long long)nx * ny);
  // the line's first element
  long long l = blockIdx.x, base;
  if (axis == 0) base = l * nx;
  else if (axis == 1) base = (l / nx) * (long long)nx * ny + (l % nx);
  else base = l;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  int any = 0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const float v = fin[base + q * stride];
    line[q] = v;
    any |= v < EDT_NONE;
  }
  if (any) s_any = 1;
  __syncthreads();
  const bool finite = s_any != 0;
  for (int pidx = threadIdx.x; pidx < n; pidx += blockDim.x) {
    float best = line[pidx];
    if (finite) {
      for (int r = 1; r < n; ++r) {
        const float r2 = (float)(r * r);
        if (r2 >= best) break;
        if (pidx - r >= 0) best = fminf(best, r2 + line[pidx - r]);
        if (pidx + r < n) best = fminf(best, r2 + line[pidx + r]);
      }
    }
    fout[base + pidx * stride] = best;
  }
}

__global__ void k_edt_final(const uint8_t* __restrict__ occ, const float* __restrict__ d_occ,
                            const float* __restrict__ d_free, long long n, float voxel,
                            float* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = occ[i] ? -voxel * sqrtf(d_free[i]) : voxel * sqrtf(d_occ[i]);
}

__global__ void k_zero_i32(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_esdf_pack(const float* vals, int nx, int ny, int nz, float4* rec,
                            hipStream_t s) {
  long long n = (long long)(nx - 1) * (ny - 1) * (nz - 1);
  int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_esdf_pack, dim3(blocks), dim3(256), 0, s, vals, nx, ny, nz, rec);
  return hipGetLastError();
}

hipError_t launch_coarse(const float* vals, int nx, int ny, int nz, int shift, int cdx, int cdy,
                         int cdz, float cq, uint8_t* out, hipStream_t s) {
  hipError_t e = launch_zero_i32(reinterpret_cast<int*>(out), COARSE_BYTES / 4, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coarse, dim3(cdx * cdy * cdz), dim3(COARSE_THREADS), 0, s, vals, nx, ny,
                     nz, shift, cdx, cdy, cq, reinterpret_cast<unsigned*>(out));
  return hipGetLastError();
}

int team_block(int W) { return (W > 1 ? W : WAVES_PER_BLOCK) * WAVE; }
// dynamic LDS of an optimiser workgroup: a team's partial sums (double
// buffered), history ring, coarse table and direction broadcast; single
// wavefronts: one coarse table each
size_t team_lds(int W) {
  return W > 1 ? ((size_t)2 * W * PART * WAVE + H_FLOATS + COARSE_FLOATS + DL_FLOATS) *
                     sizeof(float)
               : (size_t)WAVES_PER_BLOCK * COARSE_FLOATS * sizeof(float);
}

using OptKernel = void (*)(const RobotDev*, const ParamsDev*, const ProbDev*, const TileDev*,
                           const int*, const int*, int, int*, int, const int*, const int*);

static OptKernel optimize_kernel(int W, bool ext) {
  if (W > 1) return ext ? k_optimize<true, true> : k_optimize<true, false>;
  return ext ? k_optimize<false, true> : k_optimize<false, false>;
}

hipError_t launch_optimize(const RobotDev* rb, const ParamsDev* pp, const ProbDev* probs,
                           const TileDev* tiles, int n_tiles, int* counter, int grid_blocks,
                           int max_iters, int W, bool ext, hipStream_t s,
                           const int* xcd_ranges, const int* tile_list) {
  hipLaunchKernelGGL(optimize_kernel(W, ext), dim3(grid_blocks), dim3(team_block(W)),
                     team_lds(W), s, rb, pp, probs, tiles, tile_list, (const int*)nullptr,
                     n_tiles, counter, max_iters, (const int*)nullptr, xcd_ranges);
  return hipGetLastError();
}

hipError_t launch_queue_order(const TileDev* tiles, const int* xcd_ranges, int* list,
                              int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_order, dim3(N_XCD), dim3(ORDER_THREADS), 0, s, tiles, xcd_ranges,
                     list, counter);
  return hipGetLastError();
}

hipError_t launch_serve_step(const RobotDev* rb, const ParamsDev* pp, const ProbDev* probs,
                             const TileDev* tiles, const int* tile_list, int* counter,
                             int max_tiles, int grid_blocks, const int* max_iters_dev, int W,
                             bool ext, hipStream_t s) {
  // tile_list[0] holds the number of listed tiles, the indices follow; the
  // iterations of this replay are read from max_iters_dev
  hipLaunchKernelGGL(optimize_kernel(W, ext), dim3(grid_blocks), dim3(team_block(W)),
                     team_lds(W), s, rb, pp, probs, tiles, tile_list + 1, tile_list, max_tiles,
                     counter, 0, max_iters_dev, (const int*)nullptr);
  return hipGetLastError();
}

int optimize_blocks_per_cu(int W, bool ext) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, optimize_kernel(W, ext), team_block(W),
                                                   team_lds(W)) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_tile_reset(const TileDev* tiles, const ProbDev* probs, int n_tiles, int* counter,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_tile_reset, dim3(n_tiles), dim3(64), 0, s, tiles, probs, counter);
  return hipGetLastError();
}

hipError_t launch_best(const ProbDev* probs, int n_probs, const int* list, hipStream_t s) {
  hipLaunchKernelGGL(k_best, dim3(n_probs), dim3(256), 0, s, probs, list);
  return hipGetLastError();
}

// Team size for k_cost / k_guide: one wavefront per seed when the seeds
// give at least WAVES_PER_BLOCK wavefronts per CU, else teams of up to
// WAVES_PER_BLOCK wavefronts per seed.
static int cost_team(int S, int cu_count) {
  // up to 8 wavefronts per seed while the seeds alone would leave the CUs
  // below two wavefronts per SIMD
  int W = 1;
  while (W < MAX_TEAM && (long long)S * W < (long long)2 * WAVES_PER_BLOCK * cu_count) W *= 2;
  return W;
}

hipError_t launch_cost(const RobotDev* rb, const ParamsDev* pp, const ProbDev* prob,
                       const float* X, int S, int T, const float* dJ, float* J_out, float* dX,
                       int with_grad, bool ext, int cu_count, hipStream_t s) {
  const int G = T <= 16 ? 16 : (T <= 32 ? 32 : 64);
  const int W = cost_team(S, cu_count);
  const int blocks = W > 1 ? S : (S + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const size_t lds_bytes = W > 1 ? (size_t)2 * W * PART * WAVE * sizeof(float) : 0;
  hipLaunchKernelGGL(ext ? k_cost<true> : k_cost<false>, dim3(blocks), dim3(W > 1 ? W * WAVE : BLOCK),
                     lds_bytes, s, rb, pp, prob, X, S, T, G, dJ, J_out, dX, with_grad, W);
  return hipGetLastError();
}

hipError_t launch_guide(const RobotDev* rb, const ParamsDev* pp, const ProbDev* prob, float* X,
                        int S, int T, float alpha, int n_steps, float* J_out, bool ext,
                        int cu_count, hipStream_t s) {
  const int G = T <= 16 ? 16 : (T <= 32 ? 32 : 64);
  const int W = cost_team(S, cu_count);
  const int blocks = W > 1 ? S : (S + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const size_t lds_bytes = W > 1 ? (size_t)2 * W * PART * WAVE * sizeof(float) : 0;
  hipLaunchKernelGGL(ext ? k_guide<true> : k_guide<false>, dim3(blocks), dim3(W > 1 ? W * WAVE : BLOCK),
                     lds_bytes, s, rb, pp, prob, X, S, T, G, alpha, n_steps, J_out, W);
  return hipGetLastError();
}

hipError_t launch_spheres(const RobotDev* rb, const float* X, int S, int T, float* out,
                          hipStream_t s) {
  int n = S * T;
  hipLaunchKernelGGL(k_spheres, dim3((n + 255) / 256), dim3(256), 0, s, rb, X, n, out);
  return hipGetLastError();
}

hipError_t launch_esdf_from_occupancy(const uint8_t* occ, int nx, int ny, int nz, float voxel,
                                      float* w0, float* w1, float* w2, float* w3, float* out,
                                      hipStream_t s) {
  const long long n = (long long)nx * ny * nz;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
  float* chain[2][2] = {{w0, w1}, {w2, w3}};
  for (int c = 0; c < 2; ++c) {   // c = 0: distance to occupied, 1: to free
    hipLaunchKernelGGL(k_edt_init, dim3(blocks), dim3(256), 0, s, occ, n, c == 0 ? 1 : 0,
                       chain[c][0]);
    float* a = chain[c][0];
    float* b = chain[c][1];
    for (int axis = 0; axis < 3; ++axis) {
      int len = axis == 0 ? nx : (axis == 1 ? ny : nz);
      long long lines = n / len;
      hipLaunchKernelGGL(k_edt_pass, dim3((unsigned)lines), dim3(256), len * sizeof(float), s, a,
                         b, nx, ny, nz, axis);
      float* t = a;
      a = b;
      b = t;
    }
    chain[c][0] = a;   // result of the three passes
  }
  hipLaunchKernelGGL(k_edt_final, dim3(blocks), dim3(256), 0, s, occ, chain[0][0], chain[1][0],
                     n, voxel, out);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace dsk
