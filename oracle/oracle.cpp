// FP64 CPU oracle of seeded trajectory optimisation (DiffusionSeeder,
// arXiv 2410.16727).  TEST INFRASTRUCTURE ONLY: the GPU library never links
// or calls this file; only the tests, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no source with the GPU path.
//
// What it computes (App. A.6, "Optimization Problem"): for every seed
// trajectory tau = (q_0 .. q_{T-1}) of a 7-joint arm, minimise
//     C_goal(X_d, FK(q_{T-1})) + C_smooth(tau) + C_world(tau)
// subject to joint limits, for a fixed number of iterations, starting from
// the given seeds (Sec. 4.4), plus the optional self-collision term C_self
// (off unless its weight is set) and optional swept sub-samples between
// waypoints.  The paper names the terms only; the concrete forms below are
// the readings listed in the design notes:
//   * kinematics: T_i = T_{i-1} F_i Rz(q_i), spheres fixed in link frames;
//   * C_world: CHOMP smooth hinge of (trilinear ESDF distance - radius);
//   * C_smooth: squared 1st/2nd/3rd finite differences of the trajectory
//     padded with two copies of q_0 in front and two of q_{T-1} behind;
//   * C_goal: w_p |p_ee - p_d|^2 + w_r (3 - tr(R_d^T R_ee)) / 4;
//   * limits: quadratic penalty outside [q_lo, q_hi];
//   * optimiser: L-BFGS (two-loop recursion, Nocedal & Wright Alg. 7.4)
//     with a four-candidate power-of-two backtracking Armijo search.
// Waypoint 0 is pinned to q_start.  Plain loops, double precision, libm.
//
// Parity pins (tests/test_oracle_*.py): FK invariants, analytic box
// distances, closed-form smoothness on polynomial trajectories,
// quaternion identities, central finite differences, dense BFGS
// recursion, quadratic / Rosenbrock convergence, hand-worked line-search
// choices, the restart / step / cap of the direction, history eviction,
// closed-form trajectory metrics and the one-sided gradient jump that the
// ambiguity bound covers.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <limits>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int NJ = 7;

struct Robot {
  double F[8][12];          // F_1..F_7, F_ee : 3x4 row-major [R | p]
  double qlo[NJ], qhi[NJ];
  int ns = 0;
  std::vector<int> link;    // 1..7
  std::vector<double> off;  // ns*3
  std::vector<double> rad;  // ns
};

struct Grid {
  std::vector<float> v;     // x fastest
  int nx = 0, ny = 0, nz = 0;
  double h = 0, o[3] = {0, 0, 0};
};

struct Params {
  double wc, eps, lv, la, lj, wp, wr, wl;
  int m, nls;
  double c1, delta0, dmax, dt, tol_pos, tol_rot;
  double ws;   // self-collision weight (0: the term is off)
  int nsub;    // swept sub-samples per segment (0: waypoints only)
  double vlim, alim, jlim;   // joint velocity / acceleration / jerk limits (motion time)
};

struct Problem {
  double qs[NJ];
  double pd[3];
  double Rd[9];
  double quat[4];           // normalised goal quaternion (w, x, y, z)
};

// ---------------------------------------------------------------- algebra --
struct Frame { double R[9]; double p[3]; };

Frame compose(const Frame& A, const Frame& B) {
  Frame C;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A.R[3 * r + k] * B.R[3 * k + c];
      C.R[3 * r + c] = s;
    }
    double s = A.p[r];
    for (int k = 0; k < 3; ++k) s += A.R[3 * r + k] * B.p[k];
    C.p[r] = s;
  }
  return C;
}

Frame from34(const double* f) {
  Frame F;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) F.R[3 * r + c] = f[4 * r + c];
    F.p[r] = f[4 * r + 3];
  }
  return F;
}

Frame rotz(double q) {
  Frame F;
  double c = std::cos(q), s = std::sin(q);
  double R[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
  std::memcpy(F.R, R, sizeof R);
  F.p[0] = F.p[1] = F.p[2] = 0;
  return F;
}

void apply(const Frame& F, const double* x, double* y) {
  for (int r = 0; r < 3; ++r)
    y[r] = F.R[3 * r] * x[0] + F.R[3 * r + 1] * x[1] + F.R[3 * r + 2] * x[2] + F.p[r];
}

void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Unit quaternion (w, x, y, z) -> rotation matrix.
void quat_to_R(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Rotation matrix -> unit quaternion (w >= 0), branch on the largest
// diagonal combination for accuracy.
void R_to_quat(const double* R, double* q) {
  double tr = R[0] + R[4] + R[8];
  double w, x, y, z;
  if (tr > 0) {
    double s = std::sqrt(tr + 1.0) * 2;
    w = 0.25 * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    double s = std::sqrt(1.0 + R[0] - R[4] - R[8]) * 2;
    w = (R[7] - R[5]) / s; x = 0.25 * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    double s = std::sqrt(1.0 + R[4] - R[0] - R[8]) * 2;
    w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25 * s; z = (R[5] + R[7]) / s;
  } else {
    double s = std::sqrt(1.0 + R[8] - R[0] - R[4]) * 2;
    w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25 * s;
  }
  double n = std::sqrt(w * w + x * x + y * y + z * z);
  if (w < 0) n = -n;
  q[0] = w / n; q[1] = x / n; q[2] = y / n; q[3] = z / n;
}

// --------------------------------------------------------------------- FK --
// Link frames T_1..T_7 and the end-effector frame (index 7).
void fk(const Robot& rb, const double* q, Frame* T) {
  Frame cur;
  double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  std::memcpy(cur.R, I, sizeof I);
  cur.p[0] = cur.p[1] = cur.p[2] = 0;
  for (int i = 0; i < NJ; ++i) {
    cur = compose(compose(cur, from34(rb.F[i])), rotz(q[i]));
    T[i] = cur;
  }
  T[7] = compose(T[6], from34(rb.F[7]));
}

// ------------------------------------------------------------------- ESDF --
struct Sample {
  double d;
  double g[3];
  double graw[3];           // gradient before zeroing the clamped axes
  int clamped[3];
  int cell[3];
  double f[3];
};

double node(const Grid& G, int i, int j, int k) {
  return (double)G.v[(size_t)i + (size_t)G.nx * ((size_t)j + (size_t)G.ny * (size_t)k)];
}

// Trilinear value and spatial gradient.  Nodes sit at origin + idx*h; the
// query is clamped into the grid and the clamped axes have zero gradient.
// The cell for axis a is min(floor(u_a), n_a - 2).
Sample sample_in_cell(const Grid& G, const double* p, const int* force_cell) {
  Sample S;
  int n[3] = {G.nx, G.ny, G.nz};
  double u[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = (p[a] - G.o[a]) / G.h;
    if (!std::isfinite(u[a])) {
      // a non-finite query has no cell: the sample is NaN
      double nan = std::numeric_limits<double>::quiet_NaN();
      S.d = nan;
      for (int b = 0; b < 3; ++b) { S.g[b] = S.graw[b] = nan; S.clamped[b] = 0; S.cell[b] = 0; S.f[b] = 0; }
      return S;
    }
    S.clamped[a] = 0;
    if (u[a] < 0) { u[a] = 0; S.clamped[a] = 1; }
    if (u[a] > n[a] - 1) { u[a] = n[a] - 1; S.clamped[a] = 1; }
    int i = (int)std::floor(u[a]);
    if (i > n[a] - 2) i = n[a] - 2;
    if (force_cell) i = force_cell[a];
    S.cell[a] = i;
    S.f[a] = u[a] - i;
  }
  int i = S.cell[0], j = S.cell[1], k = S.cell[2];
  double fx = S.f[0], fy = S.f[1], fz = S.f[2];
  double c[2][2][2];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) c[dz][dy][dx] = node(G, i + dx, j + dy, k + dz);
  double wx[2] = {1 - fx, fx}, wy[2] = {1 - fy, fy}, wz[2] = {1 - fz, fz};
  double d = 0, gx = 0, gy = 0, gz = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        double v = c[dz][dy][dx];
        d += wx[dx] * wy[dy] * wz[dz] * v;
        gx += (dx ? 1.0 : -1.0) * wy[dy] * wz[dz] * v;
        gy += wx[dx] * (dy ? 1.0 : -1.0) * wz[dz] * v;
        gz += wx[dx] * wy[dy] * (dz ? 1.0 : -1.0) * v;
      }
  S.d = d;
  S.graw[0] = gx / G.h;
  S.graw[1] = gy / G.h;
  S.graw[2] = gz / G.h;
  S.g[0] = S.clamped[0] ? 0.0 : gx / G.h;
  S.g[1] = S.clamped[1] ? 0.0 : gy / G.h;
  S.g[2] = S.clamped[2] ? 0.0 : gz / G.h;
  return S;
}

Sample sample(const Grid& G, const double* p) { return sample_in_cell(G, p, nullptr); }

// CHOMP smooth hinge and its derivative (activation distance eps).
double hinge(double D, double eps) {
  if (D < 0) return -D + 0.5 * eps;
  if (D < eps) return (D - eps) * (D - eps) / (2 * eps);
  return 0.0;
}
double hinge_d(double D, double eps) {
  if (D < 0) return -1.0;
  if (D < eps) return (D - eps) / eps;
  return 0.0;
}

// ------------------------------------------------------------------- cost --
enum { TERM_WORLD, TERM_VEL, TERM_ACC, TERM_JERK, TERM_GOALP, TERM_GOALR, TERM_LIMIT, TERM_SELF,
       NTERMS };

// Padded sequence P_k = q_{clamp(k-2, 0, T-1)}, k = 0 .. T+3.
inline int pidx(int k, int T) { return std::min(std::max(k - 2, 0), T - 1); }

// Cost of one trajectory X[T][7]; gradient into G (may be null, row 0 zero);
// absolute-contribution magnitude into A (may be null) for tolerance
// scaling; per-term breakdown into terms (may be null).
double cost(const Robot& rb, const Grid& G, const Params& P, const Problem& pr,
            const double* X, int T, double* Gout, double* Aout, double* terms) {
  double tm[NTERMS] = {0};
  std::vector<double> grad(Gout ? (size_t)T * NJ : 0, 0.0);
  std::vector<double> absg(Aout ? (size_t)T * NJ : 0, 0.0);
  Frame Tf[8];
  // -- world collision, every waypoint; gradient by the joint-axis Jacobian
  for (int t = 0; t < T; ++t) {
    const double* q = X + (size_t)t * NJ;
    fk(rb, q, Tf);
    for (int s = 0; s < rb.ns; ++s) {
      int l = rb.link[s];
      double c[3];
      apply(Tf[l - 1], &rb.off[3 * s], c);
      Sample S = sample(G, c);
      double D = S.d - rb.rad[s];
      tm[TERM_WORLD] += P.wc * hinge(D, P.eps);
      if (Gout || Aout) {
        double dphi = P.wc * hinge_d(D, P.eps);
        if (dphi == 0.0) continue;
        double f[3] = {dphi * S.g[0], dphi * S.g[1], dphi * S.g[2]};
        for (int i = 0; i < l; ++i) {
          double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
          double r[3] = {c[0] - Tf[i].p[0], c[1] - Tf[i].p[1], c[2] - Tf[i].p[2]};
          double jc[3];
          cross(zi, r, jc);
          double v = dot3(f, jc);
          if (Gout) grad[(size_t)t * NJ + i] += v;
          if (Aout) absg[(size_t)t * NJ + i] += std::fabs(v);
        }
      }
    }
  }
  // -- swept collision: nsub configurations q = (1 - tau) q_t + tau q_{t+1},
  // tau = i / (nsub + 1), on every segment between waypoints (the paper's
  // trajectories are linearly interpolated between waypoints); the
  // gradient at q splits (1 - tau, tau) onto the two waypoints
  if (P.nsub > 0) {
    double qi[NJ];
    for (int t = 0; t + 1 < T; ++t)
      for (int i = 1; i <= P.nsub; ++i) {
        double tau = (double)i / (P.nsub + 1);
        for (int j = 0; j < NJ; ++j)
          qi[j] = (1.0 - tau) * X[(size_t)t * NJ + j] + tau * X[(size_t)(t + 1) * NJ + j];
        fk(rb, qi, Tf);
        for (int s = 0; s < rb.ns; ++s) {
          int l = rb.link[s];
          double c[3];
          apply(Tf[l - 1], &rb.off[3 * s], c);
          Sample Sm = sample(G, c);
          double D = Sm.d - rb.rad[s];
          tm[TERM_WORLD] += P.wc * hinge(D, P.eps);
          if (!(Gout || Aout)) continue;
          double dphi = P.wc * hinge_d(D, P.eps);
          if (dphi == 0.0) continue;
          double f[3] = {dphi * Sm.g[0], dphi * Sm.g[1], dphi * Sm.g[2]};
          for (int k = 0; k < l; ++k) {
            double zk[3] = {Tf[k].R[2], Tf[k].R[5], Tf[k].R[8]};
            double r[3] = {c[0] - Tf[k].p[0], c[1] - Tf[k].p[1], c[2] - Tf[k].p[2]};
            double jc[3];
            cross(zk, r, jc);
            double v = dot3(f, jc);
            if (Gout) {
              grad[(size_t)t * NJ + k] += (1.0 - tau) * v;
              grad[(size_t)(t + 1) * NJ + k] += tau * v;
            }
            if (Aout) {
              absg[(size_t)t * NJ + k] += std::fabs((1.0 - tau) * v);
              absg[(size_t)(t + 1) * NJ + k] += std::fabs(tau * v);
            }
          }
        }
      }
  }
  // -- self-collision (App. A.6 C_self): every pair of spheres on links at
  // least two apart, the same hinge on their separation
  //    D_ab = |c_a - c_b| - r_a - r_b,
  // force w_s phi'(D) n on a and its opposite on b (n = unit c_a - c_b).
  if (P.ws != 0.0) {
    std::vector<double> cen((size_t)rb.ns * 3);
    for (int t = 0; t < T; ++t) {
      fk(rb, X + (size_t)t * NJ, Tf);
      for (int s = 0; s < rb.ns; ++s) apply(Tf[rb.link[s] - 1], &rb.off[3 * s], &cen[3 * s]);
      for (int a = 0; a < rb.ns; ++a)
        for (int b = 0; b < rb.ns; ++b) {
          if (rb.link[b] - rb.link[a] < 2) continue;
          const double* ca = &cen[3 * a];
          const double* cb = &cen[3 * b];
          double dv[3] = {ca[0] - cb[0], ca[1] - cb[1], ca[2] - cb[2]};
          double dist = std::sqrt(dot3(dv, dv));
          double D = dist - rb.rad[a] - rb.rad[b];
          tm[TERM_SELF] += P.ws * hinge(D, P.eps);
          if (!(Gout || Aout)) continue;
          double dphi = P.ws * hinge_d(D, P.eps);
          if (dphi == 0.0 || dist == 0.0) continue;
          double f[3] = {dphi * dv[0] / dist, dphi * dv[1] / dist, dphi * dv[2] / dist};
          for (int side = 0; side < 2; ++side) {
            const double* c = side ? cb : ca;
            int l = side ? rb.link[b] : rb.link[a];
            double sg = side ? -1.0 : 1.0;
            for (int i = 0; i < l; ++i) {
              double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
              double r[3] = {c[0] - Tf[i].p[0], c[1] - Tf[i].p[1], c[2] - Tf[i].p[2]};
              double jc[3];
              cross(zi, r, jc);
              double v = sg * dot3(f, jc);
              if (Gout) grad[(size_t)t * NJ + i] += v;
              if (Aout) absg[(size_t)t * NJ + i] += std::fabs(v);
            }
          }
        }
    }
  }
  // -- smoothness on the padded sequence
  auto Pq = [&](int k, int j) { return X[(size_t)pidx(k, T) * NJ + j]; };
  auto addg = [&](int k, int j, double v) {
    int t = pidx(k, T);
    if (Gout) grad[(size_t)t * NJ + j] += v;
    if (Aout) absg[(size_t)t * NJ + j] += std::fabs(v);
  };
  for (int j = 0; j < NJ; ++j) {
    for (int k = 0; k <= T + 2; ++k) {
      double r = Pq(k + 1, j) - Pq(k, j);
      tm[TERM_VEL] += P.lv * r * r;
      addg(k + 1, j, 2 * P.lv * r);
      addg(k, j, -2 * P.lv * r);
    }
    for (int k = 1; k <= T + 2; ++k) {
      double r = Pq(k + 1, j) - 2 * Pq(k, j) + Pq(k - 1, j);
      tm[TERM_ACC] += P.la * r * r;
      addg(k + 1, j, 2 * P.la * r);
      addg(k, j, -4 * P.la * r);
      addg(k - 1, j, 2 * P.la * r);
    }
    for (int k = 1; k <= T + 1; ++k) {
      double r = Pq(k + 2, j) - 3 * Pq(k + 1, j) + 3 * Pq(k, j) - Pq(k - 1, j);
      tm[TERM_JERK] += P.lj * r * r;
      addg(k + 2, j, 2 * P.lj * r);
      addg(k + 1, j, -6 * P.lj * r);
      addg(k, j, 6 * P.lj * r);
      addg(k - 1, j, -2 * P.lj * r);
    }
  }
  // -- goal pose at the last waypoint
  {
    const double* q = X + (size_t)(T - 1) * NJ;
    fk(rb, q, Tf);
    const Frame& E = Tf[7];
    double e[3] = {E.p[0] - pr.pd[0], E.p[1] - pr.pd[1], E.p[2] - pr.pd[2]};
    tm[TERM_GOALP] = P.wp * dot3(e, e);
    double tr = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) tr += pr.Rd[3 * b + a] * E.R[3 * b + a];
    tm[TERM_GOALR] = P.wr * (3.0 - tr) / 4.0;
    if (Gout || Aout) {
      // M = R_ee R_d^T ; w = (M23 - M32, M31 - M13, M12 - M21)
      double M[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += E.R[3 * a + k] * pr.Rd[3 * b + k];
          M[3 * a + b] = s;
        }
      double w[3] = {M[5] - M[7], M[6] - M[2], M[1] - M[3]};
      for (int i = 0; i < NJ; ++i) {
        double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
        double r[3] = {E.p[0] - Tf[i].p[0], E.p[1] - Tf[i].p[1], E.p[2] - Tf[i].p[2]};
        double rc[3];
        cross(r, e, rc);
        double vp = 2 * P.wp * dot3(zi, rc);
        double vr = -(P.wr / 4.0) * dot3(zi, w);
        size_t ix = (size_t)(T - 1) * NJ + i;
        if (Gout) grad[ix] += vp + vr;
        if (Aout) absg[ix] += std::fabs(vp) + std::fabs(vr);
      }
    }
  }
  // -- joint limits
  for (int t = 0; t < T; ++t)
    for (int j = 0; j < NJ; ++j) {
      double q = X[(size_t)t * NJ + j];
      double hi = q - rb.qhi[j], lo = rb.qlo[j] - q;
      double v = 0;
      if (hi > 0) { tm[TERM_LIMIT] += P.wl * hi * hi; v += 2 * P.wl * hi; }
      if (lo > 0) { tm[TERM_LIMIT] += P.wl * lo * lo; v -= 2 * P.wl * lo; }
      if (Gout) grad[(size_t)t * NJ + j] += v;
      if (Aout) absg[(size_t)t * NJ + j] += std::fabs(v);
    }
  double J = 0;
  for (int k = 0; k < NTERMS; ++k) J += tm[k];
  if (terms) std::memcpy(terms, tm, sizeof tm);
  if (Gout) {
    for (int j = 0; j < NJ; ++j) grad[j] = 0.0;   // waypoint 0 is pinned
    std::memcpy(Gout, grad.data(), grad.size() * sizeof(double));
  }
  if (Aout) {
    for (int j = 0; j < NJ; ++j) absg[j] = 0.0;
    std::memcpy(Aout, absg.data(), absg.size() * sizeof(double));
  }
  return J;
}

// Per-element bound on how far the gradient can move when an FP32 caller
// picks the neighbouring trilinear cell for a sample within ``tol`` voxel of
// a cell face: |grad d(cell) - grad d(neighbour)| * |w_c phi'| * |J_c|.
// One configuration q; the bound goes into row[0..6].
static int ambiguity_config(const Robot& rb, const Grid& G, const Params& P, const double* q,
                            double tol, double* row) {
  int cnt = 0;
  Frame Tf[8];
  int n[3] = {G.nx, G.ny, G.nz};
  fk(rb, q, Tf);
  for (int s = 0; s < rb.ns; ++s) {
    int l = rb.link[s];
    double c[3];
    apply(Tf[l - 1], &rb.off[3 * s], c);
    Sample S = sample(G, c);
    double D = S.d - rb.rad[s];
    double dphi = std::fabs(P.wc * hinge_d(D, P.eps));
    double worst = 0;
    for (int a = 0; a < 3; ++a) {
      double u = (c[a] - G.o[a]) / G.h;
      double near_lo = std::fabs(u - std::floor(u));
      double near_hi = std::fabs(std::ceil(u) - u);
      bool near_face = std::min(near_lo, near_hi) < tol;
      bool near_clamp = std::fabs(u) < tol || std::fabs(u - (n[a] - 1)) < tol;
      if (!near_face && !near_clamp) continue;
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int cell[3] = {S.cell[0], S.cell[1], S.cell[2]};
        cell[a] += sgn;
        if (cell[a] < 0 || cell[a] > n[a] - 2) continue;
        Sample A = sample_in_cell(G, c, cell);
        for (int b = 0; b < 3; ++b) worst = std::max(worst, std::fabs(A.g[b] - S.g[b]));
      }
      if (near_clamp) worst = std::max(worst, std::fabs(S.graw[a]));
    }
    if (worst == 0 || dphi == 0) continue;
    ++cnt;
    for (int i = 0; i < l; ++i) {
      double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
      double r[3] = {c[0] - Tf[i].p[0], c[1] - Tf[i].p[1], c[2] - Tf[i].p[2]};
      double jc[3];
      cross(zi, r, jc);
      row[i] += dphi * worst * std::sqrt(3.0) * std::sqrt(dot3(jc, jc));
    }
  }
  return cnt;
}

// The bound for every waypoint of X[T][7] and, with swept sub-samples, for
// every interpolated configuration, spread onto the segment's two
// waypoints with the weights its gradient takes (1 - tau, tau).  Row 0 (the
// pinned start) stays zero.
void ambiguity(const Robot& rb, const Grid& G, const Params& P, const double* X, int T,
               double tol, double* amb, int* n_amb) {
  std::fill(amb, amb + (size_t)T * NJ, 0.0);
  int cnt = 0;
  for (int t = 1; t < T; ++t) cnt += ambiguity_config(rb, G, P, X + (size_t)t * NJ, tol,
                                                      amb + (size_t)t * NJ);
  for (int t = 0; t + 1 < T; ++t)
    for (int i = 1; i <= P.nsub; ++i) {
      double tau = (double)i / (P.nsub + 1);
      double qi[NJ], row[NJ] = {0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < NJ; ++j)
        qi[j] = X[(size_t)t * NJ + j] + tau * (X[(size_t)(t + 1) * NJ + j] - X[(size_t)t * NJ + j]);
      cnt += ambiguity_config(rb, G, P, qi, tol, row);
      for (int j = 0; j < NJ; ++j) {
        amb[(size_t)t * NJ + j] += (1 - tau) * row[j];
        amb[(size_t)(t + 1) * NJ + j] += tau * row[j];
      }
    }
  for (int j = 0; j < NJ; ++j) amb[j] = 0.0;
  if (n_amb) *n_amb = cnt;
}

// ------------------------------------------------- float32 error bound ----
// First-order bound, per gradient element, on how far a float32 evaluation
// of the gradient at X can be from the exact one because its kinematics are
// rounded: every sphere centre, joint origin and end-effector position may
// be off by up to `delta` (metres) and every joint axis and the end-effector
// rotation by up to `eta` (radians).  A world sample's contribution to
// element (t, i) is f . (z_i x (c - o_i)) with the force
// f = w_c phi'(d(c) - r) grad d(c); its change is bounded by
//   |K| delta |z_i x (c - o_i)| + |f| (eta |c - o_i| + 2 delta),
// K = df/dc = w_c (phi'' grad d grad d^T + phi' Hess d) (Frobenius norm),
// where Hess d is the trilinear field's (mixed) second derivative in the
// sample's cell and phi'' = 1/eps on the quadratic piece of the hinge.
// The link wrenches are summed about the world origin and then projected,
// so their rounding also scales with the moment arms about the origin:
//   kappa_w 2^-24 (|c| + |o_i|) |f| per sample (kappa_w = the number of terms
// a wrench component sums, bounded by the spheres per link plus one).
// Self-collision pairs and the goal terms are bounded the same way; the
// smoothness and limit terms use the waypoints as given and only round.
// Row 0 (pinned) is zero.
static void trilinear_hessian(const Grid& G, const Sample& S, double H[9]) {
  int i = S.cell[0], j = S.cell[1], k = S.cell[2];
  double fx = S.f[0], fy = S.f[1], fz = S.f[2];
  double wx[2] = {1 - fx, fx}, wy[2] = {1 - fy, fy}, wz[2] = {1 - fz, fz};
  double hxy = 0, hxz = 0, hyz = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        double v = node(G, i + dx, j + dy, k + dz);
        double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        hxy += sx * sy * wz[dz] * v;
        hxz += sx * wy[dy] * sz * v;
        hyz += wx[dx] * sy * sz * v;
      }
  double h2 = G.h * G.h;
  for (int a = 0; a < 9; ++a) H[a] = 0;
  H[1] = H[3] = hxy / h2;
  H[2] = H[6] = hxz / h2;
  H[5] = H[7] = hyz / h2;
  for (int a = 0; a < 3; ++a)
    if (S.clamped[a])
      for (int b = 0; b < 3; ++b) H[3 * a + b] = H[3 * b + a] = 0;
}

static double norm3(const double* v) { return std::sqrt(dot3(v, v)); }

// Bound of one configuration's world samples into row[0..6] with weight w.
static void fp32_bound_world(const Robot& rb, const Grid& G, const Params& P, const double* q,
                             double delta, double eta, double w, double* row) {
  const double u = std::ldexp(1.0, -24);
  int per_link[8] = {0};
  for (int s = 0; s < rb.ns; ++s) per_link[rb.link[s]]++;
  Frame Tf[8];
  fk(rb, q, Tf);
  for (int s = 0; s < rb.ns; ++s) {
    int l = rb.link[s];
    double c[3];
    apply(Tf[l - 1], &rb.off[3 * s], c);
    Sample S = sample(G, c);
    double D = S.d - rb.rad[s];
    double dphi = hinge_d(D, P.eps);
    double ddphi = (D >= 0 && D < P.eps) ? 1.0 / P.eps : 0.0;
    if (dphi == 0.0 && ddphi == 0.0) continue;
    double Hd[9];
    trilinear_hessian(G, S, Hd);
    double K2 = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double k = P.wc * (ddphi * S.g[a] * S.g[b] + dphi * Hd[3 * a + b]);
        K2 += k * k;
      }
    double Kn = std::sqrt(K2);
    double fn = std::fabs(P.wc * dphi) * norm3(S.g);
    double kw = per_link[l] + 1;
    for (int i = 0; i < l; ++i) {
      double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
      double r[3] = {c[0] - Tf[i].p[0], c[1] - Tf[i].p[1], c[2] - Tf[i].p[2]};
      double jc[3];
      cross(zi, r, jc);
      double b = Kn * delta * norm3(jc) + fn * (eta * norm3(r) + 2 * delta) +
                 kw * u * (norm3(c) + norm3(Tf[i].p)) * fn;
      row[i] += w * b;
    }
  }
}

void fp32_bound(const Robot& rb, const Grid& G, const Params& P, const Problem& pr,
                const double* X, int T, double delta, double eta, double* out) {
  const double u = std::ldexp(1.0, -24);
  std::fill(out, out + (size_t)T * NJ, 0.0);
  for (int t = 1; t < T; ++t)
    fp32_bound_world(rb, G, P, X + (size_t)t * NJ, delta, eta, 1.0, out + (size_t)t * NJ);
  // swept sub-samples split onto the segment's two waypoints
  for (int t = 0; t + 1 < T; ++t)
    for (int k = 1; k <= P.nsub; ++k) {
      double tau = (double)k / (P.nsub + 1);
      double qi[NJ], row[NJ] = {0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < NJ; ++j)
        qi[j] = (1.0 - tau) * X[(size_t)t * NJ + j] + tau * X[(size_t)(t + 1) * NJ + j];
      fp32_bound_world(rb, G, P, qi, delta, eta, 1.0, row);
      for (int j = 0; j < NJ; ++j) {
        out[(size_t)t * NJ + j] += (1 - tau) * row[j];
        out[(size_t)(t + 1) * NJ + j] += tau * row[j];
      }
    }
  Frame Tf[8];
  // self-collision pairs: the separation of two centres moves by 2 delta
  if (P.ws != 0.0) {
    std::vector<double> cen((size_t)rb.ns * 3);
    for (int t = 1; t < T; ++t) {
      fk(rb, X + (size_t)t * NJ, Tf);
      for (int s = 0; s < rb.ns; ++s) apply(Tf[rb.link[s] - 1], &rb.off[3 * s], &cen[3 * s]);
      for (int a = 0; a < rb.ns; ++a)
        for (int b = 0; b < rb.ns; ++b) {
          if (rb.link[b] - rb.link[a] < 2) continue;
          const double* ca = &cen[3 * a];
          const double* cb = &cen[3 * b];
          double dv[3] = {ca[0] - cb[0], ca[1] - cb[1], ca[2] - cb[2]};
          double dist = norm3(dv);
          double D = dist - rb.rad[a] - rb.rad[b];
          double dphi = hinge_d(D, P.eps);
          double ddphi = (D >= 0 && D < P.eps) ? 1.0 / P.eps : 0.0;
          if ((dphi == 0.0 && ddphi == 0.0) || dist == 0.0) continue;
          double Kn = std::fabs(P.ws) * (ddphi + std::fabs(dphi) * std::sqrt(2.0) / dist);
          double fn = std::fabs(P.ws * dphi);
          for (int side = 0; side < 2; ++side) {
            const double* c = side ? cb : ca;
            int l = side ? rb.link[b] : rb.link[a];
            for (int i = 0; i < l; ++i) {
              double zi[3] = {Tf[i].R[2], Tf[i].R[5], Tf[i].R[8]};
              double r[3] = {c[0] - Tf[i].p[0], c[1] - Tf[i].p[1], c[2] - Tf[i].p[2]};
              double jc[3];
              cross(zi, r, jc);
              out[(size_t)t * NJ + i] += Kn * 2 * delta * norm3(jc) +
                                         fn * (eta * norm3(r) + 2 * delta) +
                                         8 * u * (norm3(c) + norm3(Tf[i].p)) * fn;
            }
          }
        }
    }
  }
  // goal pose at the last waypoint
  {
    fk(rb, X + (size_t)(T - 1) * NJ, Tf);
    const Frame& E = Tf[7];
    double e[3] = {E.p[0] - pr.pd[0], E.p[1] - pr.pd[1], E.p[2] - pr.pd[2]};
    double M[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double sm = 0;
        for (int k = 0; k < 3; ++k) sm += E.R[3 * a + k] * pr.Rd[3 * b + k];
        M[3 * a + b] = sm;
      }
    double wv[3] = {M[5] - M[7], M[6] - M[2], M[1] - M[3]};
    for (int i = 0; i < NJ; ++i) {
      double r[3] = {E.p[0] - Tf[i].p[0], E.p[1] - Tf[i].p[1], E.p[2] - Tf[i].p[2]};
      double bp = 2 * P.wp * (eta * norm3(r) * norm3(e) + 2 * delta * norm3(e) + norm3(r) * delta);
      double br = (P.wr / 4.0) * (eta * norm3(wv) + 4 * eta);
      out[(size_t)(T - 1) * NJ + i] += bp + br;
    }
  }
  for (int j = 0; j < NJ; ++j) out[j] = 0.0;
}

// The robot's reach: the sum of the frame translations and the largest
// sphere offset bound the distance of every point the kinematics place
// from the base.
double reach(const Robot& rb) {
  double r = 0;
  for (int i = 0; i < 8; ++i) r += std::sqrt(rb.F[i][3] * rb.F[i][3] + rb.F[i][7] * rb.F[i][7] +
                                             rb.F[i][11] * rb.F[i][11]);
  double om = 0;
  for (int s = 0; s < rb.ns; ++s) om = std::max(om, norm3(&rb.off[3 * s]));
  return r + om;
}

// ----------------------------------------------------------- optimiser core --
// Generic L-BFGS with the power-of-two backtracking Armijo search; the
// objective returns J and writes the gradient.
using Objective = std::function<double(const double* x, double* g)>;

struct Pair { std::vector<double> s, y; double rho; };

struct History {
  std::deque<Pair> pairs;   // oldest .. newest
  void clear() { pairs.clear(); }
};

double dot(const double* a, const double* b, int n) {
  double s = 0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

double norm_inf(const double* a, int n) {
  double m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, std::fabs(a[i]));
  return m;
}

// Search direction from the gradient and the history (Alg. 7.4 with
// H_0 = gamma I, gamma = s^T y / y^T y of the newest pair); steepest-descent
// restart when the history is empty or the direction is not a descent
// direction; infinity-norm step cap.  Returns whether the history was
// cleared.
bool direction(const Params& P, History& H, const double* g, int n, double* d) {
  bool cleared = false;
  auto steepest = [&]() {
    double s = P.delta0 / std::max(norm_inf(g, n), 1e-30);
    for (int i = 0; i < n; ++i) d[i] = -g[i] * s;
  };
  if (H.pairs.empty()) {
    steepest();
  } else {
    std::vector<double> q(g, g + n), a(H.pairs.size());
    for (int k = (int)H.pairs.size() - 1; k >= 0; --k) {
      const Pair& p = H.pairs[k];
      a[k] = p.rho * dot(p.s.data(), q.data(), n);
      for (int i = 0; i < n; ++i) q[i] -= a[k] * p.y[i];
    }
    const Pair& nw = H.pairs.back();
    double gamma = dot(nw.s.data(), nw.y.data(), n) / dot(nw.y.data(), nw.y.data(), n);
    for (int i = 0; i < n; ++i) q[i] *= gamma;
    for (size_t k = 0; k < H.pairs.size(); ++k) {
      const Pair& p = H.pairs[k];
      double b = p.rho * dot(p.y.data(), q.data(), n);
      for (int i = 0; i < n; ++i) q[i] += p.s[i] * (a[k] - b);
    }
    for (int i = 0; i < n; ++i) d[i] = -q[i];
  }
  if (!(dot(g, d, n) < 0)) {
    if (!H.pairs.empty()) cleared = true;
    H.clear();
    steepest();
  }
  double dn = norm_inf(d, n);
  if (dn > P.dmax) {
    double s = P.dmax / dn;
    for (int i = 0; i < n; ++i) d[i] *= s;
  }
  return cleared;
}

// Line search: candidate costs J_k = J(x + alpha_k d), alpha_k = 2^-k.
// Largest alpha satisfying Armijo; else the smallest cost if below J(x)
// (ties to the larger step); else 0.  Returns the chosen index or -1.
int choose_step(const Params& P, double J0, double gtd, const double* Jk, int K, double* margin) {
  double mmin = std::numeric_limits<double>::infinity();
  int chosen = -1;
  for (int k = 0; k < K; ++k) {
    double a = std::ldexp(1.0, -k);
    double rhs = J0 + P.c1 * a * gtd;
    mmin = std::min(mmin, std::fabs(Jk[k] - rhs));
    if (chosen < 0 && Jk[k] <= rhs) chosen = k;
  }
  if (chosen < 0) {
    int best = -1;
    for (int k = 0; k < K; ++k)
      if (Jk[k] < J0 && (best < 0 || Jk[k] < Jk[best])) best = k;
    chosen = best;
    if (best >= 0) {
      for (int k = 0; k < K; ++k)
        if (k != best) mmin = std::min(mmin, std::fabs(Jk[k] - Jk[best]));
      mmin = std::min(mmin, std::fabs(J0 - Jk[best]));
    }
  }
  if (margin) *margin = mmin;
  return chosen;
}

struct StepInfo { double alpha; double margin; double gtd; bool cleared; bool pushed; };

// One iteration on state (x, g, J, H).  Jcand receives the K candidate costs.
StepInfo step(const Params& P, const Objective& f, std::vector<double>& x, std::vector<double>& g,
              double& J, History& H, double* d_out, double* Jcand) {
  int n = (int)x.size();
  std::vector<double> d(n), xt(n), gt(n);
  StepInfo info{0, 0, 0, false, false};
  info.cleared = direction(P, H, g.data(), n, d.data());
  info.gtd = dot(g.data(), d.data(), n);
  std::vector<double> Jk(P.nls);
  for (int k = 0; k < P.nls; ++k) {
    double a = std::ldexp(1.0, -k);
    for (int i = 0; i < n; ++i) xt[i] = x[i] + a * d[i];
    Jk[k] = f(xt.data(), nullptr);
  }
  int c = choose_step(P, J, info.gtd, Jk.data(), P.nls, &info.margin);
  if (Jcand) std::copy(Jk.begin(), Jk.end(), Jcand);
  if (d_out) std::copy(d.begin(), d.end(), d_out);
  if (c < 0) {
    if (!H.pairs.empty()) info.cleared = true;
    H.clear();
    info.alpha = 0;
    return info;
  }
  info.alpha = std::ldexp(1.0, -c);
  for (int i = 0; i < n; ++i) xt[i] = x[i] + info.alpha * d[i];
  double Jn = f(xt.data(), gt.data());
  Pair p;
  p.s.resize(n);
  p.y.resize(n);
  for (int i = 0; i < n; ++i) { p.s[i] = xt[i] - x[i]; p.y[i] = gt[i] - g[i]; }
  double sy = dot(p.s.data(), p.y.data(), n);
  double sn = std::sqrt(dot(p.s.data(), p.s.data(), n)), yn = std::sqrt(dot(p.y.data(), p.y.data(), n));
  if (sy > 1e-10 * sn * yn) {
    p.rho = 1.0 / sy;
    H.pairs.push_back(std::move(p));
    while ((int)H.pairs.size() > P.m) H.pairs.pop_front();
    info.pushed = true;
  }
  x.swap(xt);
  g.swap(gt);
  J = Jn;
  return info;
}

// Trajectory objective on the free rows 1..T-1 (row 0 = q_start).
struct TrajObjective {
  const Robot* rb; const Grid* G; const Params* P; const Problem* pr; int T;
  mutable std::vector<double> X, GX;
  double operator()(const double* x, double* g) const {
    X.resize((size_t)T * NJ);
    for (int j = 0; j < NJ; ++j) X[j] = pr->qs[j];
    std::memcpy(X.data() + NJ, x, sizeof(double) * (size_t)(T - 1) * NJ);
    if (!g) return cost(*rb, *G, *P, *pr, X.data(), T, nullptr, nullptr, nullptr);
    GX.resize((size_t)T * NJ);
    double J = cost(*rb, *G, *P, *pr, X.data(), T, GX.data(), nullptr, nullptr);
    std::memcpy(g, GX.data() + NJ, sizeof(double) * (size_t)(T - 1) * NJ);
    return J;
  }
};

// ---------------------------------------------------------------- results --
struct SeedResult {
  double J, clearance, pos_err, rot_err, max_jerk;
  int collision_free, within_limits, success, valid;
  double max_vel, max_acc, motion_time;
  int within_vel;
};

SeedResult results(const Robot& rb, const Grid& G, const Params& P, const Problem& pr,
                   const double* X, int T) {
  SeedResult R{};
  R.J = cost(rb, G, P, pr, X, T, nullptr, nullptr, nullptr);
  R.valid = std::isfinite(R.J) ? 1 : 0;
  Frame Tf[8];
  double clr = std::numeric_limits<double>::infinity();
  for (int t = 0; t < T; ++t) {
    fk(rb, X + (size_t)t * NJ, Tf);
    for (int s = 0; s < rb.ns; ++s) {
      double c[3];
      apply(Tf[rb.link[s] - 1], &rb.off[3 * s], c);
      clr = std::min(clr, sample(G, c).d - rb.rad[s]);
    }
  }
  if (P.nsub > 0) {
    double qi[NJ];
    for (int t = 0; t + 1 < T; ++t)
      for (int i = 1; i <= P.nsub; ++i) {
        double tau = (double)i / (P.nsub + 1);
        for (int j = 0; j < NJ; ++j)
          qi[j] = (1.0 - tau) * X[(size_t)t * NJ + j] + tau * X[(size_t)(t + 1) * NJ + j];
        fk(rb, qi, Tf);
        for (int s = 0; s < rb.ns; ++s) {
          double c[3];
          apply(Tf[rb.link[s] - 1], &rb.off[3 * s], c);
          clr = std::min(clr, sample(G, c).d - rb.rad[s]);
        }
      }
  }
  if (P.ws != 0.0) {
    // with the self-collision term on, the clearance also covers sphere
    // pairs on links at least two apart
    std::vector<double> cen((size_t)rb.ns * 3);
    for (int t = 0; t < T; ++t) {
      fk(rb, X + (size_t)t * NJ, Tf);
      for (int s = 0; s < rb.ns; ++s) apply(Tf[rb.link[s] - 1], &rb.off[3 * s], &cen[3 * s]);
      for (int a = 0; a < rb.ns; ++a)
        for (int b = 0; b < rb.ns; ++b) {
          if (rb.link[b] - rb.link[a] < 2) continue;
          double dv[3] = {cen[3 * a] - cen[3 * b], cen[3 * a + 1] - cen[3 * b + 1],
                          cen[3 * a + 2] - cen[3 * b + 2]};
          clr = std::min(clr, std::sqrt(dot3(dv, dv)) - rb.rad[a] - rb.rad[b]);
        }
    }
  }
  R.clearance = clr;
  R.collision_free = clr > 0 ? 1 : 0;
  fk(rb, X + (size_t)(T - 1) * NJ, Tf);
  double e[3] = {Tf[7].p[0] - pr.pd[0], Tf[7].p[1] - pr.pd[1], Tf[7].p[2] - pr.pd[2]};
  R.pos_err = std::sqrt(dot3(e, e));
  // rotation angle of q_d^{-1} q_ee
  double qe[4];
  R_to_quat(Tf[7].R, qe);
  const double* qd = pr.quat;
  // conj(qd) * qe
  double w = qd[0] * qe[0] + qd[1] * qe[1] + qd[2] * qe[2] + qd[3] * qe[3];
  double vx = qd[0] * qe[1] - qd[1] * qe[0] - qd[2] * qe[3] + qd[3] * qe[2];
  double vy = qd[0] * qe[2] + qd[1] * qe[3] - qd[2] * qe[0] - qd[3] * qe[1];
  double vz = qd[0] * qe[3] - qd[1] * qe[2] + qd[2] * qe[1] - qd[3] * qe[0];
  R.rot_err = 2.0 * std::atan2(std::sqrt(vx * vx + vy * vy + vz * vz), std::fabs(w));
  R.within_limits = 1;
  for (int t = 0; t < T; ++t)
    for (int j = 0; j < NJ; ++j) {
      double q = X[(size_t)t * NJ + j];
      if (!(q >= rb.qlo[j] && q <= rb.qhi[j])) R.within_limits = 0;
    }
  R.success = (R.valid && R.collision_free && R.pos_err < P.tol_pos && R.rot_err < P.tol_rot &&
               R.within_limits) ? 1 : 0;
  // App. A.7 trajectory metrics from the waypoints spaced dt apart: the
  // largest first, second and third difference over all joints (velocity,
  // acceleration, jerk), and the motion time of the trajectory slowed down
  // uniformly just enough to respect the velocity, acceleration and jerk
  // limits (a time scale s divides them by s, s^2 and s^3).
  double mv = 0, ma = 0, mj = 0;
  for (int t = 0; t + 1 < T; ++t)
    for (int j = 0; j < NJ; ++j) {
      double r = X[(size_t)(t + 1) * NJ + j] - X[(size_t)t * NJ + j];
      mv = std::max(mv, std::fabs(r));
    }
  for (int t = 0; t + 2 < T; ++t)
    for (int j = 0; j < NJ; ++j) {
      double r = X[(size_t)(t + 2) * NJ + j] - 2 * X[(size_t)(t + 1) * NJ + j] +
                 X[(size_t)t * NJ + j];
      ma = std::max(ma, std::fabs(r));
    }
  for (int t = 0; t + 3 < T; ++t)
    for (int j = 0; j < NJ; ++j) {
      double r = X[(size_t)(t + 3) * NJ + j] - 3 * X[(size_t)(t + 2) * NJ + j] +
                 3 * X[(size_t)(t + 1) * NJ + j] - X[(size_t)t * NJ + j];
      mj = std::max(mj, std::fabs(r));
    }
  R.max_vel = mv / P.dt;
  R.max_acc = ma / (P.dt * P.dt);
  R.max_jerk = mj / (P.dt * P.dt * P.dt);
  R.within_vel = R.max_vel <= P.vlim ? 1 : 0;
  double scale = std::max({1.0, R.max_vel / P.vlim, std::sqrt(R.max_acc / P.alim),
                           std::cbrt(R.max_jerk / P.jlim)});
  R.motion_time = scale * (T - 1) * P.dt;
  return R;
}

Problem make_problem(const double* qs, const double* goal) {
  Problem pr;
  std::memcpy(pr.qs, qs, sizeof pr.qs);
  std::memcpy(pr.pd, goal, 3 * sizeof(double));
  double n = std::sqrt(goal[3] * goal[3] + goal[4] * goal[4] + goal[5] * goal[5] + goal[6] * goal[6]);
  for (int a = 0; a < 4; ++a) pr.quat[a] = goal[3 + a] / n;
  quat_to_R(pr.quat, pr.Rd);
  return pr;
}

Params make_params(const double* p) {
  Params P;
  P.wc = p[0]; P.eps = p[1]; P.lv = p[2]; P.la = p[3]; P.lj = p[4];
  P.wp = p[5]; P.wr = p[6]; P.wl = p[7];
  P.m = (int)p[8]; P.nls = (int)p[9];
  P.c1 = p[10]; P.delta0 = p[11]; P.dmax = p[12]; P.dt = p[13];
  P.tol_pos = p[14]; P.tol_rot = p[15];
  P.ws = p[16];
  P.nsub = (int)p[17];
  P.vlim = p[18]; P.alim = p[19]; P.jlim = p[20];
  return P;
}

}  // namespace

// ================================================================ C API ====
extern "C" {

void* orc_robot_new(const float* frames /*8*12*/, const float* qlo, const float* qhi, int ns,
                    const int32_t* link, const float* off /*ns*3*/, const float* rad) {
  Robot* r = new Robot();
  for (int i = 0; i < 8; ++i)
    for (int k = 0; k < 12; ++k) r->F[i][k] = frames[12 * i + k];
  for (int j = 0; j < NJ; ++j) { r->qlo[j] = qlo[j]; r->qhi[j] = qhi[j]; }
  r->ns = ns;
  r->link.assign(link, link + ns);
  r->off.resize((size_t)ns * 3);
  r->rad.resize(ns);
  for (int s = 0; s < ns; ++s) {
    for (int a = 0; a < 3; ++a) r->off[3 * s + a] = off[3 * s + a];
    r->rad[s] = rad[s];
  }
  return r;
}
void orc_robot_free(void* r) { delete static_cast<Robot*>(r); }

void* orc_grid_new(const float* vals, int nx, int ny, int nz, float h, const float* origin) {
  Grid* g = new Grid();
  g->v.assign(vals, vals + (size_t)nx * ny * nz);
  g->nx = nx; g->ny = ny; g->nz = nz;
  g->h = h;
  for (int a = 0; a < 3; ++a) g->o[a] = origin[a];
  return g;
}
void orc_grid_free(void* g) { delete static_cast<Grid*>(g); }

// Link frames 1..7 and the end effector: R_out [8][9], p_out [8][3].
void orc_fk(void* rb, const double* q, double* R_out, double* p_out) {
  Frame T[8];
  fk(*static_cast<Robot*>(rb), q, T);
  for (int i = 0; i < 8; ++i) {
    std::memcpy(R_out + 9 * i, T[i].R, sizeof T[i].R);
    std::memcpy(p_out + 3 * i, T[i].p, sizeof T[i].p);
  }
}

// Sphere centres for X[T][7] -> out[T][ns][3].
void orc_spheres(void* rbp, const double* X, int T, double* out) {
  const Robot& rb = *static_cast<Robot*>(rbp);
  Frame Tf[8];
  for (int t = 0; t < T; ++t) {
    fk(rb, X + (size_t)t * NJ, Tf);
    for (int s = 0; s < rb.ns; ++s)
      apply(Tf[rb.link[s] - 1], &rb.off[3 * s], out + ((size_t)t * rb.ns + s) * 3);
  }
}

// out: d, gx, gy, gz, clamped-mask, cell i, j, k
void orc_esdf_sample(void* gp, const double* p, double* out) {
  Sample S = sample(*static_cast<Grid*>(gp), p);
  out[0] = S.d; out[1] = S.g[0]; out[2] = S.g[1]; out[3] = S.g[2];
  out[4] = S.clamped[0] | (S.clamped[1] << 1) | (S.clamped[2] << 2);
  out[5] = S.cell[0]; out[6] = S.cell[1]; out[7] = S.cell[2];
}

double orc_hinge(double D, double eps, double* dphi) {
  if (dphi) *dphi = hinge_d(D, eps);
  return hinge(D, eps);
}

// Cost of S trajectories X[S][T][7]; J_out[S]; G_out[S][T][7] (nullable);
// A_out (nullable) = per-element sum of |contributions|; terms_out[S][7]
// (nullable).
void orc_cost(void* rb, void* g, const double* params, const double* qs, const double* goal,
              const double* X, int S, int T, double* J_out, double* G_out, double* A_out,
              double* terms_out, int nthreads) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rb);
  const Grid& G = *static_cast<Grid*>(g);
  size_t stride = (size_t)T * NJ;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
  for (int s = 0; s < S; ++s)
    J_out[s] = cost(R, G, P, pr, X + s * stride, T, G_out ? G_out + s * stride : nullptr,
                    A_out ? A_out + s * stride : nullptr, terms_out ? terms_out + s * NTERMS : nullptr);
}

// Central differences of J for one trajectory at coordinates idx (flat
// t*7+j), step h.
void orc_fd_grad(void* rb, void* g, const double* params, const double* qs, const double* goal,
                 const double* X, int T, const int32_t* idx, int n, double h, double* out) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  std::vector<double> Y(X, X + (size_t)T * NJ);
  for (int k = 0; k < n; ++k) {
    double x0 = Y[idx[k]];
    Y[idx[k]] = x0 + h;
    double jp = cost(*static_cast<Robot*>(rb), *static_cast<Grid*>(g), P, pr, Y.data(), T, nullptr, nullptr, nullptr);
    Y[idx[k]] = x0 - h;
    double jm = cost(*static_cast<Robot*>(rb), *static_cast<Grid*>(g), P, pr, Y.data(), T, nullptr, nullptr, nullptr);
    Y[idx[k]] = x0;
    out[k] = (jp - jm) / (2 * h);
  }
}

// Gradient ambiguity bound per element for X[T][7] (see ambiguity()).
int orc_ambiguity(void* rb, void* g, const double* params, const double* X, int T, double tol,
                  double* amb) {
  Params P = make_params(params);
  int n = 0;
  ambiguity(*static_cast<Robot*>(rb), *static_cast<Grid*>(g), P, X, T, tol, amb, &n);
  return n;
}

// Float32 error bound per gradient element for X[T][7] (see fp32_bound())
// with delta = kc 2^-24 reach and eta = keta 2^-24; returns the reach.
double orc_fp32_bound(void* rb, void* g, const double* params, const double* qs,
                      const double* goal, const double* X, int T, double kc, double keta,
                      double* out) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rb);
  const double u = std::ldexp(1.0, -24);
  double rr = reach(R);
  fp32_bound(R, *static_cast<Grid*>(g), P, pr, X, T, kc * u * rr, keta * u, out);
  return rr;
}

// Free-running optimisation of S seeds X0[S][T][7] for iters iterations.
// X_out[S][T][7]; J_trace[(iters+1)][S] and alpha_trace[iters][S] nullable.
void orc_optimize(void* rb, void* g, const double* params, const double* qs, const double* goal,
                  const double* X0, int S, int T, int iters, double* X_out, double* J_trace,
                  double* alpha_trace, double* margin_trace, int nthreads) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rb);
  const Grid& G = *static_cast<Grid*>(g);
  size_t stride = (size_t)T * NJ;
  int n = (T - 1) * NJ;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
  for (int s = 0; s < S; ++s) {
    TrajObjective obj{&R, &G, &P, &pr, T, {}, {}};
    Objective f = [&obj](const double* x, double* gg) { return obj(x, gg); };
    std::vector<double> x(n), gr(n);
    for (int i = 0; i < n; ++i) x[i] = X0[s * stride + NJ + i];
    double J = f(x.data(), gr.data());
    if (J_trace) J_trace[s] = J;
    History H;
    for (int k = 0; k < iters; ++k) {
      StepInfo si = step(P, f, x, gr, J, H, nullptr, nullptr);
      if (J_trace) J_trace[(size_t)(k + 1) * S + s] = J;
      if (alpha_trace) alpha_trace[(size_t)k * S + s] = si.alpha;
      if (margin_trace) margin_trace[(size_t)k * S + s] = si.margin;
    }
    for (int j = 0; j < NJ; ++j) X_out[s * stride + j] = pr.qs[j];
    for (int i = 0; i < n; ++i) X_out[s * stride + NJ + i] = x[i];
  }
}

// Generic minimiser for the optimiser pins: f(x, g, user) returns J and
// writes g when g is non-null.
typedef double (*orc_objective_cb)(const double* x, double* g, void* user);
void orc_minimize(orc_objective_cb cb, void* user, const double* params, const double* x0, int n,
                  int iters, double* x_out, double* J_trace) {
  Params P = make_params(params);
  Objective f = [cb, user](const double* x, double* g) { return cb(x, g, user); };
  std::vector<double> x(x0, x0 + n), g(n);
  double J = f(x.data(), g.data());
  if (J_trace) J_trace[0] = J;
  History H;
  for (int k = 0; k < iters; ++k) {
    step(P, f, x, g, J, H, nullptr, nullptr);
    if (J_trace) J_trace[k + 1] = J;
  }
  std::copy(x.begin(), x.end(), x_out);
}

// Two-loop direction for gradient g and history pairs S_hist/Y_hist
// [count][n] (oldest first), without the restart or cap (for the dense
// BFGS pin).  Returns d = -H g.
void orc_two_loop(const double* g, const double* S_hist, const double* Y_hist, int count, int n,
                  double* d) {
  Params P{};
  P.delta0 = 1.0;
  P.dmax = std::numeric_limits<double>::infinity();
  History H;
  for (int k = 0; k < count; ++k) {
    Pair p;
    p.s.assign(S_hist + (size_t)k * n, S_hist + (size_t)(k + 1) * n);
    p.y.assign(Y_hist + (size_t)k * n, Y_hist + (size_t)(k + 1) * n);
    p.rho = 1.0 / dot(p.s.data(), p.y.data(), n);
    H.pairs.push_back(p);
  }
  P.m = count;
  direction(P, H, g, n, d);
}

// Line-search choice for given candidate costs Jk[K] (alpha_k = 2^-k) at
// cost J0 with directional derivative gtd; margin receives the decision
// margin.  Returns the chosen candidate or -1 (no step).
int orc_choose_step(const double* params, double J0, double gtd, const double* Jk, int K,
                    double* margin) {
  Params P = make_params(params);
  return choose_step(P, J0, gtd, Jk, K, margin);
}

// Search direction with the restart and the cap of the optimiser
// (direction()) for gradient g and history pairs S_hist/Y_hist [count][n]
// (oldest first, rho = 1/s.y).  Returns 1 when the history was cleared.
int orc_direction(const double* params, const double* g, const double* S_hist,
                  const double* Y_hist, int count, int n, double* d) {
  Params P = make_params(params);
  History H;
  for (int k = 0; k < count; ++k) {
    Pair p;
    p.s.assign(S_hist + (size_t)k * n, S_hist + (size_t)(k + 1) * n);
    p.y.assign(Y_hist + (size_t)k * n, Y_hist + (size_t)(k + 1) * n);
    p.rho = 1.0 / dot(p.s.data(), p.y.data(), n);
    H.pairs.push_back(p);
  }
  return direction(P, H, g, n, d) ? 1 : 0;
}

// The generic minimiser with a per-iteration record: x_trace, g_trace
// [iters+1][n] (iterate and gradient before each step), d_trace [iters][n]
// (search direction), alpha_trace [iters], pushed [iters] (1 when the pair
// entered the history), hist_count [iters] (history size after the step).
void orc_minimize_trace(orc_objective_cb cb, void* user, const double* params, const double* x0,
                        int n, int iters, double* x_trace, double* g_trace, double* d_trace,
                        double* alpha_trace, int* pushed, int* hist_count) {
  Params P = make_params(params);
  Objective f = [cb, user](const double* x, double* g) { return cb(x, g, user); };
  std::vector<double> x(x0, x0 + n), g(n);
  double J = f(x.data(), g.data());
  History H;
  for (int k = 0; k < iters; ++k) {
    std::copy(x.begin(), x.end(), x_trace + (size_t)k * n);
    std::copy(g.begin(), g.end(), g_trace + (size_t)k * n);
    StepInfo si = step(P, f, x, g, J, H, d_trace + (size_t)k * n, nullptr);
    alpha_trace[k] = si.alpha;
    pushed[k] = si.pushed ? 1 : 0;
    hist_count[k] = (int)H.pairs.size();
  }
  std::copy(x.begin(), x.end(), x_trace + (size_t)iters * n);
  std::copy(g.begin(), g.end(), g_trace + (size_t)iters * n);
}

// Lockstep replay of a traced GPU run of one seed.  Inputs are the GPU's
// per-iteration iterates x_k [iters+1][T][7], gradients g_k, costs J_k,
// directions d_k [iters][T][7] and accepted steps alpha_k [iters].
// Per iteration k it writes rep[k][11]:
//   0 |J_ref(x_k) - J_k| / |J_ref|
//   1 max_e (|g_ref - g_k| - amb_e - B_e - a_coef 2^-24 A_e) / |g_ref|_inf,
//     where B_e is fp32_bound() with delta = kc 2^-24 reach and
//     eta = keta 2^-24, and A_e the element's sum of absolute contributions
//     (rounding of the sums)
//   2 number of ambiguous samples at x_k
//   3 max|d_ref - d_k| / max|d_ref|   (d_ref from the replayed history and g_k)
//   4 alpha_ref (FP64 line search along the GPU's d_k from x_k)
//   5 decision margin / |J_ref|   (near-tie when below 1e-4)
//   6 max|x_{k+1} - (x_k + alpha_k d_k)|
//   7 1 if the GPU's history clear/push decision differs from the replay
//   8 gtd_ref (g_k . d_k in FP64)
//   9 |g_ref|_inf
//  10 max_e (|g_ref - g_k| - amb_e - B_e - 1e-4 |g_ref|_inf) / (2^-24 A_e):
//     the rounding coefficient the element needs beyond the other terms
void orc_lockstep(void* rbp, void* gp, const double* params, const double* qs, const double* goal,
                  int T, int iters, const double* xs, const double* gs, const double* Js,
                  const double* ds, const double* alphas, double amb_tol, double a_coef,
                  double kc, double keta, double* rep) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rbp);
  const Grid& G = *static_cast<Grid*>(gp);
  size_t stride = (size_t)T * NJ;
  int n = (T - 1) * NJ;
  TrajObjective obj{&R, &G, &P, &pr, T, {}, {}};
  History H;
  std::vector<double> gref(stride), A(stride), amb(stride), fb(stride), d(n), xt(n);
  const double u = std::ldexp(1.0, -24);
  const double delta = kc * u * reach(R), eta = keta * u;
  for (int k = 0; k < iters; ++k) {
    const double* xk = xs + k * stride;
    const double* gk = gs + k * stride;
    const double* dk = ds + k * stride;
    double* r = rep + (size_t)k * 11;
    double Jref = cost(R, G, P, pr, xk, T, gref.data(), A.data(), nullptr);
    int na = 0;
    ambiguity(R, G, P, xk, T, amb_tol, amb.data(), &na);
    fp32_bound(R, G, P, pr, xk, T, delta, eta, fb.data());
    double gn = norm_inf(gref.data(), (int)stride);
    double gerr = -std::numeric_limits<double>::infinity(), cneed = 0;
    for (size_t e = NJ; e < stride; ++e) {
      double ex = std::fabs(gref[e] - gk[e]) - amb[e] - fb[e];
      gerr = std::max(gerr, (ex - a_coef * u * A[e]) / std::max(gn, 1e-300));
      double over = ex - 1e-4 * gn;
      if (over > 0) cneed = std::max(cneed, over / std::max(u * A[e], 1e-300));
    }
    r[0] = std::fabs(Jref - Js[k]) / std::fabs(Jref);
    r[1] = gerr;
    r[2] = na;
    r[9] = gn;
    r[10] = cneed;
    // direction from the replayed history and the GPU's gradient
    size_t before = H.pairs.size();
    bool cleared = direction(P, H, gk + NJ, n, d.data());
    double dmax = norm_inf(d.data(), n), derr = 0;
    for (int i = 0; i < n; ++i) derr = std::max(derr, std::fabs(d[i] - dk[NJ + i]));
    r[3] = derr / std::max(dmax, 1e-300);
    (void)before;
    (void)cleared;
    // line search along the GPU's direction
    double gtd = dot(gk + NJ, dk + NJ, n);
    r[8] = gtd;
    std::vector<double> Jk(P.nls);
    for (int c = 0; c < P.nls; ++c) {
      double a = std::ldexp(1.0, -c);
      for (int i = 0; i < n; ++i) xt[i] = xk[NJ + i] + a * dk[NJ + i];
      Jk[c] = obj(xt.data(), nullptr);
    }
    double margin = 0;
    int ch = choose_step(P, Jref, gtd, Jk.data(), P.nls, &margin);
    r[4] = ch < 0 ? 0.0 : std::ldexp(1.0, -ch);
    r[5] = margin / std::fabs(Jref);
    const double* xn = xs + (k + 1) * stride;
    double xerr = 0;
    for (int i = 0; i < n; ++i)
      xerr = std::max(xerr, std::fabs(xn[NJ + i] - (xk[NJ + i] + alphas[k] * dk[NJ + i])));
    r[6] = xerr;
    // replay the history update with the GPU's data and decisions
    r[7] = 0;
    if (alphas[k] > 0) {
      const double* gn = gs + (k + 1) * stride;
      Pair p;
      p.s.resize(n);
      p.y.resize(n);
      for (int i = 0; i < n; ++i) { p.s[i] = xn[NJ + i] - xk[NJ + i]; p.y[i] = gn[NJ + i] - gk[NJ + i]; }
      double sy = dot(p.s.data(), p.y.data(), n);
      double sn = std::sqrt(dot(p.s.data(), p.s.data(), n)), yn = std::sqrt(dot(p.y.data(), p.y.data(), n));
      if (sy > 1e-10 * sn * yn) {
        p.rho = 1.0 / sy;
        H.pairs.push_back(std::move(p));
        while ((int)H.pairs.size() > P.m) H.pairs.pop_front();
      }
    } else {
      H.clear();
    }
  }
}

// Per-seed results for X[S][T][7]: out[S][13] = J, clearance, pos_err,
// rot_err, max_jerk, collision_free, within_limits, success, valid,
// max_vel, max_acc, motion_time, within_vel.
// best[2] = best seed index (-1 if none valid), any-success flag.
void orc_results(void* rb, void* g, const double* params, const double* qs, const double* goal,
                 const double* X, int S, int T, double* out, int* best, int nthreads) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rb);
  const Grid& G = *static_cast<Grid*>(g);
  std::vector<SeedResult> res(S);
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
  for (int s = 0; s < S; ++s) res[s] = results(R, G, P, pr, X + (size_t)s * T * NJ, T);
  int b = -1, any = 0;
  for (int s = 0; s < S; ++s) if (res[s].success) { any = 1; break; }
  for (int s = 0; s < S; ++s) {
    const SeedResult& r = res[s];
    if (!r.valid) continue;
    if (any && !r.success) continue;
    if (b < 0 || r.J < res[b].J) b = s;
  }
  for (int s = 0; s < S; ++s) {
    double* o = out + (size_t)s * 13;
    const SeedResult& r = res[s];
    o[0] = r.J; o[1] = r.clearance; o[2] = r.pos_err; o[3] = r.rot_err; o[4] = r.max_jerk;
    o[5] = r.collision_free; o[6] = r.within_limits; o[7] = r.success; o[8] = r.valid;
    o[9] = r.max_vel; o[10] = r.max_acc; o[11] = r.motion_time; o[12] = r.within_vel;
  }
  best[0] = b;
  best[1] = any;
}

// Guidance steps X <- X - alpha * grad J (rows 1..T-1), n times, per seed.
void orc_guide(void* rb, void* g, const double* params, const double* qs, const double* goal,
               double* X, int S, int T, double alpha, int n, int nthreads) {
  Params P = make_params(params);
  Problem pr = make_problem(qs, goal);
  const Robot& R = *static_cast<Robot*>(rb);
  const Grid& G = *static_cast<Grid*>(g);
  size_t stride = (size_t)T * NJ;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
  for (int s = 0; s < S; ++s) {
    std::vector<double> gr(stride);
    double* x = X + s * stride;
    for (int k = 0; k < n; ++k) {
      cost(R, G, P, pr, x, T, gr.data(), nullptr, nullptr);
      for (size_t e = 0; e < stride; ++e) x[e] -= alpha * gr[e];
    }
  }
}

// Helpers for the quaternion pins.
void orc_quat_to_R(const double* q, double* R) { quat_to_R(q, R); }
void orc_R_to_quat(const double* R, double* q) { R_to_quat(R, q); }

}  // extern "C"

// ===================================================== ESDF construction ====
// Signed Euclidean distance field of an occupancy grid, by its definition:
// a free voxel holds voxel * (distance to the nearest occupied voxel
// centre), an occupied voxel -voxel * (distance to the nearest free voxel
// centre); distances between voxel centres in index units.  Brute force
// over all voxels, for the indices listed in `which` (all when null).
extern "C" int orc_esdf_from_occupancy(const uint8_t* occ, int nx, int ny, int nz, double voxel,
                                       const int64_t* which, int64_t n_which, double* out,
                                       int nthreads) {
  const int64_t N = (int64_t)nx * ny * nz;
  std::vector<int> occ_idx, free_idx;
  for (int64_t i = 0; i < N; ++i) (occ[i] ? occ_idx : free_idx).push_back((int)i);
  if (occ_idx.empty() || free_idx.empty()) return -1;
  const int64_t M = which ? n_which : N;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t m = 0; m < M; ++m) {
    int64_t v = which ? which[m] : m;
    int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
    const std::vector<int>& other = occ[v] ? free_idx : occ_idx;
    double best = std::numeric_limits<double>::infinity();
    for (int w : other) {
      int wx = w % nx, wy = (w / nx) % ny, wz = w / (nx * ny);
      double dx = x - wx, dy = y - wy, dz = z - wz;
      best = std::min(best, dx * dx + dy * dy + dz * dz);
    }
    double d = voxel * std::sqrt(best);
    out[m] = occ[v] ? -d : d;
  }
  return 0;
}
