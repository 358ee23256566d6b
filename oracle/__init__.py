"""ctypes front of the FP64 CPU oracle (``oracle/oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark import this package; the GPU library and
its Python binding never do.  Inputs are the float32 arrays of
``workloads``; everything inside runs in double precision.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

D = C.POINTER(C.c_double)
F = C.POINTER(C.c_float)
I32 = C.POINTER(C.c_int32)
OBJ_CB = C.CFUNCTYPE(C.c_double, D, D, C.c_void_p)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_robot_new.restype = C.c_void_p
        L.orc_robot_new.argtypes = [F, F, F, C.c_int, I32, F, F]
        L.orc_robot_free.argtypes = [C.c_void_p]
        L.orc_grid_new.restype = C.c_void_p
        L.orc_grid_new.argtypes = [F, C.c_int, C.c_int, C.c_int, C.c_float, F]
        L.orc_grid_free.argtypes = [C.c_void_p]
        L.orc_fk.argtypes = [C.c_void_p, D, D, D]
        L.orc_spheres.argtypes = [C.c_void_p, D, C.c_int, D]
        L.orc_esdf_sample.argtypes = [C.c_void_p, D, D]
        L.orc_hinge.restype = C.c_double
        L.orc_hinge.argtypes = [C.c_double, C.c_double, D]
        L.orc_cost.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, C.c_int, D, D, D, D,
                               C.c_int]
        L.orc_fd_grad.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, I32, C.c_int,
                                  C.c_double, D]
        L.orc_ambiguity.restype = C.c_int
        L.orc_ambiguity.argtypes = [C.c_void_p, C.c_void_p, D, D, C.c_int, C.c_double, D]
        L.orc_optimize.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, C.c_int, C.c_int,
                                   D, D, D, D, C.c_int]
        L.orc_minimize.argtypes = [OBJ_CB, C.c_void_p, D, D, C.c_int, C.c_int, D, D]
        L.orc_two_loop.argtypes = [D, D, D, C.c_int, C.c_int, D]
        L.orc_choose_step.restype = C.c_int
        L.orc_choose_step.argtypes = [D, C.c_double, C.c_double, D, C.c_int, D]
        L.orc_direction.restype = C.c_int
        L.orc_direction.argtypes = [D, D, D, D, C.c_int, C.c_int, D]
        L.orc_minimize_trace.argtypes = [OBJ_CB, C.c_void_p, D, D, C.c_int, C.c_int, D, D, D, D,
                                         I32, I32]
        L.orc_lockstep.argtypes = [C.c_void_p, C.c_void_p, D, D, D, C.c_int, C.c_int, D, D, D, D,
                                   D, C.c_double, C.c_double, C.c_double, C.c_double, D]
        L.orc_fp32_bound.restype = C.c_double
        L.orc_fp32_bound.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, C.c_double,
                                     C.c_double, D]
        L.orc_results.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, C.c_int, D, I32,
                                  C.c_int]
        L.orc_esdf_from_occupancy.restype = C.c_int
        L.orc_esdf_from_occupancy.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double,
                                              C.c_void_p, C.c_int64, D, C.c_int]
        L.orc_guide.argtypes = [C.c_void_p, C.c_void_p, D, D, D, D, C.c_int, C.c_int, C.c_double,
                                C.c_int, C.c_int]
        L.orc_quat_to_R.argtypes = [D, D]
        L.orc_R_to_quat.argtypes = [D, D]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(D)


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(F)


def _nullable(a):
    return None if a is None else a.ctypes.data_as(D)


TERMS = ["world", "vel", "acc", "jerk", "goal_pos", "goal_rot", "limit", "self"]
RESULT_FIELDS = ["J", "clearance", "pos_err", "rot_err", "max_jerk", "collision_free",
                 "within_limits", "success", "valid", "max_vel", "max_acc", "motion_time",
                 "within_vel"]


class RobotH:
    def __init__(self, robot):
        L = lib()
        self._keep = [_f(robot.frames.reshape(-1)), _f(robot.q_lo), _f(robot.q_hi),
                      np.ascontiguousarray(robot.sphere_link, dtype=np.int32),
                      _f(robot.sphere_offset.reshape(-1)), _f(robot.sphere_radius)]
        k = self._keep
        self.ns = robot.n_spheres
        self.h = L.orc_robot_new(k[0][1], k[1][1], k[2][1], self.ns,
                                 k[3].ctypes.data_as(I32), k[4][1], k[5][1])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_robot_free(self.h)


class GridH:
    def __init__(self, grid, voxel, origin):
        L = lib()
        g, gp = _f(grid.reshape(-1))
        nz, ny, nx = grid.shape
        o, op = _f(origin)
        self.h = L.orc_grid_new(gp, nx, ny, nz, float(voxel), op)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_grid_free(self.h)


class Oracle:
    """One robot + one scene + parameters."""

    def __init__(self, robot, scene, params_list, threads: int = 1):
        self.robot = RobotH(robot)
        self.grid = GridH(scene.grid, scene.voxel, scene.origin)
        self.params, self._pp = _d(np.array(params_list, dtype=np.float64))
        self.threads = threads
        self.ns = robot.n_spheres

    # -- kinematics / sampling ------------------------------------------
    def fk(self, q):
        q, qp = _d(q)
        R = np.zeros((8, 9))
        p = np.zeros((8, 3))
        lib().orc_fk(self.robot.h, qp, R.ctypes.data_as(D), p.ctypes.data_as(D))
        return R.reshape(8, 3, 3), p

    def spheres(self, X):
        X, xp = _d(X)
        T = X.shape[0]
        out = np.zeros((T, self.ns, 3))
        lib().orc_spheres(self.robot.h, xp, T, out.ctypes.data_as(D))
        return out

    def sample(self, p):
        p, pp = _d(p)
        out = np.zeros(8)
        lib().orc_esdf_sample(self.grid.h, pp, out.ctypes.data_as(D))
        return out

    # -- cost ------------------------------------------------------------
    def cost(self, qs, goal, X, grad=False, absg=False, terms=False):
        """X [S, T, 7] -> dict(J [S], G [S,T,7], A [S,T,7], terms [S,7])."""
        X, xp = _d(X)
        if X.ndim == 2:
            X = X[None]
            xp = X.ctypes.data_as(D)
        S, T, _ = X.shape
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        J = np.zeros(S)
        G = np.zeros((S, T, 7)) if grad else None
        A = np.zeros((S, T, 7)) if absg else None
        TM = np.zeros((S, len(TERMS))) if terms else None
        lib().orc_cost(self.robot.h, self.grid.h, self._pp, qsp, gp, xp, S, T,
                       J.ctypes.data_as(D), _nullable(G), _nullable(A), _nullable(TM),
                       self.threads)
        return {"J": J, "G": G, "A": A, "terms": TM}

    def fd_grad(self, qs, goal, X, idx, h=1e-6):
        X, xp = _d(X)
        T = X.shape[0]
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        out = np.zeros(len(idx))
        lib().orc_fd_grad(self.robot.h, self.grid.h, self._pp, qsp, gp, xp, T,
                          idx.ctypes.data_as(I32), len(idx), h, out.ctypes.data_as(D))
        return out

    def ambiguity(self, X, tol=1e-4):
        X, xp = _d(X)
        T = X.shape[0]
        amb = np.zeros((T, 7))
        n = lib().orc_ambiguity(self.robot.h, self.grid.h, self._pp, xp, T, tol,
                                amb.ctypes.data_as(D))
        return amb, n

    # -- optimiser ---------------------------------------------------------
    def optimize(self, qs, goal, X0, iters, trace=False):
        X0, xp = _d(X0)
        S, T, _ = X0.shape
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        Xo = np.zeros_like(X0)
        Jt = np.zeros((iters + 1, S)) if trace else None
        At = np.zeros((iters, S)) if trace else None
        Mt = np.zeros((iters, S)) if trace else None
        lib().orc_optimize(self.robot.h, self.grid.h, self._pp, qsp, gp, xp, S, T, iters,
                           Xo.ctypes.data_as(D), _nullable(Jt), _nullable(At), _nullable(Mt),
                           self.threads)
        if trace:
            return Xo, {"J": Jt, "alpha": At, "margin": Mt}
        return Xo

    def fp32_bound(self, qs, goal, X, kc, keta):
        """Per-element float32 error bound of the gradient at X [T, 7]
        (orc_fp32_bound): returns (bound [T, 7], reach)."""
        X, xp = _d(X)
        T = X.shape[0]
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        out = np.zeros((T, 7))
        rr = lib().orc_fp32_bound(self.robot.h, self.grid.h, self._pp, qsp, gp, xp, T,
                                  float(kc), float(keta), out.ctypes.data_as(D))
        return out, rr

    def lockstep(self, qs, goal, xs, gs, Js, ds, alphas, amb_tol=1e-4, a_coef=32.0, kc=16.0,
                 keta=16.0):
        """Replay one seed's GPU trace; returns rep [iters, 11] (see
        orc_lockstep; a_coef, kc and keta are the coefficients of the
        gradient tolerance's rounding and float32-kinematics terms)."""
        xs, xp = _d(xs)
        gs, gsp = _d(gs)
        Js, jp = _d(Js)
        ds, dp = _d(ds)
        alphas, ap = _d(alphas)
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        iters = alphas.shape[0]
        T = xs.shape[1]
        rep = np.zeros((iters, 11))
        lib().orc_lockstep(self.robot.h, self.grid.h, self._pp, qsp, gp, T, iters, xp, gsp, jp,
                           dp, ap, amb_tol, float(a_coef), float(kc), float(keta),
                           rep.ctypes.data_as(D))
        return rep

    def guide(self, qs, goal, X, alpha, n):
        """n steps X <- X - alpha * grad J (returns the new X)."""
        X = np.array(X, dtype=np.float64, copy=True)
        S, T, _ = X.shape
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        lib().orc_guide(self.robot.h, self.grid.h, self._pp, qsp, gp, X.ctypes.data_as(D), S, T,
                        float(alpha), int(n), self.threads)
        return X

    def results(self, qs, goal, X):
        X, xp = _d(X)
        S, T, _ = X.shape
        qs, qsp = _d(qs)
        goal, gp = _d(goal)
        out = np.zeros((S, len(RESULT_FIELDS)))
        best = np.zeros(2, dtype=np.int32)
        lib().orc_results(self.robot.h, self.grid.h, self._pp, qsp, gp, xp, S, T,
                          out.ctypes.data_as(D), best.ctypes.data_as(I32), self.threads)
        res = {k: out[:, i] for i, k in enumerate(RESULT_FIELDS)}
        res["best"] = int(best[0])
        res["any_success"] = bool(best[1])
        return res


def minimize(f, x0, iters, params_list):
    """Run the oracle's L-BFGS on a Python objective f(x) -> (J, g)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = x0.shape[0]

    def cb(xp, gp, _user):
        x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        J, g = f(x)
        if gp:
            np.ctypeslib.as_array(gp, shape=(n,))[:] = g
        return float(J)

    cfunc = OBJ_CB(cb)
    pp = np.ascontiguousarray(params_list, dtype=np.float64)
    xo = np.zeros(n)
    Jt = np.zeros(iters + 1)
    lib().orc_minimize(cfunc, None, pp.ctypes.data_as(D), x0.ctypes.data_as(D), n, iters,
                       xo.ctypes.data_as(D), Jt.ctypes.data_as(D))
    return xo, Jt


def choose_step(J0, gtd, Jk, params_list):
    """Line-search choice for candidate costs Jk (alpha_k = 2^-k): returns
    (index or -1, decision margin)."""
    Jk, jp = _d(Jk)
    pp, ppp = _d(params_list)
    m = C.c_double()
    k = lib().orc_choose_step(ppp, float(J0), float(gtd), jp, Jk.shape[0], C.byref(m))
    return k, m.value


def direction(g, S_hist, Y_hist, params_list):
    """The optimiser's search direction (restart and cap included) for
    history pairs [count][n], oldest first: returns (d, history cleared)."""
    g, gp = _d(g)
    n = g.shape[0]
    S_hist, sp = _d(np.asarray(S_hist, dtype=np.float64).reshape(-1, n))
    Y_hist, yp = _d(np.asarray(Y_hist, dtype=np.float64).reshape(-1, n))
    pp, ppp = _d(params_list)
    d = np.zeros(n)
    cl = lib().orc_direction(ppp, gp, sp, yp, S_hist.shape[0], n, d.ctypes.data_as(D))
    return d, bool(cl)


def minimize_trace(f, x0, iters, params_list):
    """The oracle's L-BFGS on f(x) -> (J, g) with a per-iteration record:
    dict(x, g [iters+1, n], d [iters, n], alpha, pushed, count [iters])."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = x0.shape[0]

    def cb(xp, gp, _user):
        x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        J, g = f(x)
        if gp:
            np.ctypeslib.as_array(gp, shape=(n,))[:] = g
        return float(J)

    cfunc = OBJ_CB(cb)
    pp = np.ascontiguousarray(params_list, dtype=np.float64)
    out = {"x": np.zeros((iters + 1, n)), "g": np.zeros((iters + 1, n)),
           "d": np.zeros((iters, n)), "alpha": np.zeros(iters),
           "pushed": np.zeros(iters, dtype=np.int32), "count": np.zeros(iters, dtype=np.int32)}
    lib().orc_minimize_trace(cfunc, None, pp.ctypes.data_as(D), x0.ctypes.data_as(D), n, iters,
                             out["x"].ctypes.data_as(D), out["g"].ctypes.data_as(D),
                             out["d"].ctypes.data_as(D), out["alpha"].ctypes.data_as(D),
                             out["pushed"].ctypes.data_as(I32), out["count"].ctypes.data_as(I32))
    return out


def two_loop(g, S_hist, Y_hist):
    g, gp = _d(g)
    S_hist, sp = _d(S_hist)
    Y_hist, yp = _d(Y_hist)
    d = np.zeros_like(g)
    lib().orc_two_loop(gp, sp, yp, S_hist.shape[0], g.shape[0], d.ctypes.data_as(D))
    return d


def quat_to_R(q):
    q, qp = _d(q)
    R = np.zeros(9)
    lib().orc_quat_to_R(qp, R.ctypes.data_as(D))
    return R.reshape(3, 3)


def R_to_quat(R):
    R, rp = _d(np.asarray(R).reshape(-1))
    q = np.zeros(4)
    lib().orc_R_to_quat(rp, q.ctypes.data_as(D))
    return q


def hinge(D_, eps):
    dphi = C.c_double()
    v = lib().orc_hinge(D_, eps, C.byref(dphi))
    return v, dphi.value


def fk_frames(robot_h: RobotH, q):
    """Link frames 1..7 and the end effector for one configuration."""
    q, qp = _d(q)
    R = np.zeros((8, 9))
    p = np.zeros((8, 3))
    lib().orc_fk(robot_h.h, qp, R.ctypes.data_as(D), p.ctypes.data_as(D))
    return R.reshape(8, 3, 3), p


def sphere_centres(robot_h: RobotH, X):
    X, xp = _d(X)
    T = X.shape[0]
    out = np.zeros((T, robot_h.ns, 3))
    lib().orc_spheres(robot_h.h, xp, T, out.ctypes.data_as(D))
    return out


def esdf_from_occupancy(occ, voxel, which=None, threads=8):
    """Signed distance of an occupancy grid occ [nz, ny, nx] (bool/uint8) at
    all voxels (returns [nz, ny, nx]) or at flat indices ``which``."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    nz, ny, nx = occ.shape
    if which is None:
        out = np.zeros(occ.size)
        wp, n = None, 0
    else:
        which = np.ascontiguousarray(which, dtype=np.int64)
        out = np.zeros(len(which))
        wp, n = which.ctypes.data_as(C.c_void_p), len(which)
    rc = lib().orc_esdf_from_occupancy(occ.ctypes.data_as(C.c_void_p), nx, ny, nz, float(voxel),
                                       wp, n, out.ctypes.data_as(D), threads)
    if rc != 0:
        raise ValueError("occupancy grid needs at least one occupied and one free voxel")
    return out.reshape(occ.shape) if which is None else out
