"""Thin ctypes binding of ``libdsopt.so`` (argument marshalling only).

Every step of the optimiser runs in the library's gfx950 kernels; torch is
used for device memory and streams.  Importing fails loudly when the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DSOPT_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("DSOPT_LIB") or os.path.join(HERE, "libdsopt.so")

DS_OK = 0
DS_ERR_INVALID = -1
DS_ERR_NOMEM = -2
DS_ERR_BUSY = -3
DS_ERR_NOT_FOUND = -4
DS_ERR_HIP = -5
DS_ERR_STATE = -6
MAX_T = 64
MIN_T = 4
MAX_SPHERES = 128

EXPORTED = [
    "ds_version", "ds_last_error", "ds_plan_create", "ds_plan_destroy", "ds_esdf_upload",
    "ds_esdf_release", "ds_esdf_from_occupancy", "ds_optimize_seeds", "ds_optimize_traced", "ds_get_best",
    "ds_get_seed_results", "ds_problem_release", "ds_cost", "ds_cost_grad",
    "ds_sphere_centres", "ds_guide", "ds_serve_start", "ds_serve_submit", "ds_serve_step", "ds_serve_poll",
    "ds_serve_stats", "ds_serve_stop", "ds_kernel_timing", "ds_kernel_timing_read",
    "ds_optimize_noalloc",
]
NOALLOC_MAX_SEEDS = 128


class DsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dsopt error {code}: {msg}")
        self.code = code


class Sphere(C.Structure):
    _fields_ = [("link", C.c_int32), ("offset", C.c_float * 3), ("radius", C.c_float)]


class Robot(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("n_spheres", C.c_int32),
                ("joint_frame", (C.c_float * 12) * 7), ("ee_frame", C.c_float * 12),
                ("q_lo", C.c_float * 7), ("q_hi", C.c_float * 7),
                ("spheres", C.POINTER(Sphere))]


class Params(C.Structure):
    _fields_ = [("w_collision", C.c_float), ("eps", C.c_float), ("lambda_v", C.c_float),
                ("lambda_a", C.c_float), ("lambda_j", C.c_float), ("w_pos", C.c_float),
                ("w_rot", C.c_float), ("w_limit", C.c_float), ("history", C.c_int32),
                ("n_ls", C.c_int32), ("c1", C.c_float), ("delta0", C.c_float),
                ("step_max", C.c_float), ("dt", C.c_float), ("tol_pos", C.c_float),
                ("tol_rot", C.c_float), ("n_iters", C.c_int32), ("block_iters", C.c_int32),
                ("waves_per_seed", C.c_int32), ("w_self", C.c_float),
                ("swept_samples", C.c_int32), ("exact_gathers", C.c_int32),
                ("serve_drain", C.c_int32), ("v_limit", C.c_float), ("a_limit", C.c_float),
                ("j_limit", C.c_float)]


class Problem(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("n_seeds", C.c_int32), ("horizon", C.c_int32),
                ("problem_tag", C.c_int32), ("q_start", C.c_float * 7), ("goal", C.c_float * 7),
                ("seeds", C.c_void_p), ("out_traj", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("best_seed", C.c_int32), ("success", C.c_int32), ("collision_free", C.c_int32),
                ("n_valid_seeds", C.c_int32), ("pos_err_m", C.c_float),
                ("rot_err_rad", C.c_float), ("cost", C.c_float), ("min_clearance_m", C.c_float),
                ("max_jerk", C.c_float), ("n_iters", C.c_int32), ("max_vel", C.c_float),
                ("motion_time", C.c_float)]


class SeedResult(C.Structure):
    _fields_ = [("cost", C.c_float), ("clearance", C.c_float), ("pos_err", C.c_float),
                ("rot_err", C.c_float), ("max_jerk", C.c_float), ("collision_free", C.c_int32),
                ("within_limits", C.c_int32), ("success", C.c_int32), ("valid", C.c_int32),
                ("n_evals_cost", C.c_int32), ("n_evals_grad", C.c_int32), ("n_gathers", C.c_uint32),
                ("max_vel", C.c_float), ("max_acc", C.c_float), ("motion_time", C.c_float),
                ("within_vel", C.c_int32)]


class LatencyStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("problems_per_s", C.c_double),
                ("steps", C.c_int64), ("mean_active_slots", C.c_double)]


_lib = None


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2410_16727_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, f32p = C.c_void_p, C.c_int32, C.c_void_p
    L.ds_version.restype = C.c_int
    L.ds_last_error.restype = C.c_char_p
    L.ds_plan_create.argtypes = [C.POINTER(Robot), C.POINTER(Params), vp, C.c_size_t,
                                 C.POINTER(vp)]
    L.ds_plan_destroy.argtypes = [vp]
    L.ds_plan_destroy.restype = None
    L.ds_esdf_upload.argtypes = [vp, i32, vp, C.c_int, C.c_int, C.c_int, C.c_float,
                                 C.POINTER(C.c_float), vp]
    L.ds_esdf_release.argtypes = [vp, i32]
    L.ds_esdf_from_occupancy.argtypes = [vp, i32, vp, C.c_int, C.c_int, C.c_int, C.c_float,
                                         C.POINTER(C.c_float), vp, vp]
    L.ds_optimize_seeds.argtypes = [vp, C.POINTER(Problem), C.c_int, vp]
    L.ds_optimize_traced.argtypes = [vp, C.POINTER(Problem), f32p, f32p, f32p, f32p, f32p, vp]
    L.ds_get_best.argtypes = [vp, i32, vp, C.POINTER(Result)]
    L.ds_get_seed_results.argtypes = [vp, i32, C.POINTER(SeedResult), C.c_int]
    L.ds_problem_release.argtypes = [vp, i32]
    L.ds_cost.argtypes = [vp, C.POINTER(Problem), f32p, C.c_int, C.c_int, f32p, vp]
    L.ds_cost_grad.argtypes = [vp, C.POINTER(Problem), f32p, C.c_int, C.c_int, f32p, f32p, f32p,
                               vp]
    L.ds_sphere_centres.argtypes = [vp, f32p, C.c_int, C.c_int, f32p, vp]
    L.ds_guide.argtypes = [vp, C.POINTER(Problem), f32p, C.c_int, C.c_int, C.c_float, C.c_int,
                           f32p, vp]
    L.ds_kernel_timing.argtypes = [vp, C.c_int]
    L.ds_kernel_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.ds_optimize_noalloc.argtypes = [vp, C.POINTER(Problem), vp, vp, vp, vp]
    L.ds_serve_start.argtypes = [vp, C.c_int, C.c_int, vp]
    L.ds_serve_submit.argtypes = [vp, C.POINTER(Problem), C.POINTER(C.c_uint64)]
    L.ds_serve_step.argtypes = [vp]
    L.ds_serve_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result), vp]
    L.ds_serve_stats.argtypes = [vp, C.POINTER(LatencyStats)]
    L.ds_serve_stop.argtypes = [vp]
    _lib = L
    return L


def check(rc):
    if rc < 0:
        raise DsError(rc, load().ds_last_error().decode())
    return rc


def _struct_dict(s):
    return {k: getattr(s, k) for k, _ in s._fields_}


def robot_struct(robot):
    """ctypes robot from arrays (frames [8,12], q_lo, q_hi, sphere_link,
    sphere_offset [N,3], sphere_radius)."""
    ns = int(robot.sphere_link.shape[0])
    sph = (Sphere * ns)()
    for s in range(ns):
        sph[s].link = int(robot.sphere_link[s])
        for a in range(3):
            sph[s].offset[a] = float(robot.sphere_offset[s, a])
        sph[s].radius = float(robot.sphere_radius[s])
    r = Robot()
    r.n_joints = 7
    r.n_spheres = ns
    fr = np.asarray(robot.frames, dtype=np.float32)
    for i in range(7):
        for k in range(12):
            r.joint_frame[i][k] = float(fr[i, k])
    for k in range(12):
        r.ee_frame[k] = float(fr[7, k])
    for j in range(7):
        r.q_lo[j] = float(robot.q_lo[j])
        r.q_hi[j] = float(robot.q_hi[j])
    r.spheres = C.cast(sph, C.POINTER(Sphere))
    return r, sph


def params_struct(p: dict, n_iters: int, block_iters: int = 10):
    s = Params()
    s.w_collision = p["w_collision"]; s.eps = p["eps"]
    s.lambda_v = p["lambda_v"]; s.lambda_a = p["lambda_a"]; s.lambda_j = p["lambda_j"]
    s.w_pos = p["w_pos"]; s.w_rot = p["w_rot"]; s.w_limit = p["w_limit"]
    s.history = int(p["history"]); s.n_ls = int(p["n_ls"])
    s.c1 = p["c1"]; s.delta0 = p["delta0"]; s.step_max = p["step_max"]; s.dt = p["dt"]
    s.tol_pos = p["tol_pos"]; s.tol_rot = p["tol_rot"]
    s.n_iters = int(n_iters); s.block_iters = int(block_iters)
    s.waves_per_seed = int(p.get("waves_per_seed", 1))
    s.w_self = float(p.get("w_self", 0.0))
    s.swept_samples = int(p.get("swept_samples", 0))
    s.exact_gathers = int(p.get("exact_gathers", 0))
    s.serve_drain = int(p.get("serve_drain", 0))
    s.v_limit = float(p.get("v_limit", 2.5))
    s.a_limit = float(p.get("a_limit", 10.0))
    s.j_limit = float(p.get("j_limit", 5000.0))
    return s


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def problem_struct(scene_id, q_start, goal, tag=0, seeds=None, out_traj=None, S=0, T=0):
    p = Problem()
    p.scene_id = int(scene_id)
    p.problem_tag = int(tag)
    p.n_seeds = int(S)
    p.horizon = int(T)
    for j in range(7):
        p.q_start[j] = float(q_start[j])
        p.goal[j] = float(goal[j])
    p.seeds = None if seeds is None else seeds.data_ptr()
    p.out_traj = None if out_traj is None else out_traj.data_ptr()
    return p


class Plan:
    """A plan over a torch-allocated device arena."""

    def __init__(self, robot, params: dict, n_iters: int, arena_bytes: int,
                 block_iters: int = 10, device: str = "cuda"):
        import torch
        self.lib = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self._robot, self._sph = robot_struct(robot)
        self._params = params_struct(params, n_iters, block_iters)
        h = C.c_void_p()
        check(self.lib.ds_plan_create(C.byref(self._robot), C.byref(self._params),
                                      C.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                      C.byref(h)))
        self.h = h
        self.n_spheres = int(robot.sphere_link.shape[0])
        self.n_iters = n_iters
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.ds_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scenes --------------------------------------------------------------
    def upload_scene(self, scene_id, grid, voxel, origin, stream=None):
        """grid: [nz, ny, nx] float32 (numpy host array or torch tensor)."""
        import torch
        if isinstance(grid, np.ndarray):
            src = torch.from_numpy(np.ascontiguousarray(grid, dtype=np.float32))
            nz, ny, nx = grid.shape
        else:
            src = grid.contiguous()
            nz, ny, nx = src.shape
        o = (C.c_float * 3)(*[float(v) for v in origin])
        check(self.lib.ds_esdf_upload(self.h, int(scene_id), C.c_void_p(src.data_ptr()), nx, ny,
                                      nz, float(voxel), o, _stream(stream)))
        if src.device.type == "cuda":
            self._keep[("scene", scene_id)] = src

    def scene_from_occupancy(self, scene_id, occ, voxel, origin, out=None, stream=None):
        """occ: [nz, ny, nx] uint8/bool (numpy host array or torch tensor);
        out: optional cuda float tensor [nz, ny, nx] receiving the signed
        distances."""
        import torch
        if isinstance(occ, np.ndarray):
            src = torch.from_numpy(np.ascontiguousarray(occ, dtype=np.uint8))
        else:
            src = occ.to(torch.uint8).contiguous()
        nz, ny, nx = src.shape
        o = (C.c_float * 3)(*[float(v) for v in origin])
        check(self.lib.ds_esdf_from_occupancy(self.h, int(scene_id), C.c_void_p(src.data_ptr()),
                                              nx, ny, nz, float(voxel), o, _ptr(out),
                                              _stream(stream)))
        if src.device.type == "cuda":
            self._keep[("occ", scene_id)] = src

    def release_scene(self, scene_id):
        check(self.lib.ds_esdf_release(self.h, int(scene_id)))

    # -- optimisation ----------------------------------------------------------
    def optimize(self, problems, stream=None):
        """problems: list of dicts(scene, q_start, goal, seeds [S,T,7] cuda
        tensor, tag, out (optional cuda tensor))."""
        arr = (Problem * len(problems))()
        for i, p in enumerate(problems):
            S, T, _ = p["seeds"].shape
            arr[i] = problem_struct(p["scene"], p["q_start"], p["goal"], p["tag"], p["seeds"],
                                    p.get("out"), S, T)
        check(self.lib.ds_optimize_seeds(self.h, arr, len(problems), _stream(stream)))

    def optimize_noalloc(self, p, seed_results, result, best_traj, stream=None):
        """The allocation-free call: p as for optimize (seeds, optional
        out); seed_results (uint8 cuda tensor of S * sizeof(SeedResult)
        bytes), result (uint8 cuda tensor of sizeof(Result) bytes) and
        best_traj (float cuda tensor [T, 7]) receive the results."""
        S, T, _ = p["seeds"].shape
        pr = problem_struct(p["scene"], p["q_start"], p["goal"], p.get("tag", 0), p["seeds"],
                            p.get("out"), S, T)
        check(self.lib.ds_optimize_noalloc(self.h, C.byref(pr), _ptr(seed_results), _ptr(result),
                                           _ptr(best_traj), _stream(stream)))

    def optimize_traced(self, p, stream=None):
        import torch
        S, T, _ = p["seeds"].shape
        N = self.n_iters
        dev = p["seeds"].device
        tr = {"x": torch.zeros((N + 1, S, T, 7), dtype=torch.float32, device=dev),
              "g": torch.zeros((N + 1, S, T, 7), dtype=torch.float32, device=dev),
              "J": torch.zeros((N + 1, S), dtype=torch.float32, device=dev),
              "d": torch.zeros((max(N, 1), S, T, 7), dtype=torch.float32, device=dev),
              "alpha": torch.zeros((max(N, 1), S), dtype=torch.float32, device=dev)}
        pr = problem_struct(p["scene"], p["q_start"], p["goal"], p["tag"], p["seeds"],
                            p.get("out"), S, T)
        check(self.lib.ds_optimize_traced(self.h, C.byref(pr), _ptr(tr["x"]), _ptr(tr["g"]),
                                          _ptr(tr["J"]), _ptr(tr["d"]), _ptr(tr["alpha"]),
                                          _stream(stream)))
        return tr

    def get_best(self, tag, T):
        traj = np.zeros((T, 7), dtype=np.float32)
        r = Result()
        check(self.lib.ds_get_best(self.h, int(tag), traj.ctypes.data_as(C.c_void_p),
                                   C.byref(r)))
        return traj, _struct_dict(r)

    def seed_results(self, tag, S):
        arr = (SeedResult * S)()
        check(self.lib.ds_get_seed_results(self.h, int(tag), arr, S))
        out = {k: np.array([getattr(a, k) for a in arr]) for k, _ in SeedResult._fields_
               if k != "pad"}
        return out

    def release(self, tag):
        check(self.lib.ds_problem_release(self.h, int(tag)))

    # -- objective / gradient ----------------------------------------------------
    def cost(self, scene, q_start, goal, X, stream=None):
        import torch
        S, T, _ = X.shape
        J = torch.empty(S, dtype=torch.float32, device=X.device)
        pr = problem_struct(scene, q_start, goal)
        check(self.lib.ds_cost(self.h, C.byref(pr), _ptr(X), S, T, _ptr(J), _stream(stream)))
        return J

    def cost_grad(self, scene, q_start, goal, X, dJ=None, stream=None):
        import torch
        S, T, _ = X.shape
        J = torch.empty(S, dtype=torch.float32, device=X.device)
        dX = torch.empty_like(X)   # every element is written (row 0 as zero)
        pr = problem_struct(scene, q_start, goal)
        check(self.lib.ds_cost_grad(self.h, C.byref(pr), _ptr(X), S, T, _ptr(dJ), _ptr(J),
                                    _ptr(dX), _stream(stream)))
        return J, dX

    def guide(self, scene, q_start, goal, X, alpha, n_steps, stream=None):
        """In place: n_steps steps X <- X - alpha * dJ/dX; returns J after."""
        import torch
        S, T, _ = X.shape
        J = torch.empty(S, dtype=torch.float32, device=X.device)
        pr = problem_struct(scene, q_start, goal)
        check(self.lib.ds_guide(self.h, C.byref(pr), _ptr(X), S, T, float(alpha), int(n_steps),
                                _ptr(J), _stream(stream)))
        return J

    def sphere_centres(self, X, stream=None):
        import torch
        S, T, _ = X.shape
        out = torch.empty((S, T, self.n_spheres, 3), dtype=torch.float32, device=X.device)
        check(self.lib.ds_sphere_centres(self.h, _ptr(X), S, T, _ptr(out), _stream(stream)))
        return out

    # -- measurement ------------------------------------------------------------------
    def kernel_timing(self, enable=True):
        check(self.lib.ds_kernel_timing(self.h, 1 if enable else 0))

    def kernel_timing_read(self):
        ms = C.c_double()
        n = C.c_int64()
        check(self.lib.ds_kernel_timing_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # -- serving ---------------------------------------------------------------------
    def serve_start(self, max_slots, queue_cap, stream=None):
        check(self.lib.ds_serve_start(self.h, int(max_slots), int(queue_cap), _stream(stream)))

    def serve_submit(self, p):
        S, T, _ = p["seeds"].shape
        pr = problem_struct(p["scene"], p["q_start"], p["goal"], p.get("tag", 0), p["seeds"],
                            p.get("out"), S, T)
        t = C.c_uint64()
        check(self.lib.ds_serve_submit(self.h, C.byref(pr), C.byref(t)))
        return t.value

    def serve_step(self):
        return check(self.lib.ds_serve_step(self.h))

    def serve_poll(self, ticket, T=None):
        r = Result()
        traj = np.zeros((T, 7), dtype=np.float32) if T else None
        rc = self.lib.ds_serve_poll(self.h, C.c_uint64(ticket), C.byref(r),
                                    None if traj is None else traj.ctypes.data_as(C.c_void_p))
        if rc == DS_ERR_STATE:
            return None
        check(rc)
        return (traj, _struct_dict(r))

    def serve_stats(self):
        s = LatencyStats()
        check(self.lib.ds_serve_stats(self.h, C.byref(s)))
        return _struct_dict(s)

    def serve_stop(self):
        check(self.lib.ds_serve_stop(self.h))
