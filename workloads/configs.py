"""The five synthetic workloads (tiny, cluttered, differentiation,
batched-uneven, serving) and their recipes.

Everything here is seeded; every array handed to the optimizer is float32.
Start/goal configurations and goal poses are not drawn here: they need the
arm's kinematics, so they live in the committed problem tables under
``tests/golden`` (written by ``tests/golden/make_problems.py``), which this
module only reads.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

from . import gen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(os.path.dirname(HERE), "tests", "golden")

ARM_STREAM = (0, 0)          # one arm (link lengths) shared by all workloads


@dataclass
class Workload:
    name: str
    index: int
    spheres_per_link: tuple
    scene_kind: str              # "random" | "shelf"
    n_scenes: int
    boxes: tuple                 # (lo, hi) inclusive box count
    dims: tuple
    voxel: float
    origin: tuple
    iters: int


WORKLOADS = {
    "A": Workload("tiny", 0, (4,) * 7, "random", 1, (3, 3), (64, 64, 64), 0.02,
                  (-0.64, -0.64, -0.32), 25),
    "B": Workload("cluttered", 1, (8,) * 7, "shelf", 1, (20, 20), (200, 200, 200), 0.01,
                  (-1.0, -1.0, -0.5), 100),
    "C": Workload("differentiation", 2, (9, 9, 9, 9, 8, 8, 8), "shelf", 1, (20, 20),
                  (200, 200, 200), 0.01, (-1.0, -1.0, -0.5), 100),
    "D": Workload("batched-uneven", 3, (8,) * 7, "random", 64, (5, 30), (128, 128, 128),
                  0.015, (-0.96, -0.96, -0.48), 100),
    "E": Workload("serving", 4, (8,) * 7, "shelf", 16, (20, 20), (200, 200, 200), 0.01,
                  (-1.0, -1.0, -0.5), 100),
}


def robot(key: str) -> gen.Robot:
    w = WORKLOADS[key]
    return gen.make_robot(gen.rng_for(*ARM_STREAM), gen.rng_for(w.index, 1),
                          w.spheres_per_link)


def scenes(key: str, build: bool = True, only=None, threads: int = 8):
    """Scene list for a workload; ``only`` restricts to some scene ids
    (other entries are None).  Grids are built when ``build``."""
    w = WORKLOADS[key]
    out = []
    for sid in range(w.n_scenes):
        if only is not None and sid not in only:
            out.append(None)
            continue
        rng = gen.rng_for(w.index, 2, sid)
        nb = int(rng.integers(w.boxes[0], w.boxes[1] + 1))
        if w.scene_kind == "shelf":
            sc = gen.shelf_scene(rng, nb, w.dims, w.voxel, w.origin)
        else:
            sc = gen.random_box_scene(rng, nb, w.dims, w.voxel, w.origin)
        out.append(sc)
    if build:
        gen.build_grids([s for s in out if s is not None], threads=threads)
    return out


@dataclass
class Problem:
    scene: int
    q_start: np.ndarray          # [7] float32
    q_goal: np.ndarray           # [7] float32 (seed recipe only)
    goal: np.ndarray             # [7] float32: x, y, z, qw, qx, qy, qz
    S: int
    T: int


def problem_table(key: str):
    path = os.path.join(GOLDEN, f"problems_{key}.json")
    with open(path) as f:
        return json.load(f)


def problems(key: str):
    tab = problem_table(key)
    out = []
    for p in tab["problems"]:
        out.append(Problem(int(p["scene"]), np.array(p["q_start"], dtype=np.float32),
                           np.array(p["q_goal"], dtype=np.float32),
                           np.array(p["goal"], dtype=np.float32), int(p["S"]), int(p["T"])))
    return out


def seeds_for(key: str, pidx: int, prob: Problem, S=None, T=None, stream=0) -> np.ndarray:
    rng = gen.rng_for(WORKLOADS[key].index, 3, pidx, stream)
    return gen.interp_seeds(rng, prob.q_start, prob.q_goal, S or prob.S, T or prob.T)


# The shape of each workload's problem set (used when writing the tables).
def problem_shapes(key: str):
    w = WORKLOADS[key]
    if key == "A":
        return [(0, 4, 32)]
    if key == "B":
        return [(0, 32, 32)]
    if key == "C":
        return [(0, 256, 64)]
    if key == "D":
        rng = gen.rng_for(w.index, 4)
        return [(i, int(rng.integers(4, 129)), int(rng.integers(16, 65))) for i in range(64)]
    if key == "E":
        # a pool of 8 problems per scene; the request trace picks from it
        return [(sid, 0, 0) for sid in range(16) for _ in range(8)]
    raise KeyError(key)


def serving_trace(n_requests=2200, rate_hz=200.0):
    """Poisson arrivals of mixed requests: (arrival_s, pool index, S, T)."""
    w = WORKLOADS["E"]
    rng = gen.rng_for(w.index, 5)
    arr = gen.poisson_arrivals(rng, n_requests, rate_hz)
    pool = rng.integers(0, 128, size=n_requests)
    S = rng.integers(8, 129, size=n_requests)
    T = rng.integers(32, 65, size=n_requests)
    return [(float(a), int(p), int(s), int(t)) for a, p, s, t in zip(arr, pool, S, T)]
