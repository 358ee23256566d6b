"""Write the committed problem tables ``problems_<key>.json``.

Each problem is a start configuration, a goal configuration and the goal
pose [x, y, z, qw, qx, qy, qz] = FK(q_goal) (Sec. 3: start joint state and
a 7-d goal pose).  Start and goal are drawn uniformly inside the joint
limits and kept only when every collision sphere clears the scene's boxes
by at least 2 cm (exact box distance, not the grid).  The kinematics come
from the FP64 oracle only; values are stored as float32.

Run:  python tests/golden/make_problems.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs, gen  # noqa: E402

CLEARANCE = 0.02


def collision_free(rh, robot, scene, q):
    c = oracle.sphere_centres(rh, np.asarray(q, dtype=np.float64)[None])[0]
    d = gen.scene_sdf(c, scene) - robot.sphere_radius.astype(np.float64)
    return bool(np.all(d >= CLEARANCE))


def draw_config(rng, rh, robot, scene):
    for _ in range(100000):
        q = rng.uniform(-gen.Q_LIMIT, gen.Q_LIMIT, size=7).astype(np.float32)
        if collision_free(rh, robot, scene, q):
            return q
    raise RuntimeError("no collision-free configuration found")


def goal_pose(rh, q):
    R, p = oracle.fk_frames(rh, np.asarray(q, dtype=np.float64))
    quat = oracle.R_to_quat(R[7])
    return np.concatenate([p[7], quat]).astype(np.float32)


def write(key):
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    rh = oracle.RobotH(robot)
    scenes = configs.scenes(key, build=False)
    rng = gen.rng_for(w.index, 6)
    out = []
    for (sid, S, T) in configs.problem_shapes(key):
        sc = scenes[sid]
        qs = draw_config(rng, rh, robot, sc)
        qg = draw_config(rng, rh, robot, sc)
        out.append({"scene": sid, "S": S, "T": T,
                    "q_start": [float(v) for v in qs],
                    "q_goal": [float(v) for v in qg],
                    "goal": [float(v) for v in goal_pose(rh, qg)]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"problems_{key}.json")
    with open(path, "w") as f:
        json.dump({"workload": w.name, "written_by": "tests/golden/make_problems.py",
                   "clearance_m": CLEARANCE, "problems": out}, f, indent=0)
    print(path, len(out))


if __name__ == "__main__":
    for key in (sys.argv[1:] or ["A", "B", "C", "D", "E"]):
        write(key)
