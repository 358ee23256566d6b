"""Write the committed problem tables ``problems_<key>.json``.

Each problem is a start configuration, a goal configuration and the goal
pose [x, y, z, qw, qx, qy, qz] = FK(q_goal) (Sec. 3: start joint state and
a 7-d goal pose).  Start and goal are drawn uniformly inside the joint
limits and kept only when every collision sphere clears the scene's boxes
by at least 2 cm (exact box distance, not the grid).  The kinematics come
from the FP64 oracle only; values are stored as float32.

The cluttered workload's problem must exercise the collision term: its
start/goal pair is redrawn until the seed trajectories (the workload's own
seed recipe) bring at least 3 % of all sphere samples within the hinge's
activation distance of a box and at least one seed into a box.

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


# cluttered workload: fraction of hinge-active sphere samples the seeds
# must reach, and the hinge activation distance
ACTIVE_MIN = 0.03
EPS = 0.02


def seed_contact(rh, robot, scene, key, pidx, qs, qg, S, T):
    """(fraction of sphere samples of the seeds closer than EPS to a box,
    smallest clearance) for the seeds the workload draws for this pair."""
    prob = configs.Problem(0, qs, qg, np.zeros(7, dtype=np.float32), S, T)
    X = configs.seeds_for(key, pidx, prob).astype(np.float64)
    c = np.concatenate([oracle.sphere_centres(rh, X[s]) for s in range(S)])
    d = gen.scene_sdf(c, scene) - robot.sphere_radius.astype(np.float64)
    return float(np.mean(d < EPS)), float(d.min())


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
    for pidx, (sid, S, T) in enumerate(configs.problem_shapes(key)):
        sc = scenes[sid]
        for attempt in range(10000):
            qs = draw_config(rng, rh, robot, sc)
            qg = draw_config(rng, rh, robot, sc)
            if key != "B":
                break
            frac, dmin = seed_contact(rh, robot, sc, key, pidx, qs, qg, S, T)
            if frac >= ACTIVE_MIN and dmin < 0:
                print(f"{key}[{pidx}]: attempt {attempt}, hinge-active samples {frac:.3f}, "
                      f"deepest seed penetration {-dmin:.3f} m")
                break
        else:
            raise RuntimeError("no start/goal pair meets the contact rule")
        out.append({"scene": sid, "S": S, "T": T,
                    "q_start": [float(v) for v in qs],
                    "q_goal": [float(v) for v in qg],
                    "goal": [float(v) for v in goal_pose(rh, qg)]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"problems_{key}.json")
    with open(path, "w") as f:
        meta = {"workload": w.name, "written_by": "tests/golden/make_problems.py",
                "clearance_m": CLEARANCE}
        if key == "B":
            meta["seed_hinge_active_min"] = ACTIVE_MIN
        json.dump(dict(meta, problems=out), f, indent=0)
    print(path, len(out))


if __name__ == "__main__":
    for key in (sys.argv[1:] or ["A", "B", "C", "D", "E"]):
        write(key)
