"""Optimiser hyper-parameters handed identically to the oracle and to the
GPU library.  The paper states none of these (App. A.6 names the cost
terms only); every value is a reading recorded in the design notes."""
import math

DEFAULT = {
    "w_collision": 100.0,      # C_world weight
    "eps": 0.02,               # hinge activation distance [m]
    "lambda_v": 1.0,           # velocity, acceleration, jerk weights (dt folded in)
    "lambda_a": 10.0,
    "lambda_j": 10.0,
    "w_pos": 1000.0,           # goal position weight
    "w_rot": 100.0,            # goal rotation weight
    "w_limit": 100.0,          # joint-limit penalty weight
    "history": 8,              # L-BFGS memory m
    "n_ls": 4,                 # line-search candidates alpha = 1, 1/2, 1/4, 1/8
    "c1": 1e-4,                # Armijo constant
    "delta0": 0.05,            # steepest-descent step (inf-norm) [rad]
    "step_max": 0.3,           # inf-norm cap of a direction [rad]
    "dt": 0.04,                # waypoint spacing for jerk reporting [s]
    "tol_pos": 0.005,          # success threshold delta_t [m] (Sec. 5.1)
    "tol_rot": 2.86 * math.pi / 180.0,   # success threshold delta_r [rad]
    "w_self": 0.0,             # self-collision weight (0: term off)
    "swept_samples": 0,        # interpolated configurations per segment (0: waypoints only)
    "v_limit": 2.5,            # joint velocity limit [rad/s] (motion-time metric)
    "a_limit": 10.0,           # joint acceleration limit [rad/s^2]
    "j_limit": 5000.0,         # joint jerk limit [rad/s^3]
}

ORDER = ["w_collision", "eps", "lambda_v", "lambda_a", "lambda_j", "w_pos", "w_rot",
         "w_limit", "history", "n_ls", "c1", "delta0", "step_max", "dt", "tol_pos", "tol_rot",
         "w_self", "swept_samples", "v_limit", "a_limit", "j_limit"]


def as_list(p=None):
    p = dict(DEFAULT, **(p or {}))
    return [float(p[k]) for k in ORDER]
