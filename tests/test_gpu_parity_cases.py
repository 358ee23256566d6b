"""More GPU parity cases against the FP64 oracle, through the C ABI: joint
limits active (cost, gradient and optimiser), 16-lane groups and a long
horizon on a batched-workload problem, free running against the oracle's
own free run, trajectory metrics (App. A.7), seeds whose row 0 is not
q_start, non-finite seeds, and a grid too flat for the kernels' index
arithmetic.  Tolerances as in test_gpu_parity."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

from test_gpu_parity import (COST_RTOL, Setup, check_cost_grad, lockstep_check, say,  # noqa: E402
                             setup)

P = params.DEFAULT
U32 = 2.0 ** -24


def traced(su, seeds, tag):
    sd = torch.from_numpy(np.ascontiguousarray(seeds, dtype=np.float32)).cuda()
    tr = su.plan.optimize_traced({"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                                  "seeds": sd, "tag": tag})
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in tr.items()}


# ------------------------------------------------------------ joint limits --

@pytest.mark.parametrize("key", ["A", "B"])
def test_cost_grad_with_joints_outside_limits(key):
    """Trajectories with joints up to 3.4 rad (limits +-2.8): the limit
    penalty and its gradient are active on many elements."""
    su = setup(key, 1)
    X = gen.random_trajectories(np.random.default_rng(700), 16, 24, su.prob.q_start,
                                scale=3.4 / gen.Q_LIMIT)
    assert (np.abs(X[:, 1:]) > gen.Q_LIMIT).mean() > 0.1
    check_cost_grad(su, X)


def limit_seeds(su, S, T):
    """The workload's seeds with joints 2 and 4 pushed beyond the limits on
    the middle waypoints."""
    seeds = configs.seeds_for(su.key, 0, su.prob, S=S, T=T).astype(np.float64)
    bump = np.sin(np.linspace(0, np.pi, T))[None, :] * 0.9
    seeds[:, 1:, 1] += np.sign(seeds[:, 1:, 1] + 1e-3) * bump[:, 1:]
    seeds[:, 1:, 3] -= np.sign(seeds[:, 1:, 3] + 1e-3) * bump[:, 1:]
    seeds[:, 1:] = np.clip(seeds[:, 1:], -3.3, 3.3)
    return seeds.astype(np.float32)


@pytest.mark.parametrize("waves", [1, 8])
def test_lockstep_with_joints_outside_limits(waves):
    su = setup("B", 40, waves)
    seeds = limit_seeds(su, 8, 32)
    assert (np.abs(seeds) > gen.Q_LIMIT).any()
    say(f"lockstep, seeds outside the limits, W={waves}")
    tr = traced(su, seeds, 31)
    # the penalty is active at the start of the run
    assert (np.abs(tr["x"][0]) > gen.Q_LIMIT + 1e-3).any()
    lockstep_check(su, tr, seeds.shape[0])
    su.plan.release(31)


# --------------------------------------- batched-workload problem, T 12/40 --

class DSetup(Setup):
    """Problem 0 of the batched-uneven workload (its own 128^3 scene at
    1.5 cm, 5-30 random boxes)."""

    def __init__(self, iters, waves):
        super().__init__("D", iters, waves)


_d = {}


@pytest.mark.parametrize("T,waves", [(12, 1), (12, 8), (40, 1), (40, 8)])
def test_lockstep_batched_problem_horizons(T, waves):
    """T = 12 runs in 16-lane groups (four copies of the trajectory per
    wavefront split the spheres); T = 40 in one 64-lane group."""
    key = (waves,)
    if key not in _d:
        _d[key] = DSetup(100, waves)
    su = _d[key]
    seeds = configs.seeds_for("D", 0, su.prob, S=8, T=T)
    say(f"lockstep, batched-workload problem 0, T={T}, W={waves}")
    tr = traced(su, seeds, 40 + T)
    lockstep_check(su, tr, seeds.shape[0])
    su.plan.release(40 + T)


# ------------------------------------------------------------- free running --

@pytest.mark.parametrize("key,waves", [("A", 1), ("B", 1), ("B", 8)])
def test_free_run_matches_oracle_until_near_tie(key, waves):
    """The GPU's free run against the oracle's own free run from the same
    seeds.  A float32 run drifts from the FP64 one, so the comparison runs
    up to the first iteration at which either run's line-search decision is
    a near tie (margin below 1e-4 of the cost) or the two runs' costs differ
    by more than the cost tolerance (1e-4 relative: beyond it they follow
    different iterates).  Up to there every accepted step must be the same;
    seeds that reach the end that way must have the oracle's flags on its own
    final trajectory.  The point of divergence is reported."""
    su = setup(key, waves=waves)
    seeds = configs.seeds_for(key, 0, su.prob)
    S = seeds.shape[0]
    tr = traced(su, seeds, 51)
    res = su.plan.seed_results(51, S)
    Xo, otr = su.O.optimize(su.prob.q_start, su.prob.goal, seeds.astype(np.float64), su.iters,
                            trace=True)
    ref = su.O.results(su.prob.q_start, su.prob.goal, Xo)
    ends = []
    clean = 0
    for s in range(S):
        rep = su.O.lockstep(su.prob.q_start, su.prob.goal, tr["x"][:, s], tr["g"][:, s],
                            tr["J"][:, s], tr["d"][:, s], tr["alpha"][:, s])
        tie = (otr["margin"][:, s] / np.abs(otr["J"][:-1, s]) < 1e-4) | (rep[:, 5] < 1e-4)
        drift = np.abs(tr["J"][:-1, s] - otr["J"][:-1, s]) / np.abs(otr["J"][:-1, s]) > COST_RTOL
        stop = np.nonzero(tie | drift)[0]
        kstar = int(stop[0]) if stop.size else su.iters
        a_gpu, a_ref = tr["alpha"][:kstar, s], otr["alpha"][:kstar, s]
        assert np.array_equal(a_gpu, a_ref), (s, np.nonzero(a_gpu != a_ref)[0][:5], kstar)
        ends.append(kstar)
        if kstar == su.iters:
            clean += 1
            if abs(ref["clearance"][s]) < 1e-5:
                continue
            for f in ["collision_free", "within_limits", "success", "valid", "within_vel"]:
                assert res[f][s] == int(ref[f][s]), (s, f)
    ends = np.array(ends)
    say(f"free run {key} W={waves}: runs agree for {ends.min()}..{ends.max()} iterations "
        f"(median {int(np.median(ends))}), {clean}/{S} seeds to the end")
    assert ends.max() > 0
    su.plan.release(51)


# ------------------------------------------------------------------ metrics --

@pytest.mark.parametrize("key,waves", [("A", 1), ("B", 8)])
def test_trajectory_metrics_match_oracle(key, waves):
    """Max velocity, acceleration and jerk, motion time and the velocity
    flag (App. A.7) of every final trajectory against the oracle on the same
    trajectory.  The GPU forms differences of float32 waypoints: a k-th
    difference is exact to 2^k ulps of the largest |q| involved."""
    su = setup(key, waves=waves)
    seeds = configs.seeds_for(key, 0, su.prob)
    S = seeds.shape[0]
    tr = traced(su, seeds, 61)
    res = su.plan.seed_results(61, S)
    Xf = tr["x"][-1]
    ref = su.O.results(su.prob.q_start, su.prob.goal, Xf)
    dt = P["dt"]
    qmax = np.abs(Xf).max()
    for f, k in [("max_vel", 1), ("max_acc", 2), ("max_jerk", 3)]:
        tol = 4 * (2 ** k) * U32 * qmax / dt ** k + 1e-5 * np.abs(ref[f]).max()
        assert np.abs(res[f] - ref[f]).max() <= tol, (f, np.abs(res[f] - ref[f]).max(), tol)
    rel = np.abs(res["motion_time"] - ref["motion_time"]) / ref["motion_time"]
    assert rel.max() < 1e-4, rel.max()
    near = np.abs(ref["max_vel"] - P["v_limit"]) < 1e-4 * P["v_limit"]
    assert ((res["within_vel"] == ref["within_vel"].astype(int)) | near).all()
    _, best = su.plan.get_best(61, seeds.shape[1])
    b = best["best_seed"]
    assert best["max_vel"] == res["max_vel"][b] and best["motion_time"] == res["motion_time"][b]
    say(f"metrics {key}: max jerk {ref['max_jerk'].max():.1f} rad/s^3, motion time "
        f"{ref['motion_time'].min():.3f}..{ref['motion_time'].max():.3f} s")
    su.plan.release(61)


# --------------------------------------------------------- seed ingestion --

@pytest.mark.parametrize("waves", [1, 8])
def test_row0_is_replaced_by_q_start(waves):
    """Seeds whose row 0 differs from q_start: the optimiser pins waypoint 0
    to q_start, so the run equals (bitwise) the run from the same seeds with
    row 0 = q_start."""
    su = setup("A", waves=waves)
    good = configs.seeds_for("A", 0, su.prob)
    bad = good.copy()
    bad[:, 0, :] += np.float32(0.3)
    outs = []
    for i, sd in enumerate((good, bad)):
        out = torch.zeros(sd.shape, dtype=torch.float32, device="cuda")
        su.plan.optimize([{"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                           "seeds": torch.from_numpy(sd).cuda(), "tag": 71 + i, "out": out}])
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        su.plan.release(71 + i)
    assert np.array_equal(outs[1][:, 0, :], np.repeat(su.prob.q_start[None], good.shape[0], 0))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("waves", [1, 8])
def test_nonfinite_seed_is_invalid_and_isolated(waves):
    """A NaN in one seed makes that seed invalid (its cost is not finite)
    and leaves every other seed bitwise as in the run without it; the best
    seed is chosen among the valid ones."""
    su = setup("A", waves=waves)
    clean = configs.seeds_for("A", 0, su.prob)
    dirty = clean.copy()
    dirty[2, 5, 3] = np.nan
    outs, results = [], []
    for i, sd in enumerate((clean, dirty)):
        out = torch.zeros(sd.shape, dtype=torch.float32, device="cuda")
        say(f"non-finite seed run {i} W={waves}")
        su.plan.optimize([{"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                           "seeds": torch.from_numpy(sd).cuda(), "tag": 81 + i, "out": out}])
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        results.append((su.plan.seed_results(81 + i, sd.shape[0]), su.plan.get_best(81 + i, 32)[1]))
        su.plan.release(81 + i)
    keep = [s for s in range(clean.shape[0]) if s != 2]
    assert np.array_equal(outs[0][keep], outs[1][keep])
    r_clean, r_dirty = results[0][0], results[1][0]
    assert r_dirty["valid"][2] == 0 and r_dirty["success"][2] == 0
    assert np.all(r_dirty["valid"][keep] == r_clean["valid"][keep])
    best = results[1][1]
    assert best["best_seed"] != 2 and best["n_valid_seeds"] == clean.shape[0] - 1


# --------------------------------------------------------------- validation --

def test_grid_too_flat_for_24bit_indices_is_rejected():
    """(ny-1)(nz-1) >= 2^24 would overflow the kernels' 24-bit index
    products: the upload must fail with DS_ERR_INVALID (no sample is ever
    taken from such a grid)."""
    su = setup("A", 1)
    nx, ny, nz = 2, 4200, 4200
    vals = np.zeros(nx * ny * nz, dtype=np.float32)
    o = (C.c_float * 3)(0.0, 0.0, 0.0)
    rc = su.plan.lib.ds_esdf_upload(su.plan.h, 17, C.c_void_p(vals.ctypes.data), nx, ny, nz,
                                    C.c_float(0.01), o, None)
    assert rc == dsopt.DS_ERR_INVALID
    assert b"flat" in su.plan.lib.ds_last_error()
    # a grid just inside the bound is accepted
    ny2 = nz2 = 4096
    assert (ny2 - 1) * (nz2 - 1) < (1 << 24)
    small = np.zeros(2 * ny2 * nz2, dtype=np.float32)
    plan = dsopt.Plan(su.robot, P, 1, 2 << 30)
    rc = plan.lib.ds_esdf_upload(plan.h, 18, C.c_void_p(small.ctypes.data), 2, ny2, nz2,
                                 C.c_float(0.01), o, None)
    torch.cuda.synchronize()
    assert rc == dsopt.DS_OK
    plan.close()
