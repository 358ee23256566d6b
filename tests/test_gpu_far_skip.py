"""The coarse-table skip is exact: with and without it the library returns
the same bits (costs, gradients, every iterate, flags), because a skipped
sample's hinge and gradient are exactly zero.  With every sample gathered,
each seed's gather counter equals evaluations x horizon x spheres."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402


def say(*a):
    print(*a, flush=True)


def plans(key, iters, waves, scene_idx=0):
    robot = configs.robot(key)
    sc = configs.scenes(key, only={scene_idx})[scene_idx]
    out = []
    for exact in (0, 1):
        pl = dsopt.Plan(robot, dict(params.DEFAULT, waves_per_seed=waves, exact_gathers=exact),
                        iters, 512 << 20)
        pl.upload_scene(0, sc.grid, sc.voxel, sc.origin)
        out.append(pl)
    return robot, sc, out


@pytest.mark.parametrize("key,T", [("A", 16), ("B", 32), ("B", 57), ("D", 40)])
def test_cost_grad_identical(key, T):
    prob = configs.problems(key)[0]
    robot, sc, (fast, exact) = plans(key, 1, 1, prob.scene)
    say(f"skip vs exact cost/grad {key} T={T}")
    X = torch.from_numpy(gen.random_trajectories(np.random.default_rng(T), 16, T,
                                                 prob.q_start, scale=0.6)).cuda()
    Ja, Ga = fast.cost_grad(0, prob.q_start, prob.goal, X)
    Jb, Gb = exact.cost_grad(0, prob.q_start, prob.goal, X)
    assert torch.equal(Ja, Jb) and torch.equal(Ga, Gb)
    fast.close()
    exact.close()


@pytest.mark.parametrize("key,waves", [("B", 8), ("B", 1), ("A", 1), ("D", 1)])
def test_optimisation_identical_and_gathers_counted(key, waves):
    prob = configs.problems(key)[0]
    robot, sc, (fast, exact) = plans(key, configs.WORKLOADS[key].iters, waves, prob.scene)
    seeds = torch.from_numpy(configs.seeds_for(key, 0, prob)).cuda()
    S, T = seeds.shape[0], seeds.shape[1]
    say(f"skip vs exact optimisation {key} W={waves} S={S} T={T}")
    traces, res = [], []
    for pl in (fast, exact):
        tr = pl.optimize_traced({"scene": 0, "q_start": prob.q_start, "goal": prob.goal,
                                 "seeds": seeds, "tag": 5})
        torch.cuda.synchronize()
        traces.append({k: v.cpu().numpy() for k, v in tr.items()})
        res.append(pl.seed_results(5, S))
        pl.release(5)
    for k in traces[0]:
        assert np.array_equal(traces[0][k], traces[1][k]), k
    for f in ["cost", "clearance", "collision_free", "success", "n_evals_cost", "n_evals_grad"]:
        assert np.array_equal(res[0][f], res[1][f]), f
    evals = res[1]["n_evals_grad"] + res[1]["n_evals_cost"] + 1
    ns = len(robot.sphere_radius)
    assert np.array_equal(res[1]["n_gathers"], evals * T * ns)
    assert np.all(res[0]["n_gathers"] <= res[1]["n_gathers"])
    say(f"gathered with the coarse table: {res[0]['n_gathers'].sum() / res[1]['n_gathers'].sum():.3f}")
    fast.close()
    exact.close()
