"""Maximum sizes against the oracle: a robot with the largest sphere table
(128 spheres, 19 on one link, so even 8-wavefront teams take the chunked
evaluation form), the longest and shortest horizons, a single seed, and a
129-seed problem run by 8-wavefront teams."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

from test_gpu_parity import AMB_TOL, COST_RTOL, GRAD_RTOL, grad_check, lockstep_check  # noqa: E402

PER_LINK = [19, 19, 18, 18, 18, 18, 18]   # 128 spheres


def big_robot():
    return gen.make_robot(np.random.default_rng(7), np.random.default_rng(8), PER_LINK)


class Big:
    def __init__(self, iters, waves):
        self.key = "B"
        self.robot = big_robot()
        assert self.robot.n_spheres == 128
        self.scene = configs.scenes("B", only={0})[0]
        self.prob = configs.problems("B")[0]
        self.iters = iters
        self.plan = dsopt.Plan(self.robot, dict(params.DEFAULT, waves_per_seed=waves), iters,
                               512 << 20)
        self.plan.upload_scene(0, self.scene.grid, self.scene.voxel, self.scene.origin)
        self.O = oracle.Oracle(self.robot, self.scene, params.as_list(), threads=8)


@pytest.mark.parametrize("T", [64, 4])
def test_max_spheres_cost_grad(T):
    su = Big(1, 1)
    print(f"128 spheres cost/grad T={T}", flush=True)
    X = gen.random_trajectories(np.random.default_rng(T), 6, T, su.prob.q_start)
    ref = su.O.cost(su.prob.q_start, su.prob.goal, X.astype(np.float64), grad=True, absg=True)
    J, G = su.plan.cost_grad(0, su.prob.q_start, su.prob.goal, torch.from_numpy(X).cuda())
    J, G = J.cpu().numpy(), G.cpu().numpy()
    assert (np.abs(J - ref["J"]) / ref["J"]).max() < COST_RTOL
    for s in range(X.shape[0]):
        worst, need = grad_check(su.O, su.prob, X[s], G[s], ref["G"][s], ref["A"][s])
        assert worst <= GRAD_RTOL, (s, worst, need)
    c = su.plan.sphere_centres(torch.from_numpy(X).cuda()).cpu().numpy()
    for s in range(X.shape[0]):
        assert np.abs(c[s] - su.O.spheres(X[s].astype(np.float64))).max() < 1e-5
    su.plan.close()


@pytest.mark.parametrize("waves", [8, 1])
def test_max_spheres_lockstep(waves):
    su = Big(12, waves)
    seeds = configs.seeds_for("B", 0, su.prob, S=4, T=64)
    print(f"128 spheres lockstep W={waves}", flush=True)
    tr = su.plan.optimize_traced({"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                                  "seeds": torch.from_numpy(seeds).cuda(), "tag": 2})
    torch.cuda.synchronize()
    tr = {k: v.double().cpu().numpy() for k, v in tr.items()}
    lockstep_check(su, tr, seeds.shape[0])
    su.plan.close()


def test_single_seed_and_many_teams():
    """S = 1 (one tile) and S = 129 with 8-wavefront teams: every seed's
    result equals its result in a run of its own (per-seed arithmetic does
    not depend on the batch)."""
    robot = configs.robot("B")
    sc = configs.scenes("B", only={0})[0]
    prob = configs.problems("B")[0]
    plan = dsopt.Plan(robot, dict(params.DEFAULT, waves_per_seed=8), 6, 1 << 30)
    plan.upload_scene(0, sc.grid, sc.voxel, sc.origin)
    seeds = torch.from_numpy(configs.seeds_for("B", 0, prob, S=129, T=32)).cuda()
    out_all = torch.zeros_like(seeds)
    plan.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": seeds,
                    "tag": 1, "out": out_all}])
    for s in (0, 77, 128):
        one = torch.zeros_like(seeds[s:s + 1])
        plan.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal,
                        "seeds": seeds[s:s + 1].contiguous(), "tag": 10 + s, "out": one}])
        torch.cuda.synchronize()
        assert torch.equal(one[0], out_all[s]), s
        plan.release(10 + s)
    plan.release(1)
    plan.close()
