"""GPU parity of the optional self-collision term (C_self of App. A.6)
against the FP64 oracle: cost/gradient on trajectories with self-contact,
a lockstep optimisation, and flags including self-clearance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

from test_gpu_parity import (AMB_TOL, COST_RTOL, GRAD_RTOL, grad_check,  # noqa: E402
                             guidance_lockstep, lockstep_check)

PS = dict(params.DEFAULT, w_self=50.0)


def fat(key):
    rb = configs.robot(key)
    return gen.Robot(rb.link_lengths, rb.frames, rb.q_lo, rb.q_hi, rb.sphere_link,
                     rb.sphere_offset, (rb.sphere_radius * 1.6).astype(np.float32))


class SelfSetup:
    def __init__(self, key, iters, waves):
        self.key = key
        self.robot = fat(key)
        self.scene = configs.scenes(key, only={0})[0]
        self.prob = configs.problems(key)[0]
        self.iters = iters
        self.plan = dsopt.Plan(self.robot, dict(PS, waves_per_seed=waves), iters, 512 << 20)
        self.plan.upload_scene(0, self.scene.grid, self.scene.voxel, self.scene.origin)
        self.O = oracle.Oracle(self.robot, self.scene, params.as_list(PS), threads=8)


@pytest.mark.parametrize("key,T", [("B", 32), ("A", 16), ("B", 64)])
def test_self_cost_grad_parity(key, T):
    su = SelfSetup(key, 1, 1)
    X = gen.random_trajectories(np.random.default_rng(T), 8, T, su.prob.q_start)
    ref = su.O.cost(su.prob.q_start, su.prob.goal, X.astype(np.float64), grad=True, absg=True,
                    terms=True)
    assert np.all(ref["terms"][:, 7] > 0)
    J, G = su.plan.cost_grad(0, su.prob.q_start, su.prob.goal, torch.from_numpy(X).cuda())
    J, G = J.cpu().numpy(), G.cpu().numpy()
    assert (np.abs(J - ref["J"]) / ref["J"]).max() < COST_RTOL
    for s in range(X.shape[0]):
        worst, need = grad_check(su.O, su.prob, X[s], G[s], ref["G"][s], ref["A"][s])
        assert worst <= GRAD_RTOL, (s, worst, need)
    su.plan.close()


@pytest.mark.parametrize("waves", [1, 8])
def test_self_lockstep_and_flags(waves):
    su = SelfSetup("A", 15, waves)
    seeds = configs.seeds_for("A", 0, su.prob)
    sd = torch.from_numpy(seeds).cuda()
    tr = su.plan.optimize_traced({"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                                  "seeds": sd, "tag": 3})
    torch.cuda.synchronize()
    tr = {k: v.double().cpu().numpy() for k, v in tr.items()}
    lockstep_check(su, tr, seeds.shape[0])
    res = su.plan.seed_results(3, seeds.shape[0])
    ref = su.O.results(su.prob.q_start, su.prob.goal, tr["x"][-1])
    amb = np.abs(ref["clearance"]) < 1e-5
    for f in ["collision_free", "success", "valid"]:
        assert ((res[f] == ref[f].astype(int)) | amb).all(), f
    assert np.abs(res["clearance"] - ref["clearance"]).max() < 1e-4
    su.plan.close()


def test_guidance_matches_oracle():
    """Cost-gradient guidance (a few descent steps in one launch) against the
    oracle's steps from the same trajectories."""
    key = "B"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, params.DEFAULT, 1, 512 << 20)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    X = gen.random_trajectories(np.random.default_rng(8), 16, 32, prob.q_start)
    O = oracle.Oracle(robot, scene, params.as_list(), threads=8)
    J, Xg = guidance_lockstep(plan, O, prob, X, 2e-5, 4)
    Jref = O.cost(prob.q_start, prob.goal, Xg.astype(np.float64))["J"]
    assert (np.abs(J - Jref) / Jref).max() < 1e-4
    J0 = O.cost(prob.q_start, prob.goal, X.astype(np.float64))["J"]
    assert np.all(Jref < J0)
    plan.close()
