"""GPU parity of the optional swept collision term (configurations
interpolated linearly between consecutive waypoints) against the FP64
oracle: cost/gradient, a lockstep optimisation with teams and without, and
the flags and clearance of the final trajectories."""
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


class SweptSetup:
    def __init__(self, key, iters, waves, k):
        self.key = key
        self.ps = dict(params.DEFAULT, swept_samples=k)
        self.robot = configs.robot(key)
        self.scene = configs.scenes(key, only={0})[0]
        self.prob = configs.problems(key)[0]
        self.iters = iters
        self.plan = dsopt.Plan(self.robot, dict(self.ps, waves_per_seed=waves), iters, 512 << 20)
        self.plan.upload_scene(0, self.scene.grid, self.scene.voxel, self.scene.origin)
        self.O = oracle.Oracle(self.robot, self.scene, params.as_list(self.ps), threads=8)


@pytest.mark.parametrize("key,T,k", [("B", 32, 1), ("B", 32, 3), ("A", 16, 2), ("B", 64, 2),
                                     ("B", 5, 8)])
def test_swept_cost_grad_parity(key, T, k):
    su = SweptSetup(key, 1, 1, k)
    print(f"swept cost/grad {key} T={T} k={k}", flush=True)
    X = gen.random_trajectories(np.random.default_rng(40 + T + k), 8, T, su.prob.q_start)
    ref = su.O.cost(su.prob.q_start, su.prob.goal, X.astype(np.float64), grad=True, absg=True,
                    terms=True)
    J, G = su.plan.cost_grad(0, su.prob.q_start, su.prob.goal, torch.from_numpy(X).cuda())
    J2 = su.plan.cost(0, su.prob.q_start, su.prob.goal, torch.from_numpy(X).cuda())
    J, G, J2 = J.cpu().numpy(), G.cpu().numpy(), J2.cpu().numpy()
    assert (np.abs(J - ref["J"]) / ref["J"]).max() < COST_RTOL
    assert (np.abs(J2 - ref["J"]) / ref["J"]).max() < COST_RTOL
    for s in range(X.shape[0]):
        worst, need = grad_check(su.O, su.prob, X[s], G[s], ref["G"][s], ref["A"][s])
        assert worst <= GRAD_RTOL, (s, worst, need)
    assert np.all(G[:, 0, :] == 0)
    su.plan.close()


def test_swept_with_self_collision():
    """Both optional terms on at once (fat spheres so that pairs touch)."""
    from test_gpu_self import fat
    key, k = "B", 2
    ps = dict(params.DEFAULT, swept_samples=k, w_self=50.0)
    robot = fat(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, ps, 1, 512 << 20)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    O = oracle.Oracle(robot, scene, params.as_list(ps), threads=8)
    X = gen.random_trajectories(np.random.default_rng(11), 8, 32, prob.q_start)
    ref = O.cost(prob.q_start, prob.goal, X.astype(np.float64), grad=True, absg=True, terms=True)
    assert np.all(ref["terms"][:, 7] > 0)
    J, G = plan.cost_grad(0, prob.q_start, prob.goal, torch.from_numpy(X).cuda())
    J, G = J.cpu().numpy(), G.cpu().numpy()
    assert (np.abs(J - ref["J"]) / ref["J"]).max() < COST_RTOL
    for s in range(X.shape[0]):
        worst, need = grad_check(O, prob, X[s], G[s], ref["G"][s], ref["A"][s])
        assert worst <= GRAD_RTOL, (s, worst, need)
    plan.close()


@pytest.mark.parametrize("waves,k", [(1, 2), (8, 1)])
def test_swept_lockstep_and_flags(waves, k):
    su = SweptSetup("A", 15, waves, k)
    seeds = configs.seeds_for("A", 0, su.prob)
    print(f"swept lockstep W={waves} k={k}", flush=True)
    sd = torch.from_numpy(seeds).cuda()
    tr = su.plan.optimize_traced({"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                                  "seeds": sd, "tag": 4})
    torch.cuda.synchronize()
    tr = {kk: v.double().cpu().numpy() for kk, v in tr.items()}
    lockstep_check(su, tr, seeds.shape[0])
    res = su.plan.seed_results(4, seeds.shape[0])
    ref = su.O.results(su.prob.q_start, su.prob.goal, tr["x"][-1])
    amb = np.abs(ref["clearance"]) < 1e-5
    for f in ["collision_free", "success", "valid"]:
        assert ((res[f] == ref[f].astype(int)) | amb).all(), f
    assert np.abs(res["clearance"] - ref["clearance"]).max() < 1e-4
    su.plan.close()


def test_swept_samples_out_of_range_rejected():
    rb = configs.robot("A")
    with pytest.raises(dsopt.DsError):
        dsopt.Plan(rb, dict(params.DEFAULT, swept_samples=9), 1, 64 << 20)
