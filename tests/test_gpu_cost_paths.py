"""Cost/gradient and guidance in both launch forms of the evaluation
kernels: one wavefront per seed (a batch large enough to fill the chip on
its own, 2100 seeds) and teams of wavefronts per seed (small batches),
against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

from test_gpu_parity import check_cost_grad, guidance_lockstep, random_trajs, setup  # noqa: E402


@pytest.mark.parametrize("S,T", [(2100, 16), (3, 40)])
def test_cost_grad_single_wavefronts_and_teams(S, T):
    su = setup("B", 1)
    X = random_trajs(500 + S, S, T, su.prob.q_start)
    check_cost_grad(su, X)


def test_guidance_single_wavefronts():
    key = "B"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, params.DEFAULT, 1, 512 << 20)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    X = gen.random_trajectories(np.random.default_rng(81), 2100, 16, prob.q_start)
    print("guidance, 2100 seeds", flush=True)
    O = oracle.Oracle(robot, scene, params.as_list(), threads=8)
    J, Xg = guidance_lockstep(plan, O, prob, X, 2e-5, 3)
    Jref = O.cost(prob.q_start, prob.goal, Xg.astype(np.float64))["J"]
    assert (np.abs(J - Jref) / Jref).max() < 1e-4
    plan.close()
