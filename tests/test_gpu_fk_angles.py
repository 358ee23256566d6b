"""Forward kinematics over a wide range of joint angles: sphere centres and
costs of configurations far outside the joint limits (up to 100 rad, and
angles at and next to multiples of pi/2) against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, params  # noqa: E402

from test_gpu_parity import COST_RTOL  # noqa: E402

SCALES = [1.0, 3.2, 10.0, 40.0, 63.9, 64.1, 100.0]


def test_sphere_centres_and_cost_at_large_angles():
    robot = configs.robot("B")
    scene = configs.scenes("B", only={0})[0]
    prob = configs.problems("B")[0]
    plan = dsopt.Plan(robot, params.DEFAULT, 1, 512 << 20)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    O = oracle.Oracle(robot, scene, params.as_list(), threads=8)
    rng = np.random.default_rng(23)
    X = (rng.uniform(-1.0, 1.0, (len(SCALES), 16, 7)) *
         np.array(SCALES)[:, None, None]).astype(np.float32)
    # exact multiples of pi/2 and their float neighbours (quadrant edges)
    edge = (np.linspace(-40, 40, 8).round() * (np.pi / 2)).astype(np.float32)
    X[0, :, 0] = np.concatenate([edge, np.nextafter(edge, np.float32(np.inf))])
    print(f"large-angle FK: scales {SCALES}", flush=True)
    c = plan.sphere_centres(torch.from_numpy(X).cuda()).cpu().numpy()
    for s in range(X.shape[0]):
        ref = O.spheres(X[s].astype(np.float64))
        assert np.abs(c[s] - ref).max() < 2e-5, (SCALES[s], np.abs(c[s] - ref).max())
    J = plan.cost(0, prob.q_start, prob.goal, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = O.cost(prob.q_start, prob.goal, X.astype(np.float64))
    assert (np.abs(J - ref["J"]) / ref["J"]).max() < COST_RTOL
    plan.close()
