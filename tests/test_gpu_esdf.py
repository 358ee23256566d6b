"""GPU distance field from occupancy vs the oracle's brute-force
definition (squared distances are exact integers on both sides; the final
sqrt/scale differs by float rounding only)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402


def plan(arena=1 << 30, key="A", iters=1):
    return dsopt.Plan(configs.robot(key), params.DEFAULT, iters, arena)


@pytest.mark.parametrize("shape,p", [((9, 10, 11), 0.2), ((16, 17, 33), 0.05), ((2, 5, 3), 0.5)])
def test_random_grids_match_oracle(shape, p):
    rng = np.random.default_rng(sum(shape))
    occ = (rng.random(shape) < p).astype(np.uint8)
    occ.reshape(-1)[0] = 1
    occ.reshape(-1)[-1] = 0
    h = 0.013
    pl = plan()
    out = torch.zeros(shape, dtype=torch.float32, device="cuda")
    pl.scene_from_occupancy(5, occ, h, (0.1, -0.2, 0.3), out=out)
    torch.cuda.synchronize()
    d = out.cpu().numpy().astype(np.float64)
    ref = oracle.esdf_from_occupancy(occ, np.float32(h))
    assert np.abs(d - ref).max() <= 2e-7 * max(1.0, np.abs(ref).max())
    assert np.array_equal(d < 0, occ != 0)
    pl.close()


def test_full_size_shelf_grid_sampled():
    """200^3 grid of the cluttered workload's shelf scene: every sampled
    voxel equals the brute-force definition; the field drives an
    optimisation like the uploaded one."""
    sc = configs.scenes("B", only={0})[0]
    occ = gen.occupancy(sc)
    pl = plan(2 << 30, key="B", iters=20)
    out = torch.zeros(occ.shape, dtype=torch.float32, device="cuda")
    pl.scene_from_occupancy(0, occ, sc.voxel, sc.origin, out=out)
    torch.cuda.synchronize()
    d = out.cpu().numpy().reshape(-1).astype(np.float64)
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.choice(occ.size, 150, replace=False),
                          rng.choice(np.flatnonzero(occ.reshape(-1)), 50, replace=False)])
    ref = oracle.esdf_from_occupancy(occ, sc.voxel, which=idx, threads=16)
    assert np.abs(d[idx] - ref).max() <= 2e-7 * np.abs(ref).max() + 1e-9
    # outside the boxes the scene's field (min over boxes) is the exact
    # distance to their union and the voxel field lies within a voxel
    # diagonal of it; inside overlapping boxes the min over boxes understates
    # the depth, so there the voxel field is only at least as deep (less a
    # voxel diagonal)
    d3 = d.reshape(occ.shape)
    tol = np.sqrt(3) * sc.voxel + 1e-6
    out_mask = sc.grid >= 0
    assert np.abs(d3 - sc.grid)[out_mask].max() < tol
    assert np.all(-d3[~out_mask] >= -sc.grid[~out_mask] - tol)
    prob = configs.problems("B")[0]
    seeds = torch.from_numpy(configs.seeds_for("B", 0, prob, S=8)).cuda()
    pl.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": seeds,
                  "tag": 1}])
    _, res = pl.get_best(1, prob.T)
    assert res["n_valid_seeds"] == 8
    pl.close()
