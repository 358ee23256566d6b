"""GPU parity: the gfx950 library against the FP64 oracle on the same
seeded inputs, through the C ABI.

Tolerances (the FP32 path against the FP64 oracle): sphere centres within
1e-5 m and within KC 2^-24 times the robot's reach (the float32 kinematics
bound the gradient tolerance assumes); costs within 1e-4 relative; every
gradient element e within
    1e-4 |g_ref|_inf + amb_e + B_e + GRAD_C 2^-24 A_e,
where amb_e is the oracle's bound for samples within 1e-4 voxel of a
trilinear cell face (a float32 caller may legitimately take the
neighbouring cell), B_e the oracle's first-order bound of what float32
kinematics (positions off by KC 2^-24 reach, axes by KETA 2^-24) can move
the element, through the hinge's curvature, the field's second derivatives
and the moment arms (oracle fp32_bound), and A_e the element's sum of
absolute contributions (rounding of the sums); per-seed flags exactly,
except seeds whose deciding margin is below the float32 resolution
(reported as ambiguous)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

P = params.DEFAULT
COST_RTOL = 1e-4
GRAD_RTOL = 1e-4
# coefficients of the gradient tolerance (design notes, parity): rounding of
# an element's sums, and the float32 kinematics error (positions within
# KC 2^-24 reach, axes within KETA 2^-24)
GRAD_C = 8.0
KC = 4.0
KETA = 4.0
U32 = 2.0 ** -24
AMB_TOL = 1e-4
NEED = {"c": 0.0}   # largest rounding coefficient an element needed so far


def say(*a):
    print(*a, flush=True)


def grad_excess(G, Gref, A, amb, fb, w=1.0):
    """(max_e (|G - w Gref| - w (amb_e + B_e + GRAD_C u A_e)) / (w |Gref|_inf),
    the rounding coefficient the worst element needs beyond the other
    terms): the test passes when the first is <= GRAD_RTOL."""
    gn = w * np.abs(Gref).max()
    ex = np.abs(G - w * Gref) - w * amb - w * fb
    worst = float(((ex - w * GRAD_C * U32 * A) / gn).max())
    over = ex - GRAD_RTOL * gn
    pos = over > 0
    need = float((over[pos] / np.maximum(w * U32 * A[pos], 1e-300)).max()) if pos.any() else 0.0
    NEED["c"] = max(NEED["c"], need)
    return worst, need


def grad_check(O, prob, X, G, Gref, A, w=1.0):
    """grad_excess for one trajectory X [T, 7] with the oracle's ambiguity
    and float32 bounds at X."""
    X64 = np.asarray(X, dtype=np.float64)
    amb, _ = O.ambiguity(X64, AMB_TOL)
    fb, _ = O.fp32_bound(prob.q_start, prob.goal, X64, KC, KETA)
    return grad_excess(G, Gref, A, amb, fb, w)


class Setup:
    def __init__(self, key, iters=None, waves=1):
        self.key = key
        self.robot = configs.robot(key)
        self.scene = configs.scenes(key, only={0})[0]
        self.prob = configs.problems(key)[0]
        self.iters = iters if iters is not None else configs.WORKLOADS[key].iters
        self.plan = dsopt.Plan(self.robot, dict(P, waves_per_seed=waves), self.iters, 512 << 20)
        self.plan.upload_scene(0, self.scene.grid, self.scene.voxel, self.scene.origin)
        self.O = oracle.Oracle(self.robot, self.scene, params.as_list(), threads=8)


_setups = {}


def setup(key, iters=None, waves=1):
    k = (key, iters, waves)
    if k not in _setups:
        _setups[k] = Setup(key, iters, waves)
    return _setups[k]


def random_trajs(seed, S, T, q_start, spread=1.0):
    rng = np.random.default_rng(seed)
    return gen.random_trajectories(rng, S, T, q_start, scale=spread)


def check_cost_grad(su, X):
    say(f"cost/grad parity {su.key} S={X.shape[0]} T={X.shape[1]}")
    Xd = torch.from_numpy(X).cuda()
    J, G = su.plan.cost_grad(0, su.prob.q_start, su.prob.goal, Xd)
    J2 = su.plan.cost(0, su.prob.q_start, su.prob.goal, Xd)
    torch.cuda.synchronize()
    J, G, J2 = J.cpu().numpy(), G.cpu().numpy(), J2.cpu().numpy()
    ref = su.O.cost(su.prob.q_start, su.prob.goal, X.astype(np.float64), grad=True, absg=True)
    rel = np.abs(J - ref["J"]) / np.abs(ref["J"])
    assert rel.max() < COST_RTOL, rel.max()
    assert np.abs(J2 - ref["J"]).max() / np.abs(ref["J"]).min() < COST_RTOL
    need = 0.0
    for s in range(X.shape[0]):
        worst, nd = grad_check(su.O, su.prob, X[s], G[s], ref["G"][s], ref["A"][s])
        need = max(need, nd)
        assert worst <= GRAD_RTOL, (s, worst, nd)
    say(f"  cost rel {rel.max():.2e}, gradient rounding coefficient needed {need:.1f}")
    assert np.all(G[:, 0, :] == 0)
    return rel.max()


def guidance_lockstep(plan, O, prob, X, alpha, n, W_chk=None):
    """Guidance parity step by step: the n-step launch equals n one-step
    launches bitwise, and every GPU step from the GPU's own iterate X_k
    equals the oracle's step from X_k to alpha times the gradient tolerance
    (plus the float32 rounding of the update).  Returns the cost after n
    steps (GPU) and the final iterate."""
    Xd = torch.from_numpy(X).cuda()
    J = plan.guide(0, prob.q_start, prob.goal, Xd, alpha, n).cpu().numpy()
    Xn = Xd.cpu().numpy()
    Xk = X.copy()
    for k in range(n):
        Xs = torch.from_numpy(Xk).cuda()
        plan.guide(0, prob.q_start, prob.goal, Xs, alpha, 1)
        X1 = Xs.cpu().numpy()
        X64 = Xk.astype(np.float64)
        ref = O.cost(prob.q_start, prob.goal, X64, grad=True, absg=True)
        step_ref = X64 - alpha * ref["G"]
        for s in range(X.shape[0]):
            amb, _ = O.ambiguity(X64[s], AMB_TOL)
            fb, _ = O.fp32_bound(prob.q_start, prob.goal, X64[s], KC, KETA)
            gn = np.abs(ref["G"][s]).max()
            tol = alpha * (GRAD_RTOL * gn + GRAD_C * U32 * ref["A"][s] + amb + fb) + \
                2 * U32 * np.abs(X64[s])
            err = np.abs(X1[s] - step_ref[s])
            assert (err <= tol).all(), (k, s, float((err - tol).max()))
        Xk = X1
    assert np.array_equal(Xk, Xn)
    return J, Xn


@pytest.mark.parametrize("key", ["A", "B", "C"])
def test_sphere_centres(key):
    su = setup(key, 1)
    X = random_trajs(1, 256, 16, su.prob.q_start)
    say(f"sphere centres {key}")
    c = su.plan.sphere_centres(torch.from_numpy(X).cuda()).cpu().numpy()
    _, reach = su.O.fp32_bound(su.prob.q_start, su.prob.goal, X[0].astype(np.float64), KC, KETA)
    worst = 0.0
    for s in range(X.shape[0]):
        ref = su.O.spheres(X[s].astype(np.float64))
        err = np.linalg.norm(c[s] - ref, axis=-1).max()
        worst = max(worst, err)
        assert np.abs(c[s] - ref).max() < 1e-5
        assert err <= KC * U32 * reach, (s, err / (U32 * reach))
    say(f"  centre error {worst:.2e} m = {worst / (U32 * reach):.2f} x 2^-24 x reach")


@pytest.mark.parametrize("key,T", [("A", 32), ("B", 32), ("A", 16), ("A", 9)])
def test_cost_grad_random_trajectories(key, T):
    """(A, T <= 16): four lanes per waypoint hold at most one sphere per
    link, which selects the all-gathers-in-flight evaluation form."""
    su = setup(key, 1)
    X = random_trajs(2, 16, T, su.prob.q_start)
    check_cost_grad(su, X)


@pytest.mark.parametrize("T", [4, 5, 15, 16, 17, 31, 32, 33, 63, 64])
def test_cost_grad_horizons(T):
    su = setup("B", 1)
    X = random_trajs(100 + T, 5, T, su.prob.q_start)
    check_cost_grad(su, X)


def test_cost_grad_full_size_differentiation_workload():
    """256 seeds x 64 waypoints, 60 spheres, 200^3 grid (the full
    differentiation workload), seeds plus trajectories driven into the
    shelves."""
    su = setup("C", 1)
    X = configs.seeds_for("C", 0, su.prob)
    X[128:] = random_trajs(3, 128, 64, su.prob.q_start)
    check_cost_grad(su, X)


def run_traced(su, S=None, T=None, tag=7):
    seeds = configs.seeds_for(su.key, 0, su.prob, S=S, T=T)
    say(f"traced optimisation {su.key} S={seeds.shape[0]} T={seeds.shape[1]} iters={su.iters}")
    sd = torch.from_numpy(seeds).cuda()
    tr = su.plan.optimize_traced({"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                                  "seeds": sd, "tag": tag})
    torch.cuda.synchronize()
    tr = {k: v.double().cpu().numpy() for k, v in tr.items()}
    return seeds, tr


def lockstep_check(su, tr, S):
    worst = np.zeros(4)
    ties = 0
    for s in range(S):
        rep = su.O.lockstep(su.prob.q_start, su.prob.goal, tr["x"][:, s], tr["g"][:, s],
                            tr["J"][:, s], tr["d"][:, s], tr["alpha"][:, s], AMB_TOL, GRAD_C,
                            KC, KETA)
        near_tie = rep[:, 5] < 1e-4
        ties += int(near_tie.sum())
        worst[0] = max(worst[0], rep[:, 0].max())
        worst[1] = max(worst[1], rep[:, 1].max())
        worst[2] = max(worst[2], rep[:, 10].max())
        NEED["c"] = max(NEED["c"], rep[:, 10].max())
        assert rep[:, 0].max() < COST_RTOL, (s, rep[:, 0].max())
        assert rep[:, 1].max() < GRAD_RTOL, (s, rep[:, 1].max())
        # the direction is recomputed from the same history in FP64
        assert rep[:, 3].max() < 1e-3, (s, rep[:, 3].max())
        # the accepted step: identical unless the decision is a near tie
        agree = (rep[:, 4] == tr["alpha"][:, s]) | near_tie
        assert agree.all(), (s, np.nonzero(~agree))
        # x_{k+1} = x_k + alpha_k d_k (float32 rounding only)
        assert rep[:, 6].max() < 1e-5
    say(f"lockstep worst cost {worst[0]:.2e} grad {worst[1]:.2e} (rounding coefficient "
        f"needed {worst[2]:.1f}) near-ties {ties}")
    return ties


@pytest.mark.parametrize("key,waves", [("A", 1), ("B", 1), ("A", 8), ("B", 8), ("B", 2)])
def test_lockstep_iterations(key, waves):
    su = setup(key, waves=waves)
    seeds, tr = run_traced(su)
    lockstep_check(su, tr, seeds.shape[0])
    su.plan.release(7)


class ShortHistory(Setup):
    def __init__(self, key, iters, waves, m):
        self.key = key
        self.ps = dict(P, history=m)
        self.robot = configs.robot(key)
        self.scene = configs.scenes(key, only={0})[0]
        self.prob = configs.problems(key)[0]
        self.iters = iters
        self.plan = dsopt.Plan(self.robot, dict(self.ps, waves_per_seed=waves), iters, 512 << 20)
        self.plan.upload_scene(0, self.scene.grid, self.scene.voxel, self.scene.origin)
        self.O = oracle.Oracle(self.robot, self.scene, params.as_list(self.ps), threads=8)


@pytest.mark.parametrize("waves,m", [(8, 3), (2, 5), (1, 3), (8, 1), (4, 7)])
def test_lockstep_short_history(waves, m):
    """History memories below 8 (the ring wraps at m; a team's inner-product
    direction and a single wavefront's two-loop) against the oracle's FP64
    two-loop on the same history, iteration by iteration."""
    su = ShortHistory("B", 40, waves, m)
    say(f"short history m={m} W={waves}")
    seeds, tr = run_traced(su, S=8, tag=9)
    lockstep_check(su, tr, seeds.shape[0])
    su.plan.close()


@pytest.mark.parametrize("key,waves", [("A", 1), ("B", 1), ("B", 8)])
def test_flags_match_oracle_on_final_trajectories(key, waves):
    su = setup(key, waves=waves)
    seeds, tr = run_traced(su, tag=8)
    S, T = seeds.shape[0], seeds.shape[1]
    res = su.plan.seed_results(8, S)
    traj, best = su.plan.get_best(8, T)
    Xf = tr["x"][-1]
    ref = su.O.results(su.prob.q_start, su.prob.goal, Xf)
    amb = np.abs(ref["clearance"]) < 1e-5
    for f in ["collision_free", "within_limits", "success", "valid"]:
        ok = (res[f] == ref[f].astype(int)) | amb
        assert ok.all(), (f, res[f], ref[f])
    assert np.abs(res["cost"] - ref["J"]).max() / np.abs(ref["J"]).max() < COST_RTOL
    assert np.abs(res["clearance"] - ref["clearance"]).max() < 1e-4
    assert np.abs(res["pos_err"] - ref["pos_err"]).max() < 1e-5
    assert np.abs(res["rot_err"] - ref["rot_err"]).max() < 1e-3
    # best seed: the oracle's rule on the GPU's per-seed costs
    if not amb.any():
        assert best["best_seed"] == ref["best"] or \
            abs(ref["J"][best["best_seed"]] - ref["J"][ref["best"]]) < 1e-4 * ref["J"][ref["best"]]
    assert np.array_equal(traj, tr["x"][-1][best["best_seed"]].astype(np.float32))
    su.plan.release(8)


def test_invalid_inputs_are_rejected():
    su = setup("A", 1)
    seeds = torch.zeros((2, 8, 7), device="cuda")
    good = {"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal, "seeds": seeds,
            "tag": 99}
    for bad, code in [({"scene": 5}, dsopt.DS_ERR_NOT_FOUND),
                      ({"seeds": torch.zeros((2, 3, 7), device="cuda")}, dsopt.DS_ERR_INVALID),
                      ({"seeds": torch.zeros((2, 65, 7), device="cuda")}, dsopt.DS_ERR_INVALID),
                      ({"seeds": torch.zeros((0, 8, 7), device="cuda")}, dsopt.DS_ERR_INVALID),
                      ({"goal": np.array([0, 0, 0, 0, 0, 0, 0], dtype=np.float32)},
                       dsopt.DS_ERR_INVALID)]:
        with pytest.raises(dsopt.DsError) as e:
            su.plan.optimize([dict(good, **bad)])
        assert e.value.code == code
    with pytest.raises(dsopt.DsError):
        su.plan.upload_scene(3, np.zeros((1, 4, 4), dtype=np.float32), 0.1, (0, 0, 0))


@pytest.mark.parametrize("waves", [1, 4])
def test_determinism_bitwise(waves):
    su = setup("B", waves=waves)
    seeds = torch.from_numpy(configs.seeds_for("B", 0, su.prob)).cuda()
    outs = []
    for tag in (21 + 10 * waves, 22 + 10 * waves):
        out = torch.zeros_like(seeds)
        su.plan.optimize([{"scene": 0, "q_start": su.prob.q_start, "goal": su.prob.goal,
                           "seeds": seeds, "tag": tag, "out": out}])
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        su.plan.release(tag)
    assert np.array_equal(outs[0], outs[1])
