"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: kinematic invariants, hand-derived positions, analytic box
distances, closed-form smoothness sums on polynomial trajectories,
quaternion identities (scipy), central finite differences, the dense BFGS
recursion and convergence on problems with known minimisers.

Section references are to arXiv 2410.16727 (App. A.6 objective, Sec. 5.1
success thresholds, App. A.7 metrics)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from workloads import configs, gen, params

P = params.as_list()
PD = params.DEFAULT


@pytest.fixture(scope="module")
def robot():
    return configs.robot("B")


@pytest.fixture(scope="module")
def rh(robot, oracle_lib):
    return oracle.RobotH(robot)


@pytest.fixture(scope="module")
def sceneB():
    return configs.scenes("B")[0]


@pytest.fixture(scope="module")
def probB():
    return configs.problems("B")[0]


def make_oracle(robot, scene, p=None):
    return oracle.Oracle(robot, scene, p or P, threads=4)


# ------------------------------------------------------------------ FK ----

def test_fk_rotations_orthonormal(rh):
    rng = np.random.default_rng(1)
    for _ in range(2000):
        q = rng.uniform(-2.8, 2.8, 7)
        R, _ = oracle.fk_frames(rh, q)
        for i in range(8):
            assert np.abs(R[i].T @ R[i] - np.eye(3)).max() < 1e-12
            assert abs(np.linalg.det(R[i]) - 1.0) < 1e-12


def test_fk_link_lengths_preserved(robot, rh):
    rng = np.random.default_rng(2)
    L = robot.link_lengths.astype(np.float32).astype(np.float64)
    for _ in range(500):
        q = rng.uniform(-2.8, 2.8, 7)
        _, p = oracle.fk_frames(rh, q)
        assert np.linalg.norm(p[0]) < 1e-15            # joint 1 sits at the base
        for i in range(6):
            assert abs(np.linalg.norm(p[i + 1] - p[i]) - L[i]) < 1e-12
        assert abs(np.linalg.norm(p[7] - p[6]) - L[6]) < 1e-12


def test_fk_spheres_on_link_axis(robot, rh):
    rng = np.random.default_rng(3)
    off = robot.sphere_offset.astype(np.float64)
    for _ in range(200):
        X = rng.uniform(-2.8, 2.8, (1, 7))
        R, p = oracle.fk_frames(rh, X[0])
        c = oracle.sphere_centres(rh, X)[0]
        for s, l in enumerate(robot.sphere_link):
            assert abs(np.linalg.norm(c[s] - p[l - 1]) - np.linalg.norm(off[s])) < 1e-12
            # offsets lie on the link's z axis
            assert np.abs(c[s] - (p[l - 1] + off[s, 2] * R[l - 1][:, 2])).max() < 1e-12


def test_fk_zero_configuration_zigzag(robot, rh):
    """At q = 0 the +-pi/2 twists alternate the link directions between +z
    and +y; hand-derived joint origins."""
    L = robot.link_lengths.astype(np.float32).astype(np.float64)
    _, p = oracle.fk_frames(rh, np.zeros(7))
    exp = [(0, 0, 0), (0, 0, L[0]), (0, L[1], L[0]), (0, L[1], L[0] + L[2]),
           (0, L[1] + L[3], L[0] + L[2]), (0, L[1] + L[3], L[0] + L[2] + L[4]),
           (0, L[1] + L[3] + L[5], L[0] + L[2] + L[4]),
           (0, L[1] + L[3] + L[5], L[0] + L[2] + L[4] + L[6])]
    assert np.abs(p - np.array(exp)).max() < 1e-12


def test_fk_base_joint_rotates_about_world_z(rh):
    rng = np.random.default_rng(4)
    for _ in range(100):
        q = rng.uniform(-2.8, 2.8, 7)
        th = rng.uniform(-1, 1)
        q2 = q.copy()
        q2[0] += th
        c1 = oracle.sphere_centres(rh, q[None])[0]
        c2 = oracle.sphere_centres(rh, q2[None])[0]
        Rz = Rotation.from_euler("z", th).as_matrix()
        assert np.abs(c1 @ Rz.T - c2).max() < 1e-12


def test_fk_joint_axis_jacobian_matches_fd(robot, rh):
    """dc/dq_i = z_i x (c - o_i) for spheres on links >= i, else 0."""
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(20):
        q = rng.uniform(-2.8, 2.8, 7)
        R, p = oracle.fk_frames(rh, q)
        c = oracle.sphere_centres(rh, q[None])[0]
        for i in range(7):
            qp, qm = q.copy(), q.copy()
            qp[i] += h
            qm[i] -= h
            fd = (oracle.sphere_centres(rh, qp[None])[0] - oracle.sphere_centres(rh, qm[None])[0]) / (2 * h)
            z = R[i][:, 2]
            for s, l in enumerate(robot.sphere_link):
                an = np.cross(z, c[s] - p[i]) if l - 1 >= i else np.zeros(3)
                assert np.abs(fd[s] - an).max() < 1e-8


# ---------------------------------------------------------------- ESDF ----

def single_box_scene(centre, half, dims=(40, 40, 40), voxel=0.02, origin=(-0.4, -0.4, -0.4)):
    sc = gen.Scene(np.array([centre], dtype=np.float64), np.array([half], dtype=np.float64),
                   dims, gen.f32(voxel), np.asarray(origin, dtype=np.float32))
    gen.build_grids([sc])
    return sc


def analytic_box_distance(p, centre, half):
    """Distance by projecting onto the box (a different construction from
    the generator's): outside = |p - closest point|; inside = -(distance
    to the nearest face)."""
    lo, hi = np.asarray(centre) - half, np.asarray(centre) + half
    closest = np.clip(p, lo, hi)
    if np.any(p != closest):
        return float(np.linalg.norm(p - closest))
    return -float(min(np.min(p - lo), np.min(hi - p)))


def test_esdf_exact_at_nodes(robot, sceneB):
    O = make_oracle(robot, sceneB)
    rng = np.random.default_rng(6)
    for _ in range(300):
        i, j, k = rng.integers(0, 199, size=3)
        p = sceneB.origin.astype(np.float64) + np.array([i, j, k]) * sceneB.voxel
        assert abs(O.sample(p)[0] - float(sceneB.grid[k, j, i])) < 1e-12


def test_esdf_face_region_is_exact(robot):
    """In the face region of one box the distance is linear, so trilinear
    interpolation reproduces it up to float32 storage."""
    c, h = np.array([0.05, -0.03, 0.02]), np.array([0.1, 0.15, 0.08])
    sc = single_box_scene(c, h)
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(7)
    for _ in range(500):
        # a point in front of the +x face, inside the face's y/z footprint
        p = np.array([c[0] + h[0] + rng.uniform(0.03, 0.2),
                      c[1] + rng.uniform(-h[1] + 0.03, h[1] - 0.03),
                      c[2] + rng.uniform(-h[2] + 0.03, h[2] - 0.03)])
        out = O.sample(p)
        assert abs(out[0] - analytic_box_distance(p, c, h)) < 2e-7
        assert abs(out[1] - 1.0) < 1e-4 and abs(out[2]) < 1e-4 and abs(out[3]) < 1e-4


def test_esdf_general_error_bound_and_sign(robot):
    c, h = np.array([0.0, 0.02, -0.01]), np.array([0.12, 0.07, 0.1])
    sc = single_box_scene(c, h)
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(8)
    vox = sc.voxel
    for _ in range(2000):
        p = rng.uniform(-0.35, 0.35, 3)
        ref = analytic_box_distance(p, c, h)
        d = O.sample(p)[0]
        # the box distance is 1-Lipschitz: interpolation error <= voxel diagonal
        assert abs(d - ref) <= math.sqrt(3) * vox
        if ref < -math.sqrt(3) * vox:
            assert d < 0
    # strictly inside is negative
    assert O.sample(c)[0] < 0


def test_esdf_clamp_and_gradient(robot, sceneB):
    O = make_oracle(robot, sceneB)
    lo = sceneB.origin.astype(np.float64)
    hi = sceneB.hi
    rng = np.random.default_rng(9)
    for _ in range(100):
        inner = rng.uniform(lo + 0.05, hi - 0.05)
        out_pt = inner.copy()
        out_pt[0] = hi[0] + rng.uniform(0.01, 1.0)
        border = out_pt.copy()
        border[0] = hi[0]
        a = O.sample(out_pt)
        b = O.sample(border)
        assert abs(a[0] - b[0]) < 1e-12 and a[1] == 0.0 and int(a[4]) & 1
    # gradient equals the central difference of the sampled value inside a cell
    for _ in range(300):
        p = rng.uniform(lo + 0.05, hi - 0.05)
        g = O.sample(p)[1:4]
        cell = O.sample(p)[5:8]
        eps = 1e-7
        for a in range(3):
            dp = np.zeros(3)
            dp[a] = eps
            s1, s2 = O.sample(p + dp), O.sample(p - dp)
            if np.any(s1[5:8] != cell) or np.any(s2[5:8] != cell):
                continue
            assert abs((s1[0] - s2[0]) / (2 * eps) - g[a]) < 1e-6


# --------------------------------------------------------------- hinge ----

def test_hinge_pieces_and_continuity():
    eps = PD["eps"]
    assert oracle.hinge(-0.1, eps)[0] == pytest.approx(0.1 + eps / 2)
    assert oracle.hinge(eps / 2, eps)[0] == pytest.approx(eps / 8)
    assert oracle.hinge(eps * 1.5, eps) == (0.0, 0.0)
    for D0 in (0.0, eps):
        l, r = oracle.hinge(D0 - 1e-9, eps), oracle.hinge(D0 + 1e-9, eps)
        assert abs(l[0] - r[0]) < 1e-8 and abs(l[1] - r[1]) < 1e-6
    for D0 in np.linspace(-0.05, 0.05, 41):
        fd = (oracle.hinge(D0 + 1e-7, eps)[0] - oracle.hinge(D0 - 1e-7, eps)[0]) / 2e-7
        assert abs(fd - oracle.hinge(D0, eps)[1]) < 1e-5


# ---------------------------------------------------------------- costs ---

def one_sphere_robot(radius=0.05):
    base = configs.robot("A")
    return gen.Robot(base.link_lengths, base.frames, base.q_lo, base.q_hi,
                     np.array([7], dtype=np.int32), np.array([[0, 0, 0.05]], dtype=np.float32),
                     np.array([radius], dtype=np.float32))


def test_world_cost_planar_wall_closed_form(oracle_lib):
    """Distance field of the plane x = x0 (d = x - x0, exactly linear):
    C_world = w_c * sum_t phi(c_x - x0 - r)."""
    rb = one_sphere_robot()
    x0 = 0.1
    dims, vox, org = (60, 60, 60), gen.f32(0.04), np.array([-1.2, -1.2, -1.2], dtype=np.float32)
    xs = org[0] + np.arange(dims[0]) * vox
    grid = np.broadcast_to((xs - x0)[None, None, :], dims[::-1]).astype(np.float32).copy()
    sc = gen.Scene(np.zeros((0, 3)), np.zeros((0, 3)), dims, vox, org, grid)
    O = oracle.Oracle(rb, sc, params.as_list({"lambda_v": 0, "lambda_a": 0, "lambda_j": 0,
                                               "w_pos": 0, "w_rot": 0, "w_limit": 0}))
    rng = np.random.default_rng(10)
    X = rng.uniform(-2.0, 2.0, (3, 8, 7))
    c = O.cost(np.zeros(7), np.array([0, 0, 0, 1, 0, 0, 0.0]), X, grad=True, terms=True)
    for s in range(3):
        cen = O.spheres(X[s])[:, 0, :]
        exp = 0.0
        for t in range(8):
            D = (cen[t, 0] - x0) - float(np.float32(0.05))
            exp += PD["w_collision"] * oracle.hinge(D, PD["eps"])[0]
        assert c["terms"][s][0] == pytest.approx(exp, rel=1e-6, abs=1e-9)


def test_world_cost_zero_when_clear(robot):
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    X = np.random.default_rng(11).uniform(-2.8, 2.8, (4, 16, 7))
    c = O.cost(np.zeros(7), np.array([0.3, 0, 0.5, 1, 0, 0, 0]), X, grad=True, terms=True)
    assert np.all(c["terms"][:, 0] == 0.0)


@pytest.mark.parametrize("T", [4, 5, 16, 32, 64])
def test_smoothness_constant_and_ramp(robot, T):
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(12 + T)
    q0 = rng.uniform(-1, 1, 7)
    const = np.repeat(q0[None], T, axis=0)
    tm = O.cost(q0, np.array([0, 0, 0, 1, 0, 0, 0.0]), const, terms=True)["terms"][0]
    assert tm[1] == 0 and tm[2] == 0 and tm[3] == 0
    delta = rng.uniform(-0.05, 0.05, 7)
    ramp = q0[None] + np.arange(T)[:, None] * delta[None]
    tm = O.cost(q0, np.array([0, 0, 0, 1, 0, 0, 0.0]), ramp, terms=True)["terms"][0]
    n2 = float(delta @ delta)
    assert tm[1] == pytest.approx(PD["lambda_v"] * (T - 1) * n2, rel=1e-12)
    assert tm[2] == pytest.approx(2 * PD["lambda_a"] * n2, rel=1e-9)
    assert tm[3] == pytest.approx(4 * PD["lambda_j"] * n2, rel=1e-9)


@pytest.mark.parametrize("T", [4, 7, 32, 64])
def test_smoothness_quadratic_closed_form(robot, T):
    """q_t = q0 + c t^2: hand-summed velocity, acceleration and jerk terms
    including the rest-padding boundary terms."""
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(40 + T)
    q0 = rng.uniform(-1, 1, 7)
    cc = rng.uniform(-1e-3, 1e-3, 7)
    X = q0[None] + (np.arange(T) ** 2)[:, None] * cc[None]
    tm = O.cost(q0, np.array([0, 0, 0, 1, 0, 0, 0.0]), X, terms=True)["terms"][0]
    n2 = float(cc @ cc)
    n = T - 1
    vel = n2 * n * (2 * n - 1) * (2 * n + 1) / 3
    acc = n2 * (1 + 4 * (T - 2) + (2 * T - 3) ** 2)
    jerk = n2 * (2 + (2 * T - 1) ** 2 + (2 * T - 3) ** 2)
    assert tm[1] == pytest.approx(PD["lambda_v"] * vel, rel=1e-9)
    assert tm[2] == pytest.approx(PD["lambda_a"] * acc, rel=1e-9)
    assert tm[3] == pytest.approx(PD["lambda_j"] * jerk, rel=1e-9)


def test_goal_cost_zero_at_goal_and_quaternion_identity(robot, rh):
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(13)
    for _ in range(50):
        qg = rng.uniform(-2.8, 2.8, 7)
        R, p = oracle.fk_frames(rh, qg)
        quat_xyzw = Rotation.from_matrix(R[7]).as_quat()
        goal = np.concatenate([p[7], [quat_xyzw[3], *quat_xyzw[:3]]])
        X = np.repeat(qg[None], 4, axis=0)
        tm = O.cost(qg, goal, X, terms=True)["terms"][0]
        assert tm[4] < 1e-20 and abs(tm[5]) < 1e-12
        # another configuration: (3 - tr)/4 == 1 - <q, q_d>^2
        q2 = rng.uniform(-2.8, 2.8, 7)
        R2, p2 = oracle.fk_frames(rh, q2)
        tm2 = O.cost(qg, goal, np.repeat(q2[None], 4, axis=0), terms=True)["terms"][0]
        qa = Rotation.from_matrix(R2[7]).as_quat()
        qb = quat_xyzw
        assert tm2[5] == pytest.approx(PD["w_rot"] * (1 - float(qa @ qb) ** 2), rel=1e-9, abs=1e-12)
        assert tm2[4] == pytest.approx(PD["w_pos"] * float(np.sum((p2[7] - p[7]) ** 2)), rel=1e-12)


def test_rotation_error_of_a_known_rotation(robot, rh):
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    rng = np.random.default_rng(14)
    for th in [0.0, 0.01, 0.04, 0.3, 1.0, 2.5]:
        qg = rng.uniform(-2.8, 2.8, 7)
        R, p = oracle.fk_frames(rh, qg)
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        Rg = Rotation.from_matrix(R[7]) * Rotation.from_rotvec(axis * th)
        qx = Rg.as_quat()
        goal = np.concatenate([p[7] + [0.003, 0, 0], [qx[3], *qx[:3]]])
        res = O.results(qg, goal, np.repeat(qg[None, None], 4, axis=1))
        assert res["rot_err"][0] == pytest.approx(th, abs=1e-9)
        assert res["pos_err"][0] == pytest.approx(0.003, abs=1e-12)
        exp_success = th < PD["tol_rot"]
        assert bool(res["success"][0]) == exp_success


def test_limit_penalty_closed_form(robot):
    sc = gen.empty_scene()
    O = make_oracle(robot, sc)
    X = np.zeros((1, 4, 7))
    X[0, 2, 3] = 2.8 + 0.1
    X[0, 3, 5] = -2.8 - 0.2
    tm = O.cost(np.zeros(7), np.array([0, 0, 0, 1, 0, 0, 0.0]), X, terms=True)["terms"][0]
    assert tm[6] == pytest.approx(PD["w_limit"] * (0.1 ** 2 + 0.2 ** 2), rel=1e-6)
    res = O.results(np.zeros(7), np.array([0, 0, 0, 1, 0, 0, 0.0]), X)
    assert res["within_limits"][0] == 0


# ------------------------------------------------------------- gradient ---

def test_gradient_matches_central_differences(robot, sceneB, probB):
    O = make_oracle(robot, sceneB)
    rng = np.random.default_rng(15)
    # arbitrary trajectories inside the limits reach into the shelves, so
    # the collision term is active
    X = gen.random_trajectories(rng, 4, 16, probB.q_start)
    c = O.cost(probB.q_start, probB.goal, X, grad=True, terms=True)
    assert np.all(c["terms"][:, 0] > 0)
    for s in range(4):
        amb, _ = O.ambiguity(X[s], tol=3e-4)
        idx = np.arange(7, 16 * 7)
        fd = O.fd_grad(probB.q_start, probB.goal, X[s], idx, h=1e-6)
        an = c["G"][s].reshape(-1)[idx]
        ok = amb.reshape(-1)[idx] == 0
        scale = np.abs(an).max()
        err = np.abs(fd - an)[ok] / scale
        assert ok.sum() > 0.8 * len(idx)
        assert err.max() < 1e-7, err.max()
    assert np.all(c["G"][:, 0, :] == 0)


# ----------------------------------------------------------- optimiser ----

def test_two_loop_equals_dense_bfgs():
    rng = np.random.default_rng(16)
    n = 12
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)
    for k in range(1, 9):
        S = rng.normal(size=(k, n))
        Y = S @ A                      # curvature pairs of a quadratic
        g = rng.normal(size=n)
        gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
        H = gamma * np.eye(n)
        for s, y in zip(S, Y):
            rho = 1.0 / float(s @ y)
            V = np.eye(n) - rho * np.outer(y, s)
            H = V.T @ H @ V + rho * np.outer(s, s)
        d = oracle.two_loop(g, S, Y)
        assert np.abs(d - (-H @ g)).max() < 1e-10 * max(1.0, np.abs(H @ g).max())


def test_lbfgs_quadratic_converges_to_solution():
    rng = np.random.default_rng(17)
    n = 20
    A = rng.normal(size=(n, n))
    A = A @ A.T / n + np.eye(n)
    b = rng.normal(size=n)
    f = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    x, Jt = oracle.minimize(f, np.zeros(n), 200, params.as_list())
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-8
    assert np.all(np.diff(Jt) <= 1e-12)


def test_lbfgs_rosenbrock():
    def f(x):
        a, b = x
        J = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return J, g
    x, Jt = oracle.minimize(f, np.array([-1.2, 1.0]), 400, params.as_list())
    assert np.abs(x - 1.0).max() < 1e-6
    assert np.all(np.diff(Jt) <= 0)


def test_optimizer_monotone_and_reaches_goal_in_free_space(robot):
    sc = gen.empty_scene()
    prob = configs.problems("B")[0]
    O = make_oracle(robot, sc)
    X0 = configs.seeds_for("B", 0, prob, S=6, T=32)
    X, tr = O.optimize(prob.q_start, prob.goal, X0, 100, trace=True)
    assert np.all(np.diff(tr["J"], axis=0) <= 0)
    res = O.results(prob.q_start, prob.goal, X)
    assert np.all(res["pos_err"] < PD["tol_pos"])
    assert np.all(res["rot_err"] < PD["tol_rot"])
    assert np.all(X[:, 0, :] == X0[:, 0, :])


def test_best_seed_rule_and_invalid_seeds(robot):
    sc = gen.empty_scene()
    prob = configs.problems("B")[0]
    O = make_oracle(robot, sc)
    X0 = configs.seeds_for("B", 0, prob, S=1, T=16)
    X = np.repeat(X0, 4, axis=0).astype(np.float64)
    X[1, 5, 2] = np.nan
    res = O.results(prob.q_start, prob.goal, X)
    assert res["valid"].tolist() == [1, 0, 1, 1]
    assert res["best"] == 0          # equal costs: lowest index wins


def test_guidance_step_is_gradient_descent(robot, sceneB, probB):
    """One guidance step equals x - alpha * grad (the oracle's gradient is
    pinned by central differences above); small steps decrease the cost."""
    O = make_oracle(robot, sceneB)
    X = gen.random_trajectories(np.random.default_rng(21), 3, 8, probB.q_start).astype(np.float64)
    c = O.cost(probB.q_start, probB.goal, X, grad=True)
    X1 = O.guide(probB.q_start, probB.goal, X, 1e-6, 1)
    assert np.abs(X1 - (X - 1e-6 * c["G"])).max() < 1e-15
    J1 = O.cost(probB.q_start, probB.goal, X1)["J"]
    assert np.all(J1 < c["J"])
    assert np.array_equal(X1[:, 0], X[:, 0])
