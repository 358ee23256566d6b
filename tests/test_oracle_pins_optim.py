"""Pins of the oracle's optimiser decisions, trajectory metrics and
gradient-ambiguity bound against hand-worked values and closed forms.

Each test names the plausible mistake in the oracle that it catches.  The
optimiser readings (four power-of-two candidates, Armijo with c1, the
infinity-norm steepest step delta0 and cap, the steepest restart, history
memory m) follow the design notes; the metrics are App. A.7 (jerk, motion
time against velocity / acceleration / jerk limits); the ambiguity bound is
the tolerance term of the per-iteration gradient comparison.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import configs, gen, params

P = params.as_list()
PD = params.DEFAULT


# ------------------------------------------------------------ line search --

def _rhs(J0, gtd, k):
    return J0 + PD["c1"] * 2.0 ** (-k) * gtd


def test_choose_step_largest_armijo_step(oracle_lib):
    """alpha = 1 fails the Armijo test and alpha = 1/2 passes: the choice is
    1/2 although 1/4 and 1/8 pass with lower costs.  Catches: choosing the
    smallest passing step, or the cheapest passing step."""
    J0, gtd = 10.0, -4.0
    Jk = [10.5, 9.0, 8.0, 7.0]
    assert Jk[0] > _rhs(J0, gtd, 0) and all(Jk[k] <= _rhs(J0, gtd, k) for k in (1, 2, 3))
    k, margin = oracle.choose_step(J0, gtd, Jk, P)
    assert k == 1
    # the margin is the smallest |J_k - rhs_k| over the candidates
    assert margin == pytest.approx(min(abs(Jk[i] - _rhs(J0, gtd, i)) for i in range(4)))


def test_choose_step_fallback_to_cheapest_below_current(oracle_lib):
    """No candidate passes Armijo; 1/4 is the cheapest and below J(x): the
    choice is 1/4.  With J(1/2) == J(1/4) the tie goes to the larger step,
    1/2.  Catches: taking the first candidate below J(x), ties to the
    smaller step, or no fallback at all."""
    J0, gtd = 10.0, -4.0
    Jk = [10.2, 9.99995, 9.99992, 10.1]
    assert all(Jk[k] > _rhs(J0, gtd, k) for k in range(4))
    assert oracle.choose_step(J0, gtd, Jk, P)[0] == 2
    Jt = [10.2, 9.99995, 9.99995, 10.1]
    assert oracle.choose_step(J0, gtd, Jt, P)[0] == 1


def test_choose_step_no_step_when_nothing_decreases(oracle_lib):
    """Every candidate is >= J(x) (one equals it): no step.  Catches: a
    fallback that accepts a candidate equal to or above J(x)."""
    J0, gtd = 10.0, -4.0
    assert oracle.choose_step(J0, gtd, [10.0, 10.3, 10.0, 11.0], P)[0] == -1
    assert oracle.choose_step(J0, gtd, [10.0, 10.0, 10.0, 10.0], P)[0] == -1


def test_failed_line_search_clears_history(oracle_lib):
    """f = |x|^2/2 whose reported gradient flips sign once x_0 < 0.5: the
    optimiser builds a history on the honest part, then every candidate
    along the (wrong) descent direction raises f, no step is taken and the
    history must be empty afterwards.  Catches: keeping the history after
    a rejected step."""
    def f(x):
        J = 0.5 * float(x @ x)
        return J, (x.copy() if x[0] >= 0.5 else -x)
    tr = oracle.minimize_trace(f, np.array([3.0, 1.0, -2.0, 0.5]), 30, P)
    zero = np.nonzero(tr["alpha"] == 0)[0]
    assert zero.size > 0
    k = int(zero[0])
    assert k > 0 and tr["count"][k - 1] > 0          # history existed before
    assert tr["count"][k] == 0                       # ... and was cleared
    # every candidate from x_k along d_k is at least f(x_k)
    xk, dk = tr["x"][k], tr["d"][k]
    J0 = 0.5 * xk @ xk
    for c in range(PD["n_ls"]):
        xt = xk + 2.0 ** (-c) * dk
        assert 0.5 * xt @ xt >= J0


# --------------------------------------------------------------- direction --

def test_direction_empty_history_is_scaled_steepest(oracle_lib):
    """Empty history: d = -g * delta0 / |g|_inf exactly.  Catches: a 2-norm
    (or no) normalisation of the steepest step."""
    g = np.random.default_rng(30).normal(size=21) * 7.0
    d, cleared = oracle.direction(g, np.zeros((0, 21)), np.zeros((0, 21)), P)
    assert not cleared
    assert np.array_equal(d, -g * (PD["delta0"] / np.abs(g).max()))
    assert np.abs(d).max() == pytest.approx(PD["delta0"], rel=1e-15)
    assert np.linalg.norm(d) > PD["delta0"] * 1.5          # the 2-norm differs


def _textbook_direction(g, S, Y):
    """-H g with H from the dense BFGS recursion, H_0 = gamma I (newest
    pair), pairs applied oldest first."""
    n = g.shape[0]
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return -H @ g


def test_direction_non_descent_restarts(oracle_lib):
    """A pair of negative curvature (s.y < 0) makes -H g an ascent
    direction; the optimiser must clear the history and return the scaled
    steepest step.  Catches: a missing restart test, or a test on the wrong
    sign."""
    rng = np.random.default_rng(31)
    n = 9
    g = rng.normal(size=n)
    s = rng.normal(size=n)
    y = -s + 0.1 * rng.normal(size=n)
    assert float(s @ y) < 0
    raw = _textbook_direction(g, s[None], y[None])
    assert float(g @ raw) >= 0                               # really not a descent direction
    d, cleared = oracle.direction(g, s[None], y[None], P)
    assert cleared
    assert np.array_equal(d, -g * (PD["delta0"] / np.abs(g).max()))


def test_direction_cap_in_infinity_norm(oracle_lib):
    """A pair of tiny curvature gives a direction far longer than the cap:
    it is scaled (not clipped) to |d|_inf = step_max.  Catches: a 2-norm
    cap, clipping per element, or no cap."""
    rng = np.random.default_rng(32)
    n = 12
    g = rng.normal(size=n)
    S = rng.normal(size=(2, n))
    Y = 1e-3 * S + 1e-5 * rng.normal(size=(2, n))
    raw = _textbook_direction(g, S, Y)
    assert float(g @ raw) < 0 and np.abs(raw).max() > 10 * PD["step_max"]
    d, cleared = oracle.direction(g, S, Y, P)
    assert not cleared
    assert np.abs(d).max() == pytest.approx(PD["step_max"], rel=1e-12)
    assert np.abs(d - raw * (PD["step_max"] / np.abs(raw).max())).max() < 1e-12
    assert np.linalg.norm(d) > PD["step_max"] * 1.2          # the 2-norm differs


def test_direction_below_cap_is_untouched(oracle_lib):
    """A well-scaled pair gives a direction below the cap: it equals the
    dense BFGS direction (no scaling).  Catches: a cap applied always."""
    rng = np.random.default_rng(33)
    n = 12
    A = np.diag(np.linspace(1.0, 4.0, n))
    g = 0.05 * rng.normal(size=n)
    S = 0.1 * rng.normal(size=(3, n))
    Y = S @ A
    raw = _textbook_direction(g, S, Y)
    assert np.abs(raw).max() < PD["step_max"]
    d, _ = oracle.direction(g, S, Y, P)
    assert np.abs(d - raw).max() < 1e-13


# --------------------------------------------------------------- eviction --

@pytest.mark.parametrize("m", [2, 3, 5])
def test_history_keeps_newest_m_pairs(oracle_lib, m):
    """On a quadratic every accepted step pushes a pair; once more than m
    have been pushed, the direction at iteration k must equal the dense
    BFGS direction built from the newest m pairs.  Catches: evicting the
    newest pair, keeping m + 1 pairs, or a ring read in the wrong order."""
    rng = np.random.default_rng(40 + m)
    n = 14
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(np.geomspace(1.0, 30.0, n)) @ Q.T
    b = rng.normal(size=n)
    f = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    pl = params.as_list({"history": m, "step_max": 1e9})
    iters = m + 6
    tr = oracle.minimize_trace(f, np.zeros(n), iters, pl)
    assert np.all(tr["alpha"] > 0) and np.all(tr["pushed"] == 1)
    assert tr["count"].tolist() == [min(k + 1, m) for k in range(iters)]
    checked = 0
    for k in range(m + 1, iters):
        pairs = list(range(k - m, k))               # iterations whose pairs are kept
        S = np.array([tr["x"][i + 1] - tr["x"][i] for i in pairs])
        Y = np.array([tr["g"][i + 1] - tr["g"][i] for i in pairs])
        exp = _textbook_direction(tr["g"][k], S, Y)
        assert np.abs(tr["d"][k] - exp).max() <= 1e-9 * np.abs(exp).max(), k
        # with the oldest pair kept instead of the newest, it would differ
        S2 = np.array([tr["x"][i + 1] - tr["x"][i] for i in range(k - m - 1, k - 1)])
        Y2 = np.array([tr["g"][i + 1] - tr["g"][i] for i in range(k - m - 1, k - 1)])
        wrong = _textbook_direction(tr["g"][k], S2, Y2)
        assert np.abs(wrong - exp).max() > 1e-6 * np.abs(exp).max()
        checked += 1
    assert checked >= 3


# ----------------------------------------------------------------- metrics --

@pytest.fixture(scope="module")
def free_oracle():
    return oracle.Oracle(configs.robot("A"), gen.empty_scene(), P)


def _traj(T, fn, joint=2):
    X = np.zeros((1, T, 7))
    X[0, :, joint] = [fn(t) for t in range(T)]
    return X


def test_max_jerk_of_a_cubic(free_oracle):
    """q_t = c t^3 has the constant third difference 6c: max jerk is
    6|c| / dt^3.  Catches: dividing by dt^2, or a wrong stencil."""
    c, T, dt = -0.0011, 20, PD["dt"]
    r = free_oracle.results(np.zeros(7), np.array([0.3, 0, 0.4, 1, 0, 0, 0.0]),
                            _traj(T, lambda t: c * t ** 3))
    assert r["max_jerk"][0] == pytest.approx(6 * abs(c) / dt ** 3, rel=1e-9)


def test_max_velocity_and_acceleration_closed_forms(free_oracle):
    """Ramp q_t = v t: max velocity |v|/dt, zero acceleration.  Parabola
    q_t = a t^2: max acceleration 2|a|/dt^2 and max velocity
    |a|(2T - 3)/dt (the last step).  Catches: a missing 1/dt (or 1/dt^2), a
    centred instead of forward difference, or the first step instead of the
    largest."""
    dt, T = PD["dt"], 24
    goal = np.array([0.3, 0, 0.4, 1, 0, 0, 0.0])
    r = free_oracle.results(np.zeros(7), goal, _traj(T, lambda t: -0.07 * t))
    assert r["max_vel"][0] == pytest.approx(0.07 / dt, rel=1e-9)
    assert r["max_acc"][0] < 1e-9
    a = 0.0013
    r = free_oracle.results(np.zeros(7), goal, _traj(T, lambda t: a * t * t))
    assert r["max_acc"][0] == pytest.approx(2 * a / dt ** 2, rel=1e-9)
    assert r["max_vel"][0] == pytest.approx(a * (2 * T - 3) / dt, rel=1e-9)


def test_motion_time_closed_forms(free_oracle):
    """A ramp slower than every limit takes (T-1) dt.  A ramp of total
    travel D faster than the velocity limit takes D / v_limit (the time to
    cover D at the limit) and is flagged over the velocity limit.  Catches:
    scaling the time by the wrong power of the violation, or the flag on
    the wrong side."""
    dt, T = PD["dt"], 32
    goal = np.array([0.3, 0, 0.4, 1, 0, 0, 0.0])
    slow = 0.5 * PD["v_limit"] * dt
    r = free_oracle.results(np.zeros(7), goal, _traj(T, lambda t: slow * t))
    assert r["motion_time"][0] == pytest.approx((T - 1) * dt, rel=1e-12)
    assert r["within_vel"][0] == 1
    fast = 3.0 * PD["v_limit"] * dt
    r = free_oracle.results(np.zeros(7), goal, _traj(T, lambda t: fast * t))
    assert r["within_vel"][0] == 0
    assert r["motion_time"][0] == pytest.approx((T - 1) * fast / PD["v_limit"], rel=1e-9)
    # an acceleration-bound parabola: the time scale is sqrt(max_acc / a_limit)
    a = 4.0 * PD["a_limit"] * dt * dt / 2.0          # max_acc = 4 a_limit
    r = free_oracle.results(np.zeros(7), goal, _traj(T, lambda t: a * t * t * 1e-3))
    acc = r["max_acc"][0]
    vel = r["max_vel"][0]
    exp = max(1.0, vel / PD["v_limit"], math.sqrt(acc / PD["a_limit"])) * (T - 1) * dt
    assert r["motion_time"][0] == pytest.approx(exp, rel=1e-12)


# ----------------------------------------------------------- ambiguity ----

H_VOX = 2.0 ** -6                 # exactly representable spacing and origin
DIMS = (40, 40, 40)
ORIGIN = np.array([-20 * H_VOX] * 3, dtype=np.float32)
A_OFF = 0.1                       # sphere offset along link-1 x
KL, KR, D0 = 0.3, -0.2, 0.03       # field slopes left / right of x = 0, value at x = 0
R_SPH = 0.02


def _kink_oracle():
    """One sphere on link 1 at (a, 0, h/2) in the link frame (joint 1 at
    the base, so its centre is (a cos q1, a sin q1, h/2)); a field that
    depends on x only, with slope KL for x < 0 and KR for x > 0 and a kink at
    the node plane x = 0."""
    base = configs.robot("A")
    rb = gen.Robot(base.link_lengths, base.frames, base.q_lo, base.q_hi,
                   np.array([1], dtype=np.int32),
                   np.array([[A_OFF, 0.0, H_VOX / 2]], dtype=np.float32),
                   np.array([R_SPH], dtype=np.float32))
    xs = ORIGIN[0] + np.arange(DIMS[0]) * H_VOX
    d = np.where(xs < 0, D0 + KL * xs, D0 + KR * xs)
    grid = np.broadcast_to(d[None, None, :], DIMS[::-1]).astype(np.float32).copy()
    sc = gen.Scene(np.zeros((0, 3)), np.zeros((0, 3)), DIMS, H_VOX, ORIGIN, grid)
    pl = params.as_list({"lambda_v": 0, "lambda_a": 0, "lambda_j": 0, "w_pos": 0, "w_rot": 0,
                         "w_limit": 0})
    return oracle.Oracle(rb, sc, pl)


def _X(q1):
    X = np.zeros((2, 7))
    X[1, 0] = q1
    return X


def test_ambiguity_bound_covers_the_one_sided_jump(oracle_lib):
    """At q1 = pi/2 the sphere centre sits on the kink's node plane.  The
    gradient w.r.t. q1 taken just left and just right of it differs by the
    closed form w_c |phi'(D)| |KL - KR| a (the Jacobian of c_x w.r.t. q1 is
    -a there); the bound is that jump times sqrt(3) (it bounds the 3-vector
    difference by its largest component), on row 1, joint 1 only.
    Catches: a bound without the hinge slope, without the Jacobian, built
    from the wrong neighbour cell, or on the wrong joint."""
    O = _kink_oracle()
    eps = PD["eps"]
    D = D0 - float(np.float32(R_SPH))
    dphi = abs((D - eps) / eps)
    jump_closed = PD["w_collision"] * dphi * abs(KL - KR) * A_OFF
    qs = np.zeros(7)
    goal = np.array([0.3, 0, 0.4, 1, 0, 0, 0.0])
    delta = 1e-9
    gl = O.cost(qs, goal, _X(math.pi / 2 + delta), grad=True)["G"][0]   # c_x < 0: left cell
    gr = O.cost(qs, goal, _X(math.pi / 2 - delta), grad=True)["G"][0]   # c_x > 0: right cell
    jump = abs(gl[1, 0] - gr[1, 0])
    assert jump == pytest.approx(jump_closed, rel=1e-6)
    amb, n = O.ambiguity(_X(math.pi / 2))
    assert n == 1
    assert amb[1, 0] == pytest.approx(math.sqrt(3.0) * jump_closed, rel=1e-6)
    assert np.all(amb[1, 1:] == 0) and np.all(amb[0] == 0)


def test_ambiguity_bound_zero_away_from_faces(oracle_lib):
    """With the centre well inside a cell on every axis the bound is zero
    and no sample is counted ambiguous.  Catches: a face test on the wrong
    quantity (metres instead of voxels) or one that is always true."""
    O = _kink_oracle()
    for q1 in (math.pi / 2 - 0.05, math.pi / 2 + 0.031, 1.0, 2.0):
        c = np.array([A_OFF * math.cos(q1), A_OFF * math.sin(q1), H_VOX / 2])
        u = (c - ORIGIN.astype(np.float64)) / H_VOX
        assert np.min(np.abs(u - np.round(u))) > 0.05
        amb, n = O.ambiguity(_X(q1))
        assert n == 0 and np.all(amb == 0)


# ------------------------------------------------------- float32 bound ----

def _frame_motion(O, X, Y):
    """Largest displacement of any sphere centre, joint origin or the end
    effector, and largest rotation angle of any link frame, between the
    configurations of X and Y (row by row)."""
    dmax = amax = 0.0
    for t in range(X.shape[0]):
        R0, p0 = O.fk(X[t])
        R1, p1 = O.fk(Y[t])
        dmax = max(dmax, np.linalg.norm(p1 - p0, axis=1).max())
        for i in range(8):
            c = (np.trace(R0[i].T @ R1[i]) - 1.0) / 2.0
            amax = max(amax, math.acos(min(1.0, max(-1.0, c))))
    c0, c1 = O.spheres(X), O.spheres(Y)
    dmax = max(dmax, np.linalg.norm(c1 - c0, axis=-1).max())
    return dmax, amax


@pytest.mark.parametrize("key", ["B", "A"])
def test_fp32_bound_covers_kinematic_perturbations(key):
    """The float32 bound B_e is a first-order bound of how far the gradient
    moves when every centre, origin and the end effector move by at most
    delta and every frame turns by at most eta.  Moving the configuration
    by a tiny random dq does exactly that (delta, eta measured from the
    kinematics): the exact change of every gradient element must stay below
    B_e (plus the cell-face ambiguity for the few samples that cross a cell
    face), with the smoothness and limit terms off (they depend on the
    waypoints only).  The bound must also not be vacuous: below 200 x the
    largest change seen.  Catches: a dropped hinge-curvature or
    field-curvature term, a missing moment arm, or a bound that ignores the
    goal terms."""
    robot = configs.robot(key)
    sc = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    pl = params.as_list({"lambda_v": 0, "lambda_a": 0, "lambda_j": 0, "w_limit": 0})
    O = oracle.Oracle(robot, sc, pl, threads=4)
    X = configs.seeds_for(key, 0, prob, S=4).astype(np.float64)
    u = 2.0 ** -24
    rng = np.random.default_rng(90)
    worst_ratio, biggest = 0.0, 0.0
    for s in range(X.shape[0]):
        g0 = O.cost(prob.q_start, prob.goal, X[s], grad=True)["G"][0]
        for trial in range(3):
            Y = X[s].copy()
            Y[1:] += rng.uniform(-1, 1, Y[1:].shape) * 1e-5
            delta, eta = _frame_motion(O, X[s], Y)
            fb, reach = O.fp32_bound(prob.q_start, prob.goal, X[s], delta / (u * 1.0), eta / u)
            # the bound scales delta by the reach: undo it
            fb, _ = O.fp32_bound(prob.q_start, prob.goal, X[s], delta / (u * reach), eta / u)
            g1 = O.cost(prob.q_start, prob.goal, Y, grad=True)["G"][0]
            amb, _ = O.ambiguity(X[s], tol=5e-3)
            diff = np.abs(g1 - g0)
            assert np.all(diff <= 1.05 * fb + amb + 1e-9), (s, float((diff - fb - amb).max()))
            act = diff[amb == 0]
            bnd = fb[amb == 0]
            big = act > 1e-3 * act.max()
            if big.any():
                worst_ratio = max(worst_ratio, float((act[big] / bnd[big]).max()))
            biggest = max(biggest, float(act.max()))
    assert worst_ratio <= 1.05
    # not vacuous: some element's bound is within 200x of its actual change
    assert worst_ratio > 1.0 / 200.0, worst_ratio
    assert biggest > 0
