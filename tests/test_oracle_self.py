"""Pins of the oracle's self-collision term (C_self of App. A.6; pairs of
spheres on links at least two apart, smooth hinge on their separation):
a hand-derived two-sphere case, exclusion of adjacent links, invariance
under rotation of the base joint, and central differences."""
import math

import numpy as np
import pytest

import oracle
from workloads import configs, gen, params

PD = params.DEFAULT


def robot_with(spheres):
    """Synthetic arm with an explicit sphere list [(link, (ox, oy, oz), r)]."""
    base = configs.robot("A")
    return gen.Robot(base.link_lengths, base.frames, base.q_lo, base.q_hi,
                     np.array([s[0] for s in spheres], dtype=np.int32),
                     np.array([s[1] for s in spheres], dtype=np.float32),
                     np.array([s[2] for s in spheres], dtype=np.float32))


def fat_robot():
    """The cluttered workload's arm with radii doubled: random
    configurations then always have some self-contact."""
    rb = configs.robot("B")
    return gen.Robot(rb.link_lengths, rb.frames, rb.q_lo, rb.q_hi, rb.sphere_link,
                     rb.sphere_offset, (rb.sphere_radius * 2).astype(np.float32))


def self_only(w=50.0):
    return params.as_list({"w_collision": 0.0, "lambda_v": 0.0, "lambda_a": 0.0,
                           "lambda_j": 0.0, "w_pos": 0.0, "w_rot": 0.0, "w_limit": 0.0,
                           "w_self": w})


def terms(rb, X, p):
    O = oracle.Oracle(rb, gen.empty_scene(), p)
    return O, O.cost(np.zeros(7), np.array([0, 0, 0, 1, 0, 0, 0.0]), X, grad=True, terms=True)


def test_two_sphere_closed_form(oracle_lib):
    """One sphere at joint 1's origin (link 1), one at joint 3's origin
    (link 3).  At q = 0 joint 3 sits at (0, L2, L1) (the zig-zag of the
    kinematics pin), so D = sqrt(L1^2 + L2^2) - r1 - r3."""
    L = configs.robot("A").link_lengths.astype(np.float32).astype(np.float64)
    dist = math.hypot(L[0], L[1])
    for gap in (-0.05, 0.005, 0.015, 0.05):
        r = np.float32((dist - gap) / 2)
        rb = robot_with([(1, (0, 0, 0), r), (3, (0, 0, 0), r)])
        _, c = terms(rb, np.zeros((1, 4, 7)), self_only())
        D = dist - 2 * float(r)
        exp = 4 * 50.0 * oracle.hinge(D, PD["eps"])[0]    # 4 waypoints
        assert c["terms"][0][7] == pytest.approx(exp, rel=1e-9, abs=1e-12)


def test_adjacent_links_are_excluded(oracle_lib):
    rb = robot_with([(1, (0, 0, 0.05), 0.3), (2, (0, 0, 0.0), 0.3)])
    X = np.random.default_rng(1).uniform(-2, 2, (2, 5, 7))
    _, c = terms(rb, X, self_only())
    assert np.all(c["terms"][:, 7] == 0.0)
    rb2 = robot_with([(1, (0, 0, 0.05), 0.3), (2, (0, 0, 0.0), 0.3), (3, (0, 0, 0.0), 0.3)])
    _, c2 = terms(rb2, X, self_only())
    assert np.all(c2["terms"][:, 7] > 0.0)


def test_invariant_under_base_rotation(oracle_lib):
    rb = fat_robot()
    rng = np.random.default_rng(2)
    X = rng.uniform(-2.8, 2.8, (4, 6, 7))
    Y = X.copy()
    Y[:, :, 0] += rng.uniform(-1, 1, (4, 1))
    _, a = terms(rb, X, self_only())
    _, b = terms(rb, Y, self_only())
    assert np.all(a["terms"][:, 7] > 0)
    assert np.allclose(a["terms"][:, 7], b["terms"][:, 7], rtol=1e-10)
    # and the base joint gets no self-collision gradient
    assert np.abs(a["G"][:, :, 0]).max() < 1e-9 * np.abs(a["G"]).max()


def test_gradient_matches_central_differences(oracle_lib):
    rb = fat_robot()
    rng = np.random.default_rng(3)
    X = rng.uniform(-2.8, 2.8, (3, 6, 7))
    O, c = terms(rb, X, self_only())
    assert np.all(c["terms"][:, 7] > 0)
    for s in range(3):
        idx = np.arange(7, 6 * 7)
        fd = O.fd_grad(np.zeros(7), np.array([0, 0, 0, 1, 0, 0, 0.0]), X[s], idx, h=1e-6)
        an = c["G"][s].reshape(-1)[idx]
        assert np.abs(fd - an).max() < 1e-6 * max(1.0, np.abs(an).max())
