"""Pins of the oracle's swept collision term (oracle/cost.py: swept_term and its use in fwd_bwd):
a hand-computed segment, the static-trajectory reduction to the discrete world term, segments that
must not join two trajectory-candidates, central differences of the swept sum w.r.t. the sphere
centres, and the joint gradient through kinematics with the term switched on."""
import numpy as np
import pytest

from oracle import cost as C
from synthetic import Robot, Worlds, make_configs, make_robot, make_worlds


def _unit_box_world():
    """One world holding one axis-aligned cube of half extent 0.5 centred at the origin."""
    pose = np.zeros((1, 1, 3, 4))
    pose[0, 0, :, :3] = np.eye(3)
    return pose, np.full((1, 1, 3), 0.5)


def test_hand_computed_segment():
    # sphere of radius 0.1 moving from x = 0.6 to x = 1.0 beside the cube, k = 3, eta = 0.25:
    # samples x = 0.7, 0.8, 0.9 -> sd 0.2, 0.3, 0.4 -> clearance 0.1, 0.2, 0.3 -> d 0.15, 0.05, 0
    pose, half = _unit_box_world()
    S = np.array([[[0.6, 0.0, 0.0]], [[1.0, 0.0, 0.0]]])
    cost, X, _ = C.swept_term(S, np.array([0.1]), pose, half, np.zeros(2, dtype=int), 0.25, T=2, k=3)
    assert cost[0] == pytest.approx((0.15 ** 2 + 0.05 ** 2) / 3, abs=1e-15)
    assert cost[1] == 0.0
    # d/dp(t): weights 1 - u = 0.75, 0.5, 0.25; d/dp(t+1): u = 0.25, 0.5, 0.75; grad of sd = +x
    assert X[0, 0] == pytest.approx([-(2 / 3) * (0.75 * 0.15 + 0.5 * 0.05), 0.0, 0.0], abs=1e-15)
    assert X[1, 0] == pytest.approx([-(2 / 3) * (0.25 * 0.15 + 0.5 * 0.05), 0.0, 0.0], abs=1e-15)


def test_static_trajectory_reduces_to_the_discrete_term():
    """Every sample of a segment between equal positions is that position, so the mean over the k
    samples is the discrete activation depth squared; the last timestep has no segment."""
    robot = make_robot(40, 0, seed=3, exact=True)
    w = make_worlds(1, 12, seed=3, exact=True)
    w.half_ext[:] = w.half_ext * 2.0
    T = 5
    S0 = np.random.default_rng(0).uniform(-0.6, 0.6, size=(1, robot.sphere_radius.size, 3))
    S = np.repeat(S0, T, axis=0)
    wid = np.zeros(T, dtype=int)
    d, _, _, _ = C.world_term(S, robot.sphere_radius, w.pose, w.half_ext, wid, 0.02)
    assert (d > 0).any()
    for k in (1, 4):
        cost, X, _ = C.swept_term(S, robot.sphere_radius, w.pose, w.half_ext, wid, 0.02, T, k)
        np.testing.assert_allclose(cost[:-1], np.sum(d[:-1] ** 2, axis=1), rtol=1e-13, atol=0)
        assert cost[-1] == 0.0


def test_segments_do_not_join_trajectory_candidates():
    """Two 2-step trajectories on either side of the cube: the last point of the first and the
    first point of the second are joined by a line through the cube, which must not count."""
    pose, half = _unit_box_world()
    S = np.array([[[-2.0, 0.0, 0.0]], [[-1.0, 0.0, 0.0]], [[1.0, 0.0, 0.0]], [[2.0, 0.0, 0.0]]])
    cost, X, _ = C.swept_term(S, np.array([0.1]), pose, half, np.zeros(4, dtype=int), 0.02, T=2, k=4)
    assert np.all(cost == 0.0) and np.all(X == 0.0)
    # the same four points as one trajectory do cross it
    cost1, _, _ = C.swept_term(S, np.array([0.1]), pose, half, np.zeros(4, dtype=int), 0.02, T=4, k=4)
    assert cost1[1] > 0.0


def test_swept_gradient_central_differences():
    robot = make_robot(20, 0, seed=5, exact=True)
    w = make_worlds(1, 8, seed=5, exact=True)
    w.half_ext[:] = w.half_ext * 2.5
    T, k, eta = 4, 3, 0.05
    rng = np.random.default_rng(5)
    S = rng.uniform(-0.7, 0.7, size=(2 * T, robot.sphere_radius.size, 3))
    wid = np.zeros(2 * T, dtype=int)
    cost, X, margin = C.swept_term(S, robot.sphere_radius, w.pose, w.half_ext, wid, eta, T, k)
    assert (np.abs(X) > 0).sum() > 20

    def total(Sx):
        return C.swept_term(Sx, robot.sphere_radius, w.pose, w.half_ext, wid, eta, T, k)[0].sum()

    h = 1e-7
    checked = 0
    for b in range(2 * T):
        if margin[b] < 1e-4:
            continue
        for s in range(robot.sphere_radius.size):
            for c in range(3):
                Sp, Sm = S.copy(), S.copy()
                Sp[b, s, c] += h
                Sm[b, s, c] -= h
                fd = (total(Sp) - total(Sm)) / (2 * h)
                assert fd == pytest.approx(X[b, s, c], rel=1e-5, abs=1e-7), (b, s, c)
                checked += 1
    assert checked >= 200


def test_joint_gradient_with_swept_term_central_differences():
    """fwd_bwd with the swept term: the joint gradient (adjoint of G + X) against central
    differences of the trajectory cost through kinematics."""
    robot = make_robot(52, 300, seed=7, exact=True)
    w = make_worlds(2, 10, seed=7, exact=True)
    w.half_ext[:] = w.half_ext * 2.0
    T, n_ls, tpw = 4, 1, 3
    B = 2 * tpw * T
    rng = np.random.default_rng(7)
    # smooth trajectories, so that segments are short and the sweep stays near the waypoints
    start = rng.uniform(-2.5, 2.5, size=(2 * tpw, 1, 7))
    step = rng.uniform(-0.2, 0.2, size=(2 * tpw, 1, 7))
    q = (start + step * np.arange(T)[None, :, None]).reshape(B, 7)
    params = C.CostParams(swept_steps=3, w_swept=50.0)
    o = C.fwd_bwd(robot, w, q, tpw, T, n_ls, params=params)
    assert np.abs(o["X"]).max() > 0.0
    active = o["D"] > 0
    margin = np.minimum(np.where(active, o["margin"], np.inf).min(axis=1), o["swept_margin"])
    eps = 1e-6
    checked = 0
    for b in range(B):
        if margin[b] < 1e-4 or (b > 0 and margin[b - 1] < 1e-4) or (b + 1 < B and margin[b + 1] < 1e-4):
            continue
        tc = b // T
        for j in range(7):
            qp, qm = q.copy(), q.copy()
            qp[b, j] += eps
            qm[b, j] -= eps
            cp = C.fwd_bwd(robot, w, qp, tpw, T, n_ls, params=params)["cost_traj"][tc]
            cm = C.fwd_bwd(robot, w, qm, tpw, T, n_ls, params=params)["cost_traj"][tc]
            assert (cp - cm) / (2 * eps) == pytest.approx(o["J"][b, j], rel=1e-6, abs=1e-6), (b, j)
            checked += 1
    assert checked >= 70


def test_swept_off_leaves_fwd_bwd_unchanged():
    robot = make_robot(30, 50, seed=9, exact=True)
    w = make_worlds(1, 6, seed=9, exact=True)
    q = make_configs(8, seed=9, exact=True)
    a = C.fwd_bwd(robot, w, q, 2, 4, 1)
    b = C.fwd_bwd(robot, w, q, 2, 4, 1, params=C.CostParams(swept_steps=0, w_swept=1e6))
    assert np.array_equal(a["cost_traj"], b["cost_traj"]) and np.array_equal(a["J"], b["J"])
    assert "X" not in b
