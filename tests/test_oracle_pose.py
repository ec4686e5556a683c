"""Pins of the oracle's pose (goal) cost for inverse kinematics (oracle/cost.py: pose_term and its
use in fwd_bwd): zero at the goal, closed forms for a pure offset and a pure rotation, the
end-effector wrench route against the matrix chain rule, and central differences."""
import numpy as np
import pytest

from oracle import cost as C
from oracle.kinematics import forward_kinematics
from synthetic import make_configs, make_robot, make_worlds


def _axis_angle(axis, theta):
    a = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(theta) * K + (1 - np.cos(theta)) * K @ K


def _goal_of(T):
    return T[:, 8, :3, :].copy()


def test_zero_cost_and_gradient_at_the_goal():
    robot = make_robot(20, 0, seed=1, exact=True)
    q = make_configs(6, seed=1, exact=True)
    T = forward_kinematics(robot.fixed_tf, q)
    cost, F, tau = C.pose_term(T, _goal_of(T), 100.0, 10.0)
    assert np.abs(cost).max() < 1e-24
    assert np.abs(C.pose_grad_adjoint(T, F, tau)).max() < 1e-12


def test_closed_forms_offset_and_rotation():
    robot = make_robot(20, 0, seed=2, exact=True)
    q = make_configs(4, seed=2, exact=True)
    T = forward_kinematics(robot.fixed_tf, q)
    g = _goal_of(T)
    delta = np.array([0.03, -0.1, 0.2])
    g_off = g.copy()
    g_off[:, :, 3] += delta
    cost, _, _ = C.pose_term(T, g_off, 7.0, 3.0)
    np.testing.assert_allclose(cost, 7.0 * np.sum(delta * delta), rtol=1e-12)
    # goal rotation R_g = R Q with Q a rotation by theta: ||R - R Q||^2 = 6 - 2 tr(Q) = 4 (1 - cos theta)
    theta = 0.7
    Q = _axis_angle([1.0, 2.0, -0.5], theta)
    g_rot = g.copy()
    g_rot[:, :, :3] = T[:, 8, :3, :3] @ Q
    cost, _, _ = C.pose_term(T, g_rot, 7.0, 3.0)
    np.testing.assert_allclose(cost, 3.0 * 4.0 * (1.0 - np.cos(theta)), rtol=1e-12)


def test_wrench_route_equals_matrix_chain_rule():
    robot = make_robot(20, 0, seed=3, exact=True)
    q = make_configs(16, seed=3, exact=True)
    T = forward_kinematics(robot.fixed_tf, q)
    rng = np.random.default_rng(3)
    goal = np.zeros((16, 3, 4))
    for b in range(16):
        goal[b, :, :3] = _axis_angle(rng.normal(size=3), rng.uniform(0, 3))
    goal[:, :, 3] = rng.uniform(-1, 1, size=(16, 3))
    _, F, tau = C.pose_term(T, goal, 50.0, 5.0)
    a = C.pose_grad_adjoint(T, F, tau)
    e = C.pose_grad_explicit(T, goal, 50.0, 5.0)
    assert np.abs(a).max() > 1.0
    assert np.abs(a - e).max() <= 1e-12 * np.abs(a).max()


def test_pose_gradient_central_differences():
    robot = make_robot(20, 0, seed=4, exact=True)
    q = make_configs(5, seed=4, exact=True)
    rng = np.random.default_rng(4)
    goal = np.zeros((5, 3, 4))
    for b in range(5):
        goal[b, :, :3] = _axis_angle(rng.normal(size=3), rng.uniform(0, 3))
    goal[:, :, 3] = rng.uniform(-1, 1, size=(5, 3))

    def cost(qq):
        return C.pose_term(forward_kinematics(robot.fixed_tf, qq), goal, 20.0, 4.0)[0]

    _, F, tau = C.pose_term(forward_kinematics(robot.fixed_tf, q), goal, 20.0, 4.0)
    g = C.pose_grad_adjoint(forward_kinematics(robot.fixed_tf, q), F, tau)
    h = 1e-6
    for j in range(7):
        qp, qm = q.copy(), q.copy()
        qp[:, j] += h
        qm[:, j] -= h
        np.testing.assert_allclose((cost(qp) - cost(qm)) / (2 * h), g[:, j], rtol=1e-6, atol=1e-6)


def test_fwd_bwd_with_goals_joint_gradient_central_differences():
    """IK layout (one timestep per trajectory): pose, collision, self and bound costs together."""
    robot = make_robot(52, 300, seed=5, exact=True)
    w = make_worlds(2, 10, seed=5, exact=True)
    tpw, T, n_ls = 6, 1, 1
    B = 2 * tpw
    q = make_configs(B, seed=5, exact=True)
    rng = np.random.default_rng(5)
    goals = np.zeros((2, 3, 4))
    for k in range(2):
        goals[k, :, :3] = _axis_angle(rng.normal(size=3), rng.uniform(0, 3))
    goals[:, :, 3] = rng.uniform(-0.6, 0.6, size=(2, 3))
    params = C.CostParams(w_goal_pos=30.0, w_goal_rot=3.0)
    o = C.fwd_bwd(robot, w, q, tpw, T, n_ls, params=params, goals=goals)
    assert np.all(o["pose_cost"] > 0)
    active = o["D"] > 0
    margin = np.where(active, o["margin"], np.inf).min(axis=1)
    eps = 1e-6
    checked = 0
    for b in range(B):
        if margin[b] < 1e-4:
            continue
        for j in range(7):
            qp, qm = q.copy(), q.copy()
            qp[b, j] += eps
            qm[b, j] -= eps
            cp = C.fwd_bwd(robot, w, qp, tpw, T, n_ls, params=params, goals=goals)["cost_traj"][b]
            cm = C.fwd_bwd(robot, w, qm, tpw, T, n_ls, params=params, goals=goals)["cost_traj"][b]
            assert (cp - cm) / (2 * eps) == pytest.approx(o["J"][b, j], rel=1e-6, abs=1e-6), (b, j)
            checked += 1
    assert checked >= 56
