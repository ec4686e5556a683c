"""Pins of oracle/cost.py: two independent gradient routes, finite differences, closed forms."""
import numpy as np
import pytest

from oracle import cost as C
from oracle import formats as F
from oracle.kinematics import forward_kinematics, sphere_positions
from synthetic import Robot, Worlds, make_robot, make_worlds, make_workload, make_configs


def _dense_workload(seed=0, B=24, T=4, n_ls=2):
    """A small, collision-rich problem: big cuboids so that many spheres are active."""
    robot = make_robot(52, 300, seed=seed, exact=True)
    w = make_worlds(2, 10, seed=seed, exact=True)
    w.half_ext[:] = w.half_ext * 2.0
    q = make_configs(B, seed=seed, lo=-3.2, hi=3.2, exact=True)
    return robot, w, q, T, n_ls


def test_adjoint_equals_explicit_jacobian():
    robot, w, q, T, n_ls = _dense_workload()
    o = C.fwd_bwd(robot, w, q, 3, T, n_ls)
    Ja = C.joint_grad_adjoint(o["poses"], o["S"], o["G"], robot.sphere_link)
    Jj = C.joint_grad_jacobian(o["poses"], o["S"], o["G"], robot.sphere_link)
    assert np.abs(Ja).max() > 1.0
    assert np.abs(Ja - Jj).max() <= 1e-12 * np.abs(Ja).max()


def test_joint_gradient_central_differences():
    robot, w, q, T, n_ls = _dense_workload(1)
    tpw = 3
    o = C.fwd_bwd(robot, w, q, tpw, T, n_ls)
    assert (o["D"] > 0).mean() > 0.05
    # kink margins: runner-up cuboid / inside axis gaps of active spheres, coincident pairs
    active = o["D"] > 0
    margin = np.where(active, o["margin"], np.inf).min(axis=1)
    ok_cfg = margin > 1e-4
    eps = 1e-6
    checked = 0
    for b in range(q.shape[0]):
        if not ok_cfg[b]:
            continue
        tc = b // T
        for j in range(7):
            qp, qm = q.copy(), q.copy()
            qp[b, j] += eps
            qm[b, j] -= eps
            cp = C.fwd_bwd(robot, w, qp, tpw, T, n_ls)["cost_traj"][tc]
            cm = C.fwd_bwd(robot, w, qm, tpw, T, n_ls)["cost_traj"][tc]
            fd = (cp - cm) / (2 * eps)
            assert fd == pytest.approx(o["J"][b, j], rel=1e-6, abs=1e-6), (b, j)
            checked += 1
    assert checked >= 100


def test_sphere_gradient_central_differences():
    robot, w, q, T, n_ls = _dense_workload(2, B=8)
    wid = np.zeros(8, dtype=int)
    o = C.fwd_bwd(robot, w, q, 2, T, n_ls)
    S = o["S"]
    eps = 1e-7
    active = o["D"] > 0
    ok = (o["margin"] > 1e-4) | ~active
    for b in range(2):
        for s in range(robot.n_spheres):
            if not ok[b, s]:
                continue
            for i in range(3):
                Sp, Sm = S[b:b + 1].copy(), S[b:b + 1].copy()
                Sp[0, s, i] += eps
                Sm[0, s, i] -= eps
                fd = (C.sphere_cost(robot, w, Sp, wid[:1], C.CostParams())
                      - C.sphere_cost(robot, w, Sm, wid[:1], C.CostParams()))[0] / (2 * eps)
                assert fd == pytest.approx(o["G"][b, s, i], rel=1e-5, abs=1e-5)


def test_single_sphere_hand_case():
    # one sphere of radius 0.05 at x = 0.11 in front of an axis-aligned box of half extent 0.1:
    # clearance 0.11 - 0.1 - 0.05 = -0.04, depth d = 0.02 + 0.04 = 0.06, cost 100 * 0.06^2 = 0.36,
    # gradient -2 * 100 * 0.06 * e_x = -12 e_x
    pose = np.zeros((1, 1, 3, 4))
    pose[0, 0, :, :3] = np.eye(3)
    half = np.full((1, 1, 3), 0.1)
    S = np.array([[[0.11, 0.0, 0.0]]])
    d, g, k, _ = C.world_term(S, np.array([0.05]), pose, half, np.zeros(1, dtype=int), 0.02)
    assert d[0, 0] == pytest.approx(0.06, abs=1e-15)
    np.testing.assert_allclose(-2 * 100 * d[0, 0] * g[0, 0], [-12.0, 0, 0], atol=1e-12)


def test_self_pair_closed_form():
    S = np.array([[[0.0, 0.0, 0.0], [0.07, 0.0, 0.0], [1.0, 1.0, 1.0]]])
    r = np.array([0.03, 0.05, 0.04])
    pairs = np.array([[0, 1], [0, 2]], dtype=np.int32)
    cost, grad, mind = C.self_term(S, r, pairs, 0.02)
    # e = 0.07 - 0.08 = -0.01 -> act 0.03 -> cost 9e-4; second pair inactive
    assert cost[0] == pytest.approx(9e-4, abs=1e-17)
    np.testing.assert_allclose(grad[0, 0], [2 * 0.03, 0, 0], atol=1e-15)
    np.testing.assert_allclose(grad[0, 1], [-2 * 0.03, 0, 0], atol=1e-15)
    np.testing.assert_allclose(grad[0, 2], 0.0, atol=0)
    # coincident centres: gradient zero, cost counted
    S2 = np.zeros((1, 2, 3))
    c2, g2, _ = C.self_term(S2, r[:2], pairs[:1], 0.02)
    assert c2[0] == pytest.approx(0.1 ** 2)
    assert np.all(g2 == 0)


def test_bound_and_smoothness_gradients_fd():
    q = np.random.default_rng(3).uniform(-3.3, 3.3, size=(12, 7))
    lo, hi = np.full(7, -2.9), np.full(7, 2.9)
    c, g = C.bound_term(q, lo, hi)
    v, gs = C.smoothness_grad(q, 4, 1)
    eps = 1e-6
    for b in range(12):
        for j in range(7):
            qp, qm = q.copy(), q.copy()
            qp[b, j] += eps
            qm[b, j] -= eps
            fd = (C.bound_term(qp, lo, hi)[0][b] - C.bound_term(qm, lo, hi)[0][b]) / (2 * eps)
            assert fd == pytest.approx(g[b, j], abs=1e-7)
            fs = (C.smoothness_grad(qp, 4, 1)[0] - C.smoothness_grad(qm, 4, 1)[0]).sum() / (2 * eps)
            assert fs == pytest.approx(gs[b, j], abs=1e-6)


def test_f32_emulation_is_fp32_rounding_only():
    wl = make_workload("tiny", exact=False)
    truth = C.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls)
    emu = C.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls, prec=C.Precision())
    np.testing.assert_allclose(emu["cost_traj"], truth["cost_traj"], rtol=1e-6)
    np.testing.assert_allclose(emu["J"], truth["J"], rtol=1e-5, atol=1e-5)
    assert np.array_equal(emu["S_codes"], F.fp32(truth["S"]).view(np.uint32))


def test_quantised_tensors_take_format_values():
    robot, w, q, T, n_ls = _dense_workload(4, B=8)
    prec = C.Precision(link_poses=("e4m3", -5), sphere_pos=("bf16", 0), sphere_dist=("e2m1", -4),
                       sphere_grad=("e3m2", 0), joint_grad=("e5m2", 0))
    o = C.fwd_bwd(robot, w, q, 2, T, n_ls, prec=prec)
    vals = F.magnitude_table("e2m1")[1] * 2.0 ** -4
    assert np.all(np.isin(np.abs(o["D_hat"]), vals))
    assert np.all(np.isin(np.abs(o["G_hat"]), F.magnitude_table("e3m2")[1]))
    # the cost is aggregated from the stored distances
    np.testing.assert_allclose(o["cfg_cost"], 100 * np.sum(o["D_hat"] ** 2, axis=1) + o["self_cost"]
                               + 10 * o["bound_cost"], rtol=1e-15)
    # stored mode rebuilds poses from quantised L, recompute mode does not
    o2 = C.fwd_bwd(robot, w, q, 2, T, n_ls, prec=C.Precision(**{**prec.__dict__, "recompute_poses": True}))
    assert o2["L_codes"] is None
    assert not np.allclose(o2["J"], o["J"])
