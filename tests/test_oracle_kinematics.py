"""Pins of oracle/kinematics.py: closed forms and invariants of the serial chain."""
import numpy as np

from oracle.kinematics import forward_kinematics, joint_axes, sphere_positions
from synthetic import make_configs, make_robot


def _rz(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def test_identity_fixed_transforms_give_summed_rotation():
    fixed = np.zeros((8, 3, 4))
    fixed[:, :, :3] = np.eye(3)
    q = make_configs(5, exact=True)
    T = forward_kinematics(fixed, q)
    for b in range(5):
        for j in range(1, 8):
            np.testing.assert_allclose(T[b, j, :3, :3], _rz(q[b, :j].sum()), atol=1e-14)
            np.testing.assert_allclose(T[b, j, :3, 3], 0.0, atol=0)
        np.testing.assert_allclose(T[b, 8], T[b, 7], atol=0)
    # zero configuration with identity transforms: every link pose is the identity
    T0 = forward_kinematics(fixed, np.zeros((1, 7)))
    np.testing.assert_array_equal(T0[0], np.broadcast_to(np.eye(4), (9, 4, 4)))


def test_zero_configuration_is_product_of_fixed_transforms():
    r = make_robot(exact=True)
    T = forward_kinematics(r.fixed_tf, np.zeros((1, 7)))[0]
    acc = np.eye(4)
    for j in range(8):
        Fj = np.eye(4)
        Fj[:3, :] = r.fixed_tf[j]
        acc = acc @ Fj
        np.testing.assert_allclose(T[j + 1], acc, atol=1e-14)


def test_single_joint_closed_form():
    fixed = np.zeros((8, 3, 4))
    fixed[:, :, :3] = np.eye(3)
    fixed[0, :, 3] = [0.1, -0.2, 0.3]
    q = np.zeros((1, 7))
    q[0, 0] = 0.7
    T = forward_kinematics(fixed, q)
    c = np.array([0.4, 0.0, 0.05])
    p = sphere_positions(T, c[None], np.array([1]))[0, 0]
    expect = np.array([0.1 + 0.4 * np.cos(0.7), -0.2 + 0.4 * np.sin(0.7), 0.35])
    np.testing.assert_allclose(p, expect, atol=1e-15)
    z, o = joint_axes(T)
    np.testing.assert_allclose(z[0, 0], [0, 0, 1], atol=0)
    np.testing.assert_allclose(o[0, 0], [0.1, -0.2, 0.3], atol=0)


def test_orthonormal_and_rigid():
    r = make_robot(exact=True)
    q = make_configs(64, exact=True)
    T = forward_kinematics(r.fixed_tf, q)
    R = T[:, :, :3, :3]
    err = np.einsum("blji,bljk->blik", R, R) - np.eye(3)
    assert np.abs(err).max() < 1e-12
    assert np.abs(np.linalg.det(R) - 1.0).max() < 1e-12
    P = sphere_positions(T, r.sphere_center, r.sphere_link)
    dist = np.linalg.norm(P - T[:, r.sphere_link][:, :, :3, 3], axis=-1)
    np.testing.assert_allclose(dist, np.broadcast_to(np.linalg.norm(r.sphere_center, axis=1), dist.shape),
                               rtol=1e-12, atol=1e-15)


def test_joint_only_moves_later_links():
    r = make_robot(exact=True)
    q = make_configs(4, exact=True)
    T = forward_kinematics(r.fixed_tf, q)
    for j in range(1, 8):
        q2 = q.copy()
        q2[:, j - 1] += 0.3
        T2 = forward_kinematics(r.fixed_tf, q2)
        np.testing.assert_array_equal(T2[:, :j], T[:, :j])
        assert np.all(np.abs(T2[:, j:] - T[:, j:]).max(axis=(2, 3)) > 0)
