"""Pins of oracle/geometry.py: brute-force surface sampling, special cases, invariance, gradient."""
import numpy as np
import pytest

from oracle.geometry import obb_signed_distance
from synthetic.generators import _random_rotations


def _box(seed):
    rng = np.random.default_rng(seed)
    R = _random_rotations(rng, 1)[0]
    c = rng.uniform(-0.5, 0.5, 3)
    h = rng.uniform(0.025, 0.25, 3)
    return R, c, h


def _surface_samples(R, c, h, n=400):
    """Points on the six faces on an n x n grid each (box frame -> world)."""
    g = np.linspace(-1.0, 1.0, n)
    A, Bm = np.meshgrid(g, g, indexing="ij")
    pts = []
    for ax in range(3):
        o1, o2 = [i for i in range(3) if i != ax]
        for sgn in (-1.0, 1.0):
            u = np.zeros((n * n, 3))
            u[:, ax] = sgn * h[ax]
            u[:, o1] = A.ravel() * h[o1]
            u[:, o2] = Bm.ravel() * h[o2]
            pts.append(u)
    u = np.concatenate(pts)
    return u @ R.T + c, u


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_surface_sampling(seed):
    R, c, h = _box(seed)
    surf, _ = _surface_samples(R, c, h)
    spacing = np.sqrt(2.0) * 2.0 * h.max() / 399
    rng = np.random.default_rng(100 + seed)
    pts = c + rng.normal(size=(40, 3)) * 0.3
    sd, _, _ = obb_signed_distance(pts, R, c, h)
    for p, s in zip(pts, sd):
        dmin = np.min(np.linalg.norm(surf - p, axis=1))
        inside = np.all(np.abs((p - c) @ R) <= h)
        ref = -dmin if inside else dmin
        assert abs(s - ref) <= spacing, (s, ref)


def test_special_points():
    R, c, h = _box(7)
    sd, _, _ = obb_signed_distance(c[None], R, c, h)
    assert sd[0] == pytest.approx(-h.min(), abs=1e-15)
    face = c + R @ np.array([h[0], 0.3 * h[1], -0.2 * h[2]])
    sd, g, _ = obb_signed_distance(face[None], R, c, h)
    assert abs(sd[0]) < 1e-15
    np.testing.assert_allclose(g[0], R[:, 0], atol=1e-15)


def test_axis_aligned_textbook():
    h = np.array([0.1, 0.2, 0.3])
    rng = np.random.default_rng(8)
    pts = rng.uniform(-0.6, 0.6, size=(500, 3))
    sd, _, _ = obb_signed_distance(pts, np.eye(3), np.zeros(3), h)
    closest = np.clip(pts, -h, h)
    outside = np.linalg.norm(pts - closest, axis=1)
    inside = -np.min(h - np.abs(pts), axis=1)
    ref = np.where(outside > 0, outside, inside)
    np.testing.assert_allclose(sd, ref, atol=1e-15)


def test_rotation_invariance():
    R, c, h = _box(9)
    Q = _random_rotations(np.random.default_rng(10), 1)[0]
    pts = np.random.default_rng(11).normal(size=(100, 3)) * 0.4
    sd, g, _ = obb_signed_distance(pts, R, c, h)
    sd2, g2, _ = obb_signed_distance(pts @ Q.T, Q @ R, Q @ c, h)
    np.testing.assert_allclose(sd2, sd, atol=1e-14)
    np.testing.assert_allclose(g2, g @ Q.T, atol=1e-13)


def test_gradient_central_differences():
    R, c, h = _box(12)
    pts = c + np.random.default_rng(13).normal(size=(300, 3)) * 0.3
    sd, g, gap = obb_signed_distance(pts, R, c, h)
    ok = (gap > 1e-4) & (np.abs(sd) > 1e-4)
    eps = 1e-6
    for i in range(3):
        e = np.zeros(3)
        e[i] = eps
        fd = (obb_signed_distance(pts + e, R, c, h)[0] - obb_signed_distance(pts - e, R, c, h)[0]) / (2 * eps)
        np.testing.assert_allclose(fd[ok], g[ok, i], atol=1e-8)
    np.testing.assert_allclose(np.linalg.norm(g, axis=1), 1.0, atol=1e-14)
