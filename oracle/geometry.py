"""Signed distance from a point to an oriented cuboid, and its gradient, in FP64.  TEST INFRASTRUCTURE.

The paper's collision kernel queries robot spheres against the environment (Sec. II-B, III-C) but
does not define the query.  Reading used here: obstacles are oriented cuboids given by a rotation
R, a centre c and half extents h.  With u = R^T (p - c) and a = |u| - h (componentwise):

  sd(p) = || max(a, 0) ||_2 + min(max_i a_i, 0)

and the gradient is R n with
  outside (||max(a,0)|| > 0):  n = sign(u) * max(a, 0) / ||max(a, 0)||
  inside or on the surface:    n = sign(u_i) e_i,   i = the first index of max_i a_i,
where sign(0) = +1.  The gradient is set-valued where the inside axis i is not unique; `axis_gap`
reports the gap between the two largest a_i so tests can avoid those points.

Parity pins (tests/test_oracle_geometry.py): brute-force surface sampling of the six faces; the
centre gives -min(h); points on faces give 0; the axis-aligned case equals the textbook box
distance; rotating point and box together leaves sd unchanged; the gradient matches central
differences away from the medial set.
"""
from __future__ import annotations

import numpy as np


def obb_signed_distance(p: np.ndarray, R: np.ndarray, c: np.ndarray, h: np.ndarray):
    """Signed distance of points p [..., 3] to one cuboid (R [3, 3], c [3], h [3]).
    Returns (sd [...], grad [..., 3], axis_gap [...])."""
    p = np.asarray(p, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    u = (p - c) @ R                      # u_i = sum_j R[j, i] (p - c)_j  (that is, R^T (p - c))
    a = np.abs(u) - h
    o = np.maximum(a, 0.0)
    norm_o = np.sqrt(np.sum(o * o, axis=-1))
    amax = np.max(a, axis=-1)
    sd = norm_o + np.minimum(amax, 0.0)

    sgn = np.where(u >= 0.0, 1.0, -1.0)
    safe = np.where(norm_o > 0.0, norm_o, 1.0)[..., None]
    n_out = sgn * o / safe
    axis = np.argmax(a, axis=-1)
    n_in = np.zeros_like(u)
    np.put_along_axis(n_in, axis[..., None], np.take_along_axis(sgn, axis[..., None], axis=-1), axis=-1)
    n = np.where((norm_o > 0.0)[..., None], n_out, n_in)
    grad = n @ R.T                       # R n
    a_sorted = np.sort(a, axis=-1)
    axis_gap = np.where(norm_o > 0.0, np.inf, a_sorted[..., 2] - a_sorted[..., 1])
    return sd, grad, axis_gap


def obb_hessian(p: np.ndarray, R: np.ndarray, c: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Hessian of sd w.r.t. p [..., 3] for one cuboid: [..., 3, 3].  Outside, sd = ||o|| with
    o = max(|u| - h, 0) over the axes where |u_i| > h_i, whose Hessian in the box frame is
    (P - n n^T) / ||o|| (P: those axes, n: the unit outward direction sign(u) o / ||o||), turned into
    the world frame as R (.) R^T.  Inside sd is max_i a_i, piecewise linear: zero Hessian.  Undefined
    where an axis is exactly on its face plane or the inside axis is not unique (the kinks)."""
    p = np.asarray(p, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    u = (p - c) @ R
    a = np.abs(u) - h
    o = np.maximum(a, 0.0)
    norm_o = np.sqrt(np.sum(o * o, axis=-1))
    out = norm_o > 0.0
    safe = np.where(out, norm_o, 1.0)[..., None]
    n = np.where(u >= 0.0, 1.0, -1.0) * o / safe
    P = (a > 0.0).astype(np.float64)
    Hu = (P[..., :, None] * np.eye(3) - n[..., :, None] * n[..., None, :]) / safe[..., None]
    Hu = np.where(out[..., None, None], Hu, 0.0)
    return R @ Hu @ R.T
