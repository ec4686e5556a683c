"""Serial-chain forward kinematics and collision-sphere placement in FP64.  TEST INFRASTRUCTURE.

The paper names the forward-kinematics stage (robot joint configuration -> Cartesian poses and the
collision spheres, Sec. II-B and step (2) of the optimisation iteration in Sec. III-B) but gives no
formulas.  Reading used here (standard revolute serial chain):

  T_0 = I,   T_j = T_{j-1} F_j Rz(q_j)  for j = 1..7,   T_8 = T_7 F_8,
  Rz(t) = [[cos t, -sin t, 0], [sin t, cos t, 0], [0, 0, 1]],
  sphere s on link l(s):  p_s = R_{l(s)} c_s + t_{l(s)}.

Joint j turns about the z axis of frame T_j, whose world direction is z_j = R_j e_z (Rz leaves the
z axis fixed) and whose origin is o_j = t_j.

Parity pins (tests/test_oracle_kinematics.py): F_j = I gives T_j = Rz(q_1 + ... + q_j); q = 0
gives the plain product of the F_j; a one-joint chain matches the closed-form rotation about z;
R^T R = I and det R = +1 for exactly orthonormal inputs; |p_s - t_{l(s)}| = |c_s| for every q;
changing q_j leaves links < j unchanged.
"""
from __future__ import annotations

import numpy as np

N_JOINTS = 7
N_LINKS = 9  # link 0 (base) .. link 8


def homogeneous(tf34: np.ndarray) -> np.ndarray:
    """[..., 3, 4] -> [..., 4, 4]."""
    tf34 = np.asarray(tf34, dtype=np.float64)
    out = np.zeros(tf34.shape[:-2] + (4, 4))
    out[..., :3, :] = tf34
    out[..., 3, 3] = 1.0
    return out


def rot_z(theta: np.ndarray) -> np.ndarray:
    """[B] angles -> [B, 4, 4] homogeneous rotations about z."""
    theta = np.asarray(theta, dtype=np.float64)
    c, s = np.cos(theta), np.sin(theta)
    out = np.zeros(theta.shape + (4, 4))
    out[..., 0, 0], out[..., 0, 1] = c, -s
    out[..., 1, 0], out[..., 1, 1] = s, c
    out[..., 2, 2] = 1.0
    out[..., 3, 3] = 1.0
    return out


def forward_kinematics(fixed_tf: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Link poses T_0..T_8 as [B, 9, 4, 4] for configurations q [B, 7]."""
    q = np.asarray(q, dtype=np.float64)
    B = q.shape[0]
    F = homogeneous(fixed_tf)  # F[j-1] is F_j
    T = np.zeros((B, N_LINKS, 4, 4))
    T[:, 0] = np.eye(4)
    for j in range(1, N_JOINTS + 1):
        T[:, j] = T[:, j - 1] @ F[j - 1] @ rot_z(q[:, j - 1])
    T[:, N_LINKS - 1] = T[:, N_JOINTS] @ F[N_JOINTS]
    return T


def link_pose_values(T: np.ndarray) -> np.ndarray:
    """The stored link-pose tensor: links 1..8 as row-major 3x4 [R | t], shape [B, 8, 12]."""
    return T[:, 1:, :3, :].reshape(T.shape[0], N_LINKS - 1, 12)


def poses_from_values(L: np.ndarray) -> np.ndarray:
    """Inverse of `link_pose_values`: [B, 8, 12] -> [B, 9, 4, 4] with T_0 = I."""
    B = L.shape[0]
    T = np.zeros((B, N_LINKS, 4, 4))
    T[:, 0] = np.eye(4)
    T[:, 1:, :3, :] = L.reshape(B, N_LINKS - 1, 3, 4)
    T[:, 1:, 3, 3] = 1.0
    return T


def sphere_positions(T: np.ndarray, sphere_center: np.ndarray, sphere_link: np.ndarray) -> np.ndarray:
    """p_s = R_{l(s)} c_s + t_{l(s)} as [B, n_s, 3]."""
    Ts = T[:, np.asarray(sphere_link)]                      # [B, n_s, 4, 4]
    c = np.asarray(sphere_center, dtype=np.float64)
    return np.einsum("bsij,sj->bsi", Ts[:, :, :3, :3], c) + Ts[:, :, :3, 3]


def joint_axes(T: np.ndarray):
    """(z_j, o_j) for j = 1..7 as two [B, 7, 3] arrays."""
    return T[:, 1:N_JOINTS + 1, :3, 2], T[:, 1:N_JOINTS + 1, :3, 3]
