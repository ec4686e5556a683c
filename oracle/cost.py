"""Trajectory-optimisation costs and their joint-space gradient in FP64.  TEST INFRASTRUCTURE.

One optimisation iteration (Sec. III-B) computes kinematics (2), the collision, self-collision and
bound costs (3), aggregates them (4) and back-propagates through those steps (5).  The paper names
the costs without formulas; the readings used here:

  activation depth of sphere s:  d_s = max(0, eta - min_k (sd_k(p_s) - r_s)),  k* = first arg-min
  world cost                      w_c * d_s^2
  self pair (a, b):               e = |p_a - p_b| - r_a - r_b,   w_s * max(0, eta - e)^2
  bound cost:                     w_b * sum_j max(0, q_j - hi_j)^2 + max(0, lo_j - q_j)^2
  configuration cost              c = w_c sum_s d_s^2 + w_s sum_pairs max(0, eta - e)^2 + w_b bound
  trajectory cost                 sum_t c_t + w_v sum_t |q_{t+1} - q_t|^2

The stored per-sphere distance tensor holds d_s (zero for spheres farther than eta from every
cuboid, which is what makes it mostly zeros, Sec. III-C).  Its gradient w.r.t. the sphere centre is
-2 w_c d_s grad sd_{k*} plus the self-pair terms -2 w_s max(0, eta - e) (p_a - p_b)/|p_a - p_b| (zero
for coincident centres).  Joint-space gradient, by reverse accumulation down the chain:

  J_j = z_j . sum_{s: l(s) >= j} (p_s - o_j) x G_s

and, independently, through the explicit geometric Jacobian dp_s/dq_j = z_j x (p_s - o_j).

Quantisation emulation (Sec. IV-B: quantise-then-dequantise at every kernel invocation): with a
precision assignment the five stored tensors -- link poses L, sphere positions S, distances D,
sphere gradients G, joint gradients J -- are each replaced by dec(enc(.)) of their FP32 rounding at
the point where the GPU path writes them; all other arithmetic stays FP64.  S is computed from the
unquantised poses; the backward pass uses the quantised poses in stored mode and recomputes them
from q in recompute mode.

Swept collision (the fifth large tensor of trajectory optimisation, closest_pt_swept, Sec. III-C;
the paper does not define the sweep).  Reading used here: between consecutive timesteps t and t+1
of one trajectory-candidate each sphere centre moves on the straight segment between its two stored
positions, sampled at k interior points u_i = i / (k + 1), i = 1..k:

  p_i = (1 - u_i) p_s(t) + u_i p_s(t+1),     d_i = activation depth of p_i (as above)
  swept cost of configuration t   (w_sw / k) sum_s sum_i d_i^2       (0 for the last timestep)
  swept gradient X_s(t)           d/dp_s(t) of the sum over all segments: the segment (t, t+1)
                                  with weights (1 - u_i), the segment (t-1, t) with weights u_i

and it is stored as its own tensor X (format of its own), added to G in the backward pass.

Pose (goal) cost of inverse-kinematics optimisation (the IK stage turns the goal pose of the end
effector into joint configurations, Sec. II-A, III-B; the paper gives no formula).  Reading used
here: the end-effector frame is link 8, T_8 = [R | p]; with the goal pose [R_g | p_g] of the
configuration's problem (one per world),

  pose cost   w_gp |p - p_g|^2 + w_gr ||R - R_g||_F^2      (= w_gr (6 - 2 tr(R_g^T R)))

Its joint gradient, from dp/dq_j = z_j x (p - o_j) and dR/dq_j = [z_j]_x R, is a force
F = 2 w_gp (p - p_g) at p plus a couple tau = -2 w_gr m(R R_g^T) on link 8, with
m(M) = (M_23 - M_32, M_31 - M_13, M_12 - M_21):  dC/dq_j = z_j . ((p - o_j) x F + tau).

Parity pins (tests/test_oracle_cost.py): adjoint == explicit Jacobian to 1e-12; joint gradient ==
central differences of the trajectory cost; sphere gradient == central differences of the
configuration cost; self pair closed form; hand-computed single-sphere cases; at f32 with emulation
the costs differ from the unquantised ones by FP32 rounding only.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

from . import exmy
from . import formats as fmts
from .geometry import obb_signed_distance
from .kinematics import (N_JOINTS, forward_kinematics, joint_axes, link_pose_values, poses_from_values,
                         sphere_positions)

TENSORS = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")
SWEPT = "swept_grad"


@dataclass
class CostParams:
    eta: float = 0.02
    w_coll: float = 100.0
    w_self: float = 100.0
    w_bound: float = 10.0
    w_smooth: float = 1.0
    swept_steps: int = 0       # k interior samples per segment; 0 turns the swept term off
    w_swept: float = 100.0
    w_goal_pos: float = 100.0  # pose cost weights (used when goals are given)
    w_goal_rot: float = 10.0


@dataclass
class Precision:
    """Format name and power-of-two scale exponent per stored tensor, plus the pose mode."""

    link_poses: Tuple[str, int] = ("f32", 0)
    sphere_pos: Tuple[str, int] = ("f32", 0)
    sphere_dist: Tuple[str, int] = ("f32", 0)
    sphere_grad: Tuple[str, int] = ("f32", 0)
    joint_grad: Tuple[str, int] = ("f32", 0)
    recompute_poses: bool = False
    swept_grad: Tuple[str, int] = ("f32", 0)

    def get(self, tensor: str) -> Tuple[str, int]:
        return getattr(self, tensor)


def world_term(S: np.ndarray, radius: np.ndarray, pose: np.ndarray, half_ext: np.ndarray,
               world_of_cfg: np.ndarray, eta: float):
    """Per sphere: activation depth d [B, n_s], unit gradient of sd at k* [B, n_s, 3], k* [B, n_s]
    and the kink margin [B, n_s] (gap to the runner-up cuboid, inside-axis gap)."""
    B, n_s, _ = S.shape
    d = np.zeros((B, n_s))
    grad = np.zeros((B, n_s, 3))
    kstar = np.zeros((B, n_s), dtype=np.int64)
    margin = np.full((B, n_s), np.inf)
    for w in np.unique(world_of_cfg):
        idx = np.nonzero(world_of_cfg == w)[0]
        P = S[idx]                                    # [b, n_s, 3]
        best = np.full(P.shape[:2], np.inf)
        second = np.full(P.shape[:2], np.inf)
        bgrad = np.zeros(P.shape)
        bgap = np.full(P.shape[:2], np.inf)
        bk = np.zeros(P.shape[:2], dtype=np.int64)
        for k in range(pose.shape[1]):
            R, c, h = pose[w, k, :, :3], pose[w, k, :, 3], half_ext[w, k]
            sd, g, gap = obb_signed_distance(P, R, c, h)
            e = sd - radius[None, :]
            better = e < best                          # strict: ties keep the lower index
            second = np.where(better, best, np.minimum(second, e))
            best = np.where(better, e, best)
            bk = np.where(better, k, bk)
            bgrad = np.where(better[..., None], g, bgrad)
            bgap = np.where(better, gap, bgap)
        d[idx] = np.maximum(0.0, eta - best)
        grad[idx] = bgrad
        kstar[idx] = bk
        # no runner-up (fewer than two cuboids): no switch to guard against
        with np.errstate(invalid="ignore"):  # inf - inf where there is no runner-up; replaced below
            gap2 = np.where(np.isfinite(second), second - best, np.inf)
        margin[idx] = np.minimum(gap2, bgap)
    return d, grad, kstar, margin


def self_term(S: np.ndarray, radius: np.ndarray, pairs: np.ndarray, eta: float):
    """Per configuration: sum of max(0, eta - e)^2 over pairs [B], the gradient of that sum w.r.t.
    every sphere centre [B, n_s, 3] and the smallest centre distance [B]."""
    B, n_s, _ = S.shape
    a, b = pairs[:, 0], pairs[:, 1]
    diff = S[:, a] - S[:, b]                           # [B, P, 3]
    dist = np.sqrt(np.sum(diff * diff, axis=-1))
    e = dist - radius[a] - radius[b]
    act = np.maximum(0.0, eta - e)
    cost = np.sum(act * act, axis=1)
    unit = np.where(dist[..., None] > 0, diff / np.where(dist > 0, dist, 1.0)[..., None], 0.0)
    ga = -2.0 * act[..., None] * unit                  # d/dp_a; d/dp_b is the negative
    grad = np.zeros((B, n_s, 3))
    for p in range(pairs.shape[0]):
        grad[:, a[p]] += ga[:, p]
        grad[:, b[p]] -= ga[:, p]
    return cost, grad, np.min(dist, axis=1) if pairs.shape[0] else np.full(B, np.inf)


def swept_term(S: np.ndarray, radius: np.ndarray, pose: np.ndarray, half_ext: np.ndarray,
               world_of_cfg: np.ndarray, eta: float, T: int, k: int):
    """Unweighted swept term for configurations laid out with timestep fastest in runs of T.
    Returns the per-configuration cost (1/k) sum_s sum_i d_i^2 of the segment (t, t+1) [B], its
    gradient summed over both segments at each configuration [B, n_s, 3] and the smallest kink
    margin of any active sample point (d > 0) of either segment [B]; inactive samples contribute
    nothing to the gradient, so their kinks do not matter."""
    B, n_s, _ = S.shape
    cost = np.zeros(B)
    X = np.zeros((B, n_s, 3))
    margin = np.full(B, np.inf)
    t = np.arange(B) % T
    seg = np.nonzero(t < T - 1)[0]                    # segment starts
    if k <= 0 or seg.size == 0:
        return cost, X, margin
    P0, P1 = S[seg], S[seg + 1]
    for i in range(1, k + 1):
        u = i / (k + 1)
        Pi = (1.0 - u) * P0 + u * P1
        d, gdir, _, mg = world_term(Pi, radius, pose, half_ext, world_of_cfg[seg], eta)
        cost[seg] += np.sum(d * d, axis=1) / k
        g = np.where(d[..., None] > 0, (-2.0 / k) * d[..., None] * gdir, 0.0)
        X[seg] += (1.0 - u) * g
        X[seg + 1] += u * g
        m = np.min(np.where(d > 0, mg, np.inf), axis=1)
        margin[seg] = np.minimum(margin[seg], m)
        margin[seg + 1] = np.minimum(margin[seg + 1], m)
    return cost, X, margin


def pose_term(T: np.ndarray, goal: np.ndarray, w_pos: float, w_rot: float):
    """Pose cost [B] of link 8 against per-configuration goals [B, 3, 4], and the end-effector
    wrench: force F [B, 3] at p and couple tau [B, 3] (see the module notes)."""
    R, p = T[:, 8, :3, :3], T[:, 8, :3, 3]
    Rg, pg = goal[:, :, :3], goal[:, :, 3]
    dp = p - pg
    dR = R - Rg
    cost = w_pos * np.sum(dp * dp, axis=1) + w_rot * np.sum(dR * dR, axis=(1, 2))
    M = R @ np.swapaxes(Rg, 1, 2)
    m = np.stack([M[:, 1, 2] - M[:, 2, 1], M[:, 2, 0] - M[:, 0, 2], M[:, 0, 1] - M[:, 1, 0]], axis=1)
    return cost, 2.0 * w_pos * dp, -2.0 * w_rot * m


def pose_grad_adjoint(T: np.ndarray, F: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Joint gradient of the pose cost from the end-effector wrench: z_j . ((p - o_j) x F + tau)."""
    z, o = joint_axes(T)
    p = T[:, 8, :3, 3]
    arm = p[:, None, :] - o
    return np.sum(z * (np.cross(arm, F[:, None, :]) + tau[:, None, :]), axis=2)


def pose_grad_explicit(T: np.ndarray, goal: np.ndarray, w_pos: float, w_rot: float) -> np.ndarray:
    """The same gradient by the chain rule on the matrices themselves: 2 w_gp (p - p_g).(z_j x
    (p - o_j)) - 2 w_gr tr(R_g^T [z_j]_x R)."""
    z, o = joint_axes(T)
    R, p = T[:, 8, :3, :3], T[:, 8, :3, 3]
    Rg, pg = goal[:, :, :3], goal[:, :, 3]
    B = T.shape[0]
    out = np.zeros((B, N_JOINTS))
    for j in range(N_JOINTS):
        zj = z[:, j]
        dp = np.cross(zj, p - o[:, j])
        Z = np.zeros((B, 3, 3))
        Z[:, 0, 1], Z[:, 0, 2], Z[:, 1, 2] = -zj[:, 2], zj[:, 1], -zj[:, 0]
        Z[:, 1, 0], Z[:, 2, 0], Z[:, 2, 1] = zj[:, 2], -zj[:, 1], zj[:, 0]
        dR = Z @ R
        out[:, j] = (2.0 * w_pos * np.sum((p - pg) * dp, axis=1)
                     - 2.0 * w_rot * np.einsum("bij,bij->b", Rg, dR))
    return out


def bound_term(q: np.ndarray, q_lo: np.ndarray, q_hi: np.ndarray):
    over = np.maximum(0.0, q - q_hi)
    under = np.maximum(0.0, q_lo - q)
    return np.sum(over * over + under * under, axis=1), 2.0 * over - 2.0 * under


def joint_grad_adjoint(T: np.ndarray, P: np.ndarray, G: np.ndarray, sphere_link: np.ndarray) -> np.ndarray:
    """J[b, j-1] = z_j . sum_{s: l(s) >= j} (p_s - o_j) x G_s  (reverse accumulation)."""
    z, o = joint_axes(T)
    B = P.shape[0]
    J = np.zeros((B, N_JOINTS))
    link = np.asarray(sphere_link)
    for j in range(1, N_JOINTS + 1):
        sel = link >= j
        r = P[:, sel] - o[:, j - 1][:, None, :]
        torque = np.sum(np.cross(r, G[:, sel]), axis=1)
        J[:, j - 1] = np.sum(z[:, j - 1] * torque, axis=1)
    return J


def joint_grad_jacobian(T: np.ndarray, P: np.ndarray, G: np.ndarray, sphere_link: np.ndarray) -> np.ndarray:
    """J = Jac^T G with the explicit geometric Jacobian dp_s/dq_j = z_j x (p_s - o_j) (l(s) >= j)."""
    z, o = joint_axes(T)
    B, n_s, _ = P.shape
    jac = np.zeros((B, n_s, 3, N_JOINTS))
    for s in range(n_s):
        for j in range(1, int(sphere_link[s]) + 1 if sphere_link[s] <= N_JOINTS else N_JOINTS + 1):
            jac[:, s, :, j - 1] = np.cross(z[:, j - 1], P[:, s] - o[:, j - 1])
    return np.einsum("bsij,bsi->bj", jac, G)


def smoothness_grad(q: np.ndarray, T: int, n_ls: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per trajectory-candidate smoothness sum |q_{t+1} - q_t|^2 [n_tc] and its gradient [B, 7]."""
    B = q.shape[0]
    qt = q.reshape(B // T, T, N_JOINTS)
    dq = qt[:, 1:] - qt[:, :-1]
    val = np.sum(dq * dq, axis=(1, 2))
    g = np.zeros_like(qt)
    g[:, 1:] += 2.0 * dq
    g[:, :-1] -= 2.0 * dq
    return val, g.reshape(B, N_JOINTS)


def world_index(B: int, traj_per_world: int, T: int, n_ls: int) -> np.ndarray:
    b = np.arange(B)
    return (b // (T * n_ls)) // traj_per_world


def _store(x: np.ndarray, prec: Optional[Precision], tensor: str):
    """(codes, stored float64 values) at a storage point; unquantised pass-through when prec is None.
    A storage format (f32, f16, bf16, e4m3, e5m2, e3m2, e2m1) goes through its codec; any other
    'eXmY' is emulated: the FP32 value rounded to that type (codes: its FP32 bit patterns)."""
    if prec is None:
        return None, np.asarray(x, dtype=np.float64)
    fmt, k = prec.get(tensor)
    if fmt in fmts.FORMATS:
        return fmts.roundtrip(x, fmt, k)
    E, M = exmy.parse(fmt)
    return exmy.roundtrip(x, E, M, k)


def fwd_bwd(robot, worlds, q: np.ndarray, traj_per_world: int, T: int, n_ls: int,
            prec: Optional[Precision] = None, params: CostParams = CostParams(),
            upstream: Optional[np.ndarray] = None, emulate_scalars: bool = True,
            goals: Optional[np.ndarray] = None,
            perturb: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """Whole forward + backward pass for configurations q [B, 7] laid out as
    b = ((traj * n_ls + candidate) * T + t).  With `prec` None this is the unquantised FP64 truth;
    otherwise each stored tensor goes through the reference codec (f32 = FP32 rounding) where the
    GPU path writes it.  `upstream` is d(loss)/d(cost_traj) per trajectory-candidate (default 1).
    `goals` [n_worlds, 3, 4] adds the pose cost of each world's goal (inverse kinematics): its value
    from the unquantised poses, its gradient from the poses the backward pass reads.
    `perturb` maps some of "L", "S", "D", "G", "J" to arrays added to that stored tensor right after
    its store (the brute-force check of the error budget's sensitivities); a perturbed L is read by
    the backward pass even without a precision assignment."""
    q = np.asarray(q, dtype=np.float64)
    B = q.shape[0]
    n_tc = B // T
    assert n_tc * T == B and (n_tc // n_ls) * n_ls == n_tc
    wid = world_index(B, traj_per_world, T, n_ls)
    eta = params.eta
    out: Dict[str, np.ndarray] = {}

    # (2) kinematics: link poses and sphere centres
    Tk = forward_kinematics(robot.fixed_tf, q)
    Lval = link_pose_values(Tk)
    perturb = perturb or {}
    out["L_codes"], L_hat = _store(Lval, None if (prec is not None and prec.recompute_poses) else prec,
                                   "link_poses")
    L_hat = L_hat + perturb.get("L", 0.0)
    S = sphere_positions(Tk, robot.sphere_center, robot.sphere_link)
    out["S_codes"], S_hat = _store(S, prec, "sphere_pos")
    S_hat = S_hat + perturb.get("S", 0.0)
    bcost, bgrad = bound_term(q, robot.q_lo, robot.q_hi)

    # (3) costs from the stored sphere positions
    d, gdir, kstar, margin = world_term(S_hat, robot.sphere_radius, worlds.pose, worlds.half_ext, wid, eta)
    scost, sgrad, min_pair = self_term(S_hat, robot.sphere_radius, robot.pairs, eta)
    # an inactive sphere (d = 0) contributes an exact zero (+0), not -0 from the product
    G = np.where(d[..., None] > 0, -2.0 * params.w_coll * d[..., None] * gdir, 0.0) + params.w_self * sgrad
    out["D_codes"], D_hat = _store(d, prec, "sphere_dist")
    out["G_codes"], G_hat = _store(G, prec, "sphere_grad")
    D_hat = D_hat + perturb.get("D", 0.0)
    G_hat = G_hat + perturb.get("G", 0.0)
    if prec is not None and emulate_scalars:
        scost_st = fmts.fp32(params.w_self * scost).astype(np.float64)
        bcost_st = fmts.fp32(bcost).astype(np.float64)
    else:
        scost_st, bcost_st = params.w_self * scost, bcost
    swept = params.swept_steps > 0
    if swept:
        wcost, Xs, wmargin = swept_term(S_hat, robot.sphere_radius, worlds.pose, worlds.half_ext, wid, eta, T,
                                        params.swept_steps)
        X = params.w_swept * Xs
        out["X_codes"], X_hat = _store(X, prec, SWEPT)
        wcost_st = params.w_swept * wcost
        if prec is not None and emulate_scalars:
            wcost_st = fmts.fp32(wcost_st).astype(np.float64)
        out.update(X=X, X_hat=X_hat, swept_cost=wcost_st, swept_margin=wmargin)
    else:
        X_hat, wcost_st = 0.0, 0.0
    if goals is not None:
        gcfg = np.asarray(goals, dtype=np.float64)[wid]
        pcost, _, _ = pose_term(Tk, gcfg, params.w_goal_pos, params.w_goal_rot)
        pcost_st = fmts.fp32(pcost).astype(np.float64) if (prec is not None and emulate_scalars) else pcost
        out["pose_cost"] = pcost_st
    else:
        pcost_st = 0.0

    # (4) aggregation
    cfg = params.w_coll * np.sum(D_hat * D_hat, axis=1) + scost_st + params.w_bound * bcost_st + wcost_st + pcost_st
    smooth, sgr = smoothness_grad(q, T, n_ls)
    cost_traj = cfg.reshape(n_tc, T).sum(axis=1) + params.w_smooth * smooth

    # (5) backward to joint space
    if (prec is not None and not prec.recompute_poses) or "L" in perturb:
        Tb = poses_from_values(L_hat)
        Pb = sphere_positions(Tb, robot.sphere_center, robot.sphere_link)
    else:
        Tb, Pb = Tk, S
    Jsph = joint_grad_adjoint(Tb, Pb, G_hat + X_hat, robot.sphere_link)
    if goals is not None:
        _, Fp, taup = pose_term(Tb, gcfg, params.w_goal_pos, params.w_goal_rot)
        Jsph = Jsph + pose_grad_adjoint(Tb, Fp, taup)
    up = np.ones(n_tc) if upstream is None else np.asarray(upstream, dtype=np.float64)
    J = up.repeat(T)[:, None] * (Jsph + params.w_bound * bgrad + params.w_smooth * sgr)
    out["J_codes"], J_hat = _store(J, prec, "joint_grad")
    J_hat = J_hat + perturb.get("J", 0.0)

    out.update(L=Lval, L_hat=L_hat, S=S, S_hat=S_hat, D=d, D_hat=D_hat, G=G, G_hat=G_hat, J=J, J_hat=J_hat,
               self_cost=scost_st, bound_cost=bcost_st, cfg_cost=cfg, cost_traj=cost_traj, grad_q=J_hat,
               kstar=kstar, margin=margin, min_pair_dist=min_pair, world=wid, poses=Tk)
    return out


def config_cost(robot, worlds, q: np.ndarray, world_of_cfg: np.ndarray, params: CostParams = CostParams()):
    """Unquantised configuration cost c(q) [B] (for finite-difference checks)."""
    Tk = forward_kinematics(robot.fixed_tf, q)
    S = sphere_positions(Tk, robot.sphere_center, robot.sphere_link)
    d, _, _, _ = world_term(S, robot.sphere_radius, worlds.pose, worlds.half_ext, world_of_cfg, params.eta)
    sc, _, _ = self_term(S, robot.sphere_radius, robot.pairs, params.eta)
    bc, _ = bound_term(q, robot.q_lo, robot.q_hi)
    return params.w_coll * np.sum(d * d, axis=1) + params.w_self * sc + params.w_bound * bc


def sphere_cost(robot, worlds, S: np.ndarray, world_of_cfg: np.ndarray, params: CostParams = CostParams()):
    """Collision part of the configuration cost as a function of the sphere centres [B, n_s, 3]."""
    d, _, _, _ = world_term(S, robot.sphere_radius, worlds.pose, worlds.half_ext, world_of_cfg, params.eta)
    sc, _, _ = self_term(S, robot.sphere_radius, robot.pairs, params.eta)
    return params.w_coll * np.sum(d * d, axis=1) + params.w_self * sc
