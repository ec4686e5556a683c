"""First-order error budget of storing the five large tensors in reduced formats.  TEST INFRASTRUCTURE.

The paper evaluates a format assignment by quantising each large tensor at every kernel invocation
(Sec. IV-B) and keeps the narrowest assignment whose planning success holds (Sec. V-A, VI-A); it
states no numeric error bound.  The bound used here is the first-order one: rounding an in-range
element x of tensor T to nearest moves it by at most half the width u_T(x) of the interval of
representable values enclosing it (oracle.formats.ulp_at, at T's scale), so an output y changes by at
most

    budget(y) = sum over stored tensors T, over elements e of T:  |dy / dT_e| * u_T(T_e) / 2

to first order in the rounding errors.  Everything is evaluated at the unquantised FP64 values.

Sensitivities (readings of the kernels' data flow, the oracle's fwd_bwd):
  trajectory cost (per trajectory candidate, summed over its timesteps)
    S: dc/dS_{s,i} = G_{s,i}, the sphere-cost gradient (world and self terms)
    D: dc/dd_s = 2 w_c d_s (the cost is w_c sum d^2 of the stored depths)
    the FP32 per-configuration scalars (self cost, bound cost): their own FP32 rounding
    L, G and J do not enter the cost.
  joint gradient J_{b,j} (per configuration and joint; every term times the upstream weight)
    J: the rounding of J itself
    G: dJ_j/dG_s = z_j x (p_s - o_j) for spheres on links >= j (the geometric Jacobian column)
    S: through G = dc/dp, so dJ_j/dS_{s'} = sum_s (dG_s/dp_{s'})^T (z_j x (p_s - o_j)), with the
       sphere-cost Hessian: world term of an active sphere 2 w_c g g^T - 2 w_c d Hess(sd) (g the unit
       gradient of the closest cuboid's signed distance); active self pair (a, b) with unit
       direction v from b to a, activation r and centre distance l:
       dG_a/dp_a = w_s (2 v v^T - 2 r (I - v v^T) / l) = dG_b/dp_b = -dG_a/dp_b = -dG_b/dp_a
    L (stored poses only): J_j = z_j . E_j with E_j = sum_{l(s) >= j} (p_s - o_j) x G_s and
       F_j = sum_{l(s) >= j} G_s; z_j is the third column of R_j, o_j = t_j, and p_s = R_l c_s + t_l:
       dJ_j/dR_l[r][c] = sum_{l(s) = l >= j} (G_s x z_j)_r c_s[c]  + [l = j, c = 2] E_j[r]
       dJ_j/dt_l[r]    = sum_{l(s) = l >= j} (G_s x z_j)_r         - [l = j] (F_j x z_j)_r
    D does not enter the gradient (G is formed from the unquantised depth).
The swept and pose terms are not covered.  The bound is first order: where the rounding of S can
switch the closest cuboid or an OBB region (the kinks), or where narrow formats make the rounding
comparable to the values, the measured error may exceed it; the GPU tests allow twice the budget.

Parity pins (tests/test_oracle_budget.py): every sensitivity against central differences of the
oracle's own forward + backward pass with one stored element perturbed (perturb hook of fwd_bwd),
for every element of S, D, G, L and J on a small collision-rich batch; the budget's sum against
one-ulp perturbations of each stored element; the unquantised-vs-emulated error of FP16 assignments
within the budget; ulp_at against numpy's float16 spacing and the rounding error it bounds.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from . import exmy
from . import formats as fmts
from .cost import CostParams, Precision, fwd_bwd, world_index
from .geometry import obb_hessian
from .kinematics import N_JOINTS, joint_axes


def half_ulp(x: np.ndarray, fmt: str, k: int = 0) -> np.ndarray:
    """Largest rounding error of storing x in format fmt at scale 2^k (first order: in range)."""
    x = np.asarray(x, dtype=np.float64)
    if fmt in fmts.FORMATS:
        return 0.5 * fmts.ulp_at(x, fmt, k)
    E, M = exmy.parse(fmt)
    e_min, _, _ = exmy.limits(E, M)
    y = np.abs(x) * 2.0 ** -k
    _, ex = np.frexp(np.where(y > 0, y, 1.0))
    gap = np.ldexp(1.0, np.maximum(ex - 1, e_min) - M)
    return 0.5 * gap * 2.0 ** k


def world_hessian(S: np.ndarray, d: np.ndarray, gdir: np.ndarray, kstar: np.ndarray, pose: np.ndarray,
                  half_ext: np.ndarray, world_of_cfg: np.ndarray, w_c: float) -> np.ndarray:
    """d G_s / d p_s of the world term per configuration and sphere [B, n_s, 3, 3] (zero for
    inactive spheres)."""
    B, n_s, _ = S.shape
    H = np.zeros((B, n_s, 3, 3))
    act = d > 0
    for b, s in zip(*np.nonzero(act)):
        w, k = world_of_cfg[b], kstar[b, s]
        Hsd = obb_hessian(S[b, s], pose[w, k, :, :3], pose[w, k, :, 3], half_ext[w, k])
        g = gdir[b, s]
        H[b, s] = 2.0 * w_c * np.outer(g, g) - 2.0 * w_c * d[b, s] * Hsd
    return H


def pair_hessian(S: np.ndarray, radius: np.ndarray, pairs: np.ndarray, eta: float, w_s: float) -> np.ndarray:
    """d G_a / d p_a of each self pair (a, b) [B, P, 3, 3]; the other three blocks follow by sign."""
    a, b = pairs[:, 0], pairs[:, 1]
    diff = S[:, a] - S[:, b]
    dist = np.sqrt(np.sum(diff * diff, axis=-1))
    act = np.maximum(0.0, eta - (dist - radius[a] - radius[b]))
    live = (act > 0) & (dist > 0)
    safe = np.where(live, dist, 1.0)
    v = diff / safe[..., None]
    vv = v[..., :, None] * v[..., None, :]
    H = w_s * (2.0 * vv - 2.0 * (act / safe)[..., None, None] * (np.eye(3) - vv))
    return np.where(live[..., None, None], H, 0.0)


def jacobian_columns(T: np.ndarray, P: np.ndarray, sphere_link: np.ndarray) -> np.ndarray:
    """A[b, j, s] = z_{j+1} x (p_s - o_{j+1}) where sphere s rides on link >= j + 1, else 0:
    [B, 7, n_s, 3]."""
    z, o = joint_axes(T)
    A = np.cross(z[:, :, None, :], P[:, None, :, :] - o[:, :, None, :])
    on = np.asarray(sphere_link)[None, :] >= np.arange(1, N_JOINTS + 1)[:, None]  # [7, n_s]
    return A * on[None, :, :, None]


def sensitivities(robot, ref: Dict[str, np.ndarray], pose: np.ndarray, half_ext: np.ndarray,
                  params: CostParams, up_cfg: np.ndarray, stored_poses: bool) -> Dict[str, np.ndarray]:
    """|d output / d stored element| of the oracle's unquantised pass `ref`:
      cost_S [B, n_s, 3], cost_D [B, n_s]          (configuration cost)
      grad_G, grad_S [B, 7, n_s, 3], grad_L [B, 7, 8, 12]   (joint gradient, upstream included;
      grad_L zero in recompute mode)
    Signed values (not absolute), so that tests can compare them with central differences."""
    Tk, P, G, d = ref["poses"], ref["S"], ref["G"], ref["D"]
    B, n_s, _ = P.shape
    link = np.asarray(robot.sphere_link)
    wid = ref["world"]
    radius = np.asarray(robot.sphere_radius, dtype=np.float64)
    pairs = np.asarray(robot.pairs).reshape(-1, 2)
    out = {"cost_S": G.copy(), "cost_D": 2.0 * params.w_coll * d}

    A = jacobian_columns(Tk, P, link) * up_cfg[:, None, None, None]
    out["grad_G"] = A

    # through the sphere-cost Hessian
    from .cost import world_term
    _, gdir, kstar, _ = world_term(P, radius, pose, half_ext, wid, params.eta)
    Hw = world_hessian(P, d, gdir, kstar, pose, half_ext, wid, params.w_coll)
    W = np.einsum("bsij,bksj->bksi", Hw, A)
    if pairs.shape[0]:
        Hp = pair_hessian(P, radius, pairs, params.eta, params.w_self)
        a, bb = pairs[:, 0], pairs[:, 1]
        dA = A[:, :, a] - A[:, :, bb]                       # [B, 7, P, 3]
        contrib = np.einsum("bpij,bkpj->bkpi", Hp, dA)
        for p in range(pairs.shape[0]):
            W[:, :, a[p]] += contrib[:, :, p]
            W[:, :, bb[p]] -= contrib[:, :, p]
    out["grad_S"] = W

    # link poses read by the backward pass
    gL = np.zeros((B, N_JOINTS, 8, 12))
    if stored_poses:
        z, o = joint_axes(Tk)
        c_s = np.asarray(robot.sphere_center, dtype=np.float64)
        for j in range(1, N_JOINTS + 1):
            zj, oj = z[:, j - 1], o[:, j - 1]
            sel = link >= j
            Gs = G[:, sel]
            F = Gs.sum(axis=1)
            E = np.cross(P[:, sel] - oj[:, None, :], Gs).sum(axis=1)
            GxZ = np.cross(G, zj[:, None, :])             # [B, n_s, 3]
            for l in range(j, 9):
                on = link == l
                dR = np.einsum("bsr,sc->brc", GxZ[:, on], c_s[on])   # [B, 3, 3]
                dt = GxZ[:, on].sum(axis=1)                          # [B, 3]
                if l == j:
                    dR[:, :, 2] += E
                    dt -= np.cross(F, zj)
                gL[:, j - 1, l - 1].reshape(B, 3, 4)[:] = np.concatenate([dR, dt[:, :, None]], axis=2)
        gL *= up_cfg[:, None, None, None]
    out["grad_L"] = gL
    return out


def error_budget(robot, worlds, q: np.ndarray, traj_per_world: int, T: int, n_ls: int, prec: Precision,
                 params: CostParams = CostParams(), upstream: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """First-order bound of the quantisation error of `prec` against the unquantised FP64 pass:
      cost [n_tc]       per trajectory candidate
      grad [B, 7]       per configuration and joint
      cost_parts, grad_parts: the same split by stored tensor
      ref               the unquantised pass (fwd_bwd with prec None)
    Only the cost and collision terms of trajectory optimisation (no swept or pose term)."""
    if params.swept_steps:
        raise NotImplementedError("the budget does not cover the swept term")
    q = np.asarray(q, dtype=np.float64)
    B = q.shape[0]
    ref = fwd_bwd(robot, worlds, q, traj_per_world, T, n_ls, prec=None, params=params, upstream=upstream)
    n_tc = B // T
    up = np.ones(n_tc) if upstream is None else np.asarray(upstream, dtype=np.float64)
    up_cfg = up.repeat(T)
    stored = not prec.recompute_poses
    sens = sensitivities(robot, ref, worlds.pose, worlds.half_ext, params, up_cfg, stored)

    def hu(name, x):
        f, k = prec.get(name)
        return half_ulp(x, f, k)

    f32 = lambda x: half_ulp(x, "f32")  # noqa: E731
    cp = {
        "sphere_pos": np.sum(np.abs(sens["cost_S"]) * hu("sphere_pos", ref["S"]), axis=(1, 2)),
        "sphere_dist": np.sum(np.abs(sens["cost_D"]) * hu("sphere_dist", ref["D"]), axis=1),
        "scalars": f32(ref["self_cost"]) + params.w_bound * f32(ref["bound_cost"]),
    }
    per_cfg = sum(cp.values())
    gp = {
        "joint_grad": hu("joint_grad", ref["J"]),
        "sphere_grad": np.einsum("bksi,bsi->bk", np.abs(sens["grad_G"]), hu("sphere_grad", ref["G"])),
        "sphere_pos": np.einsum("bksi,bsi->bk", np.abs(sens["grad_S"]), hu("sphere_pos", ref["S"])),
        "link_poses": (np.einsum("bkle,ble->bk", np.abs(sens["grad_L"]), hu("link_poses", ref["L"]))
                       if stored else np.zeros((B, N_JOINTS))),
    }
    return {
        "cost": per_cfg.reshape(n_tc, T).sum(axis=1),
        "grad": sum(gp.values()),
        "cost_parts": {k: v.reshape(n_tc, T).sum(axis=1) for k, v in cp.items()},
        "grad_parts": gp,
        "sens": sens,
        "ref": ref,
    }


def hessian_margin(ref: Dict[str, np.ndarray], pose: np.ndarray, half_ext: np.ndarray) -> np.ndarray:
    """Per configuration, the smallest distance of an active sphere from a face plane of its closest
    cuboid (min_i ||u_i| - h_i|), where the signed distance's Hessian jumps; inf with no active
    sphere.  Central differences of the gradient are meaningful only well inside these regions."""
    P, d, kstar, wid = ref["S"], ref["D"], ref["kstar"], ref["world"]
    B, n_s, _ = P.shape
    m = np.full(B, np.inf)
    for b, s in zip(*np.nonzero(d > 0)):
        w, k = wid[b], kstar[b, s]
        R, c, h = pose[w, k, :, :3], pose[w, k, :, 3], half_ext[w, k]
        u = (P[b, s] - c) @ R
        m[b] = min(m[b], float(np.min(np.abs(np.abs(u) - h))))
    return m


def smooth_configurations(robot, ref: Dict[str, np.ndarray], pose: np.ndarray, half_ext: np.ndarray,
                          gap: float, eta: float = CostParams().eta) -> np.ndarray:
    """[B] bool: configurations whose cost and gradient are smooth within `gap` of the unquantised
    sphere centres -- every active sphere's closest cuboid, inside axis and OBB region unambiguous by
    more than gap, every active depth and every self-pair activation more than gap from zero.  The
    first-order budget describes the rounding error only there; elsewhere a rounding within gap may
    switch a branch of the cost."""
    d = ref["D"]
    active = d > 0
    ok = np.where(active, ref["margin"], np.inf).min(axis=1) > gap
    ok &= hessian_margin(ref, pose, half_ext) > gap
    ok &= ~np.any(active & (d < gap), axis=1)
    pairs = np.asarray(robot.pairs).reshape(-1, 2)
    if pairs.shape[0]:
        r = np.asarray(robot.sphere_radius, dtype=np.float64)
        S = ref["S"]
        dist = np.linalg.norm(S[:, pairs[:, 0]] - S[:, pairs[:, 1]], axis=-1)
        act = eta - (dist - r[pairs[:, 0]] - r[pairs[:, 1]])
        ok &= ~np.any(np.abs(act) < gap, axis=1)
    return ok


def position_gap(prec: Precision, ref: Dict[str, np.ndarray]) -> float:
    """Four times the largest rounding of a sphere centre under `prec` (at least 1 mm): the `gap` of
    smooth_configurations for this assignment."""
    f, k = prec.get("sphere_pos")
    return max(1e-3, 4.0 * float(np.max(half_ulp(ref["S"], f, k))))


__all__ = ["half_ulp", "world_hessian", "pair_hessian", "jacobian_columns", "sensitivities", "error_budget",
           "hessian_margin", "smooth_configurations", "position_gap", "world_index"]
