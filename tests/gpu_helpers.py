"""Shared pieces of the GPU parity tests: contexts built from synthetic workloads, oracle runs, and
comparisons of stored codes that allow a one-step difference only where the oracle flags a value
as lying within the FP32 computation error of a rounding boundary."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import cost as OC
from oracle import formats as F

torch = pytest.importorskip("torch")

TENSORS = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")
ORACLE_KEY = {"link_poses": "L", "sphere_pos": "S", "sphere_dist": "D", "sphere_grad": "G", "joint_grad": "J"}

# Bounds on the error of the float32 computation of each stored quantity before it is encoded
# (absolute in the tensor's units, plus a relative part).  Positions and poses come out of an
# 8-transform chain of float32 products (about 24 roundings of unit-size terms); distances add the
# cuboid transform.  A sphere gradient sums up to 1 + 8 terms (its closest cuboid and its active
# pairs), each a distance carrying about 2.4e-7 m of rounding (two roundings of 2 m coordinates)
# scaled by 2w = 200: 4.3e-4, doubled.  A joint gradient sums lever arm x sphere gradient over the
# spheres beyond the joint.  The FP32 assignment of the stage tests prints how much of each band
# its arithmetic uses (at most about a quarter for G at this band, a twentieth for the others).
RISK = {
    "link_poses": (1e-5, 4e-6),
    "sphere_pos": (1e-5, 4e-6),
    "sphere_dist": (1e-5, 8e-6),
    "sphere_grad": (1e-4, 1e-3),
    "joint_grad": (2e-4, 2e-3),
    "swept_grad": (1e-4, 1e-3),
}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def make_context(wl, prec=None, recompute=False, params=None):
    from paper_2310_07854_amd import Context

    ctx = Context(0)
    ctx.set_robot(wl.robot)
    ctx.set_worlds(wl.worlds.pose, wl.worlds.half_ext)
    if params is not None:
        ctx.set_cost_params(**params)
    if prec is not None:
        ctx.set_precision(prec, recompute)
    return ctx


def oracle_precision(prec, recompute=False) -> OC.Precision:
    kw = {}
    for t in TENSORS:
        v = (prec or {}).get(t, "f32")
        kw[t] = (v, 0) if isinstance(v, str) else tuple(v)
    return OC.Precision(recompute_poses=recompute, **kw)


def shape_of(wl):
    from paper_2310_07854_amd import Shape

    return Shape(wl.n_worlds, wl.traj_per_world, wl.T, wl.n_ls)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def export_codes(ctx, name, ws, shape) -> np.ndarray:
    fmt = ctx.precision[name][0]
    raw = ctx.ws_export(name, ws, shape).cpu().numpy()
    n = shape.B * ctx.tensor_count(name)
    return F.unpack(raw, fmt, n)


def import_codes(ctx, name, ws, shape, codes: np.ndarray) -> None:
    fmt = ctx.precision[name][0]
    packed = F.pack(codes.ravel(), fmt)
    ctx.ws_import(name, ws, shape, torch.from_numpy(packed).to("cuda:0"))


def ordinal(codes: np.ndarray, fmt: str) -> np.ndarray:
    """Position of each code on the number line (monotone in value; +0 and -0 share 0)."""
    f = F.get(fmt)
    c = codes.astype(np.int64)
    mag = c & (f.sign_bit - 1)
    return np.where((c & f.sign_bit) != 0, -mag, mag)


def compare_codes(name, fmt, k, gpu_codes, oracle_codes, oracle_values, exempt=None):
    """Every GPU code must be the encoding of some value within the float32 computation error band
    [x - tol, x + tol] of the oracle value x (tol = rel |x| + abs from RISK); where the band holds
    no rounding boundary this means equality with the oracle's code.  Elements in `exempt` (kink
    points, where the exact result itself is set-valued) are skipped.  Returns (n_flagged, n_diff)."""
    rel, abs_ = RISK[name]
    gpu_codes = gpu_codes.reshape(-1).astype(np.uint32)
    oracle_codes = oracle_codes.reshape(-1).astype(np.uint32)
    x = np.asarray(oracle_values, dtype=np.float64).reshape(-1)
    keep = np.ones(x.shape, dtype=bool) if exempt is None else ~exempt.reshape(-1)
    tol = rel * np.abs(x) + abs_
    lo = ordinal(F.quantize(x - tol, fmt, k), fmt)
    hi = ordinal(F.quantize(x + tol, fmt, k), fmt)
    og = ordinal(gpu_codes, fmt)
    ok = (og >= np.minimum(lo, hi)) & (og <= np.maximum(lo, hi))
    bad = keep & ~ok
    assert not bad.any(), (f"{name}/{fmt}: {int(bad.sum())} codes outside the error band, e.g. idx "
                           f"{np.nonzero(bad)[0][:5]} gpu {gpu_codes[bad][:5]} oracle {oracle_codes[bad][:5]} "
                           f"values {x[bad][:5]}")
    flagged = keep & (lo != hi)
    # +0 and -0 are one value (ordinal 0): which sign an exact zero carries is not compared
    diff = keep & (og != ordinal(oracle_codes, fmt))
    assert not (diff & ~flagged).any()
    ratio = ""
    if fmt == "f32" and keep.any():
        # FP32 codes are the computed values themselves: how much of the band the error uses
        err = np.abs(F.dequantize(gpu_codes, fmt, k).astype(np.float64) - x)
        ratio = f", worst error / band {float((err / tol)[keep].max()):.3f}"
    print(f"[codes] {name}/{fmt} k={k}: {int(keep.sum())} compared, {int(flagged.sum())} near a boundary, "
          f"{int(diff.sum())} differ from the oracle{ratio}")
    return int(flagged.sum()), int(diff.sum())


def cfg_cost_tolerance(ref, n_pairs, params=OC.CostParams(), eps_pos=4e-6):
    """Per-configuration part of cost_tolerance (see there)."""
    world = 2.0 * params.w_coll * ref["D"].sum(axis=1) * eps_pos
    sum_act = np.sqrt(n_pairs * np.maximum(ref["self_cost"], 0.0) / params.w_self)
    self_ = 2.0 * params.w_self * sum_act * 2.0 * eps_pos
    return world + self_ + 2e-6 * np.abs(ref["cfg_cost"])


def cost_tolerance(ref, n_pairs, T, params=OC.CostParams(), eps_pos=4e-6):
    """Per trajectory-candidate bound on |cost_gpu - cost_oracle|.  A term w (max(0, eta - e))^2
    moves by at most 2 w act |de| when its clearance moves by de; sphere clearances carry the
    position error eps_pos, pair clearances two of them, and sum_p act_p <= sqrt(P sum_p act_p^2)
    bounds the pair activations from the stored self cost.  A relative 2e-6 covers FP32 rounding
    of the per-configuration sums."""
    per_cfg = cfg_cost_tolerance(ref, n_pairs, params, eps_pos)
    return per_cfg.reshape(-1, T).sum(axis=1) + 1e-6 * np.abs(ref["cost_traj"]) + 1e-9


def grad_tolerance(ref):
    """Per-configuration bound on |grad_gpu - grad_oracle| of the FP32 path: 1e-4 (|J|_inf + 1e-3)
    of the configuration's joint gradient (the acceptance band of the FP32 path against FP64)."""
    J = ref["J"]
    return 1e-4 * (np.abs(J).max(axis=1, keepdims=True) + 1e-3)


def kink_free(ref, margin=1e-4):
    """Configurations whose gradient is single-valued with room to spare: every active sphere's
    runner-up cuboid and inside axis are at least `margin` away."""
    active = ref["D"] > 0
    m = np.where(active, ref["margin"], np.inf).min(axis=1)
    return (m > margin) & (ref["min_pair_dist"] > 1e-6)
