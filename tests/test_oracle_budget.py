"""Pins of the first-order error budget (oracle/budget.py) against brute force: every sensitivity
against central differences of the oracle's forward + backward pass with one stored element
perturbed, the budget against one-ulp perturbations of every stored element, the emulated FP16
error within the budget, and ulp_at against numpy's float16 spacing and the rounding it bounds."""
import numpy as np
import pytest

from oracle import budget as BG
from oracle import cost as OC
from oracle import formats as F
from synthetic import Worlds, make_configs, make_robot, make_worlds

SHAPES = {"L": (8, 12), "S": (None, 3), "D": (None,), "G": (None, 3), "J": (7,)}


def small_workload(seed=5, W=2, tpw=2, T=4, n_s=20, K=10, P=40):
    """Collision-rich batch: cuboids twice the standard size, so that many spheres and pairs are
    active; 20 spheres keep the brute force quick."""
    robot = make_robot(n_s, P, seed=seed)
    w = make_worlds(W, K, seed=seed)
    worlds = Worlds(pose=w.pose, half_ext=(w.half_ext * 2.0).astype(np.float32).astype(np.float64))
    q = make_configs(W * tpw * T, seed=seed)
    return robot, worlds, q, tpw, T


def away_from_kinks(robot, worlds, ref, gap=1e-3):
    return BG.smooth_configurations(robot, ref, worlds.pose, worlds.half_ext, gap)


def run(robot, worlds, q, tpw, T, perturb=None, prec=None):
    return OC.fwd_bwd(robot, worlds, q, tpw, T, 1, prec=prec, perturb=perturb)


def element_shape(name, B, n_s):
    return (B,) + tuple(n_s if s is None else s for s in SHAPES[name])


def test_sensitivities_match_central_differences():
    robot, worlds, q, tpw, T = small_workload()
    B, n_s = q.shape[0], robot.sphere_radius.shape[0]
    ref = run(robot, worlds, q, tpw, T)
    keep = away_from_kinks(robot, worlds, ref)
    assert keep.sum() >= 6, keep
    assert (ref["D"][keep] > 0).sum() >= 10 and ref["self_cost"][keep].max() > 0
    sens = BG.sensitivities(robot, ref, worlds.pose, worlds.half_ext, OC.CostParams(), np.ones(B), True)
    checks = {"S": ("cost_S", "grad_S", 1e-6), "D": ("cost_D", None, 1e-6), "G": (None, "grad_G", 1e-4),
              "L": (None, "grad_L", 1e-6)}
    worst = {}
    for name, (ck, gk, h) in checks.items():
        shp = element_shape(name, B, n_s)
        for idx in np.ndindex(*shp[1:]):
            delta = np.zeros(shp)
            delta[(slice(None),) + idx] = h
            up = run(robot, worlds, q, tpw, T, perturb={name: delta})
            dn = run(robot, worlds, q, tpw, T, perturb={name: -delta})
            if ck:
                fd = (up["cfg_cost"] - dn["cfg_cost"]) / (2 * h)
                an = sens[ck][(slice(None),) + idx]
                err = np.abs(fd - an)[keep]
                tol = 1e-5 * np.abs(an[keep]) + 1e-6
                assert np.all(err <= tol), (name, idx, fd[keep], an[keep])
                worst[ck] = max(worst.get(ck, 0.0), float(np.max(err / tol)))
            if gk:
                fd = (up["J_hat"] - dn["J_hat"]) / (2 * h)                         # [B, 7]
                sel = (slice(None), slice(None)) + idx
                an = sens[gk][sel]
                err = np.abs(fd - an)[keep]
                tol = 1e-5 * np.abs(an[keep]) + 1e-5 * (1.0 + np.abs(sens[gk][keep]).max())
                assert np.all(err <= tol), (name, idx, fd[keep], an[keep])
                worst[gk] = max(worst.get(gk, 0.0), float(np.max(err / tol)))
    # the joint gradient's own rounding enters with derivative one
    print("worst error / tolerance:", {k: f"{v:.2e}" for k, v in worst.items()})


def test_budget_matches_one_ulp_perturbations():
    """Half the output change of a one-ulp move of each stored element, summed over elements, is the
    budget's sum to first order (FP16 ulps)."""
    robot, worlds, q, tpw, T = small_workload(seed=8)
    B, n_s = q.shape[0], robot.sphere_radius.shape[0]
    prec = OC.Precision(**{t: ("f16", 0) for t in OC.TENSORS})
    bud = BG.error_budget(robot, worlds, q, tpw, T, 1, prec)
    ref = bud["ref"]
    keep = away_from_kinks(robot, worlds, ref, gap=5e-3)
    assert keep.sum() >= 4
    vals = {"L": ref["L"], "S": ref["S"], "D": ref["D"], "G": ref["G"], "J": ref["J"]}
    brute_cost = np.zeros(B)
    brute_grad = np.zeros((B, 7))
    for name, v in vals.items():
        ulp = F.ulp_at(v, "f16")
        for idx in np.ndindex(*v.shape[1:]):
            delta = np.zeros(v.shape)
            delta[(slice(None),) + idx] = ulp[(slice(None),) + idx]
            up = run(robot, worlds, q, tpw, T, perturb={name: delta})
            dn = run(robot, worlds, q, tpw, T, perturb={name: -delta})
            brute_cost += 0.25 * np.abs(up["cfg_cost"] - dn["cfg_cost"])   # half of the one-ulp change
            brute_grad += 0.25 * np.abs(up["J_hat"] - dn["J_hat"])
    budget_cfg = (bud["cost_parts"]["sphere_pos"] + bud["cost_parts"]["sphere_dist"])  # per trajectory
    brute_traj = brute_cost.reshape(-1, T).sum(axis=1)
    rel_c = np.abs(brute_traj - budget_cfg) / budget_cfg
    assert np.all(rel_c < 0.02), rel_c
    g_budget = bud["grad"][keep]
    rel_g = np.abs(brute_grad[keep] - g_budget) / g_budget
    assert np.all(rel_g < 0.05), rel_g.max()
    print(f"one-ulp brute force vs budget: cost within {rel_c.max():.1e}, gradient within {rel_g.max():.1e}")


@pytest.mark.parametrize("grad_fmt", ["f16", "bf16"])
def test_emulated_error_within_budget(grad_fmt):
    """The quantisation-emulating oracle differs from the unquantised one by no more than the
    budget (poses and positions FP16, the other three FP16 or BF16, where first order holds), on
    configurations away from kinks."""
    robot, worlds, q, tpw, T = small_workload(seed=9, W=2, tpw=4, T=4)
    fmt = "f16"
    prec = OC.Precision(link_poses=(fmt, 0), sphere_pos=(fmt, 0), sphere_dist=(grad_fmt, 0),
                        sphere_grad=(grad_fmt, 0), joint_grad=(grad_fmt, 0))
    bud = BG.error_budget(robot, worlds, q, tpw, T, 1, prec)
    ref = bud["ref"]
    emu = run(robot, worlds, q, tpw, T, prec=prec)
    dc = np.abs(emu["cost_traj"] - ref["cost_traj"])
    assert np.all(dc <= bud["cost"] * 1.01 + 1e-12), (dc / bud["cost"]).max()
    # a position moved by up to half an ulp must not cross a kink
    gap = float(F.ulp_at(np.abs(ref["S"]).max(), fmt))
    keep = away_from_kinks(robot, worlds, ref, gap=4 * gap)
    assert keep.sum() >= 4
    dg = np.abs(emu["J_hat"] - ref["J"])[keep]
    ratio = dg / bud["grad"][keep]
    assert np.all(ratio <= 1.01), ratio.max()
    print(f"{grad_fmt}: cost error / budget max {(dc / bud['cost']).max():.2f}, gradient {ratio.max():.2f}")


def test_recompute_mode_has_no_pose_term():
    robot, worlds, q, tpw, T = small_workload(seed=3)
    prec = OC.Precision(**{t: ("e4m3", 0) for t in OC.TENSORS}, recompute_poses=True)
    bud = BG.error_budget(robot, worlds, q, tpw, T, 1, prec)
    assert np.all(bud["grad_parts"]["link_poses"] == 0)
    assert np.all(bud["grad_parts"]["sphere_grad"] > 0)


@pytest.mark.parametrize("k", [0, -4, 3])
@pytest.mark.parametrize("fmt", F.REDUCED)
def test_ulp_at_bounds_rounding_tightly(fmt, k):
    """|dec(enc(x)) - x| <= ulp_at(x) / 2 for in-range x, with equality at the midpoints between
    neighbouring values (the ties)."""
    _, vals = F.magnitude_table(fmt)
    vals = vals[vals * 2.0 ** k < 1e38]  # scaled-up BF16 reaches past FP32 range: out of contract
    vmax = vals[-1] * 2.0 ** k
    rng = np.random.default_rng(1)
    lo = max(vals[1] * 2.0 ** k, 1e-30)
    x = np.exp(rng.uniform(np.log(lo), np.log(vmax), 20000)) * rng.choice([-1.0, 1.0], 20000)
    x = F.fp32(x).astype(np.float64)
    x = x[np.abs(x) <= vmax]
    _, xr = F.roundtrip(x, fmt, k)
    assert np.all(np.abs(xr - x) <= 0.5 * F.ulp_at(x, fmt, k))
    mids = 0.5 * (vals[1:] + vals[:-1]) * 2.0 ** k
    mids = mids[(F.fp32(mids) == mids) & (mids > 0)]
    _, mr = F.roundtrip(mids, fmt, k)
    assert np.all(np.abs(np.abs(mr - mids) - 0.5 * F.ulp_at(mids, fmt, k)) == 0)


def test_ulp_at_f16_against_numpy_spacing():
    rng = np.random.default_rng(2)
    x = np.exp(rng.uniform(np.log(1e-7), np.log(6e4), 50000))
    below = x.astype(np.float16)
    below = np.where(below.astype(np.float64) > x, np.nextafter(below, np.float16(0)), below)
    inside = below.astype(np.float64) < x   # x not itself representable
    want = np.spacing(below).astype(np.float64)
    assert np.array_equal(F.ulp_at(x, "f16")[inside], want[inside])
    # scales shift the grid exactly
    assert np.array_equal(F.ulp_at(x * 2.0 ** -5, "f16", -5), F.ulp_at(x, "f16") * 2.0 ** -5)


def test_half_ulp_of_emulated_types_matches_their_grid():
    """For an emulated ExMy type the budget's half-gap bounds the emulated rounding, tight at ties."""
    from oracle import exmy

    rng = np.random.default_rng(4)
    for E, M in [(3, 1), (2, 2), (5, 4), (4, 5), (5, 7)]:
        _, _, vmax = exmy.limits(E, M)
        x = F.fp32(np.exp(rng.uniform(np.log(1e-3), np.log(vmax), 5000))).astype(np.float64)
        _, xr = exmy.roundtrip(x, E, M)
        assert np.all(np.abs(xr - x) <= BG.half_ulp(x, f"e{E}m{M}")), (E, M)
