"""GPU parity of the inverse-kinematics workload (pose cost of link 8 against per-world goals,
with the collision, self and bound costs; one configuration per trajectory) against the FP64
oracle (oracle/cost.py: pose_term inside fwd_bwd), and the optimiser with free rows.

Tolerances: the pose cost moves by at most 2 w |e| |de| when a pose value moves by de, and FP32
forward kinematics keeps every pose value within 4e-6 of the exact one (the bound used for the
link-pose tensor); the joint gradient uses the same per-configuration bound as the other parity
tests, at configurations whose active spheres are away from kinks."""
import ctypes

import numpy as np
import pytest

from oracle import cost as OC
from oracle import formats as F
from oracle import optimizer as O
from synthetic import Worlds, make_configs, make_robot, make_worlds
from synthetic.generators import Workload
from tests.gpu_helpers import (cost_tolerance, dev, export_codes, grad_tolerance, import_codes, kink_free, make_context,
                               need_gpu, oracle_precision, shape_of, torch)

pytestmark = pytest.mark.gpu

W_GP, W_GR = 100.0, 10.0


def _rotation(rng):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0, np.pi)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def ik_workload(seed=31, n_worlds=3, seeds=100, n_cuboids=20, n_pairs=300):
    robot = make_robot(60, n_pairs, seed=seed)
    w = make_worlds(n_worlds, n_cuboids, seed=seed)
    q = make_configs(n_worlds * seeds, seed=seed)
    rng = np.random.default_rng(seed)
    goals = np.zeros((n_worlds, 3, 4))
    for k in range(n_worlds):
        goals[k, :, :3] = _rotation(rng)
        goals[k, :, 3] = rng.uniform(-0.5, 0.5, size=3)
    goals = goals.astype(np.float32).astype(np.float64)
    return Workload("ik", robot, w, seeds, 1, 1, q), goals


def run(wl, goals, prec=None, recompute=False):
    ctx = make_context(wl, prec if prec is not None else {}, recompute,
                       params={"w_goal_pos": W_GP, "w_goal_rot": W_GR})
    ctx.set_goals(goals)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    cost, ws = ctx.cost_fwd(q, shape)
    grad = ctx.cost_bwd(q, ws)
    torch.cuda.synchronize()
    ref = OC.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, 1, 1, prec=oracle_precision(prec or {}, recompute),
                     params=OC.CostParams(w_goal_pos=W_GP, w_goal_rot=W_GR), goals=goals)
    return ctx, ws, shape, cost.cpu().numpy(), grad.cpu().numpy(), ref


def pose_tolerance(wl, goals, ref, eps=4e-6):
    from oracle.kinematics import forward_kinematics

    T = forward_kinematics(wl.robot.fixed_tf, wl.q)
    g = goals[ref["world"]]
    e_p = np.sqrt(np.sum((T[:, 8, :3, 3] - g[:, :, 3]) ** 2, axis=1))
    e_r = np.sqrt(np.sum((T[:, 8, :3, :3] - g[:, :, :3]) ** 2, axis=(1, 2)))
    return 2 * W_GP * e_p * np.sqrt(3) * eps + 2 * W_GR * e_r * 3 * eps + 2e-6 * ref["pose_cost"] + 1e-9


def check(wl, goals, ctx, ws, shape, cost, grad, ref):
    ptol = pose_tolerance(wl, goals, ref)
    pc = ctx.ws_export("pose_cost", ws, shape).cpu().numpy().astype(np.float64)
    perr = np.abs(pc - ref["pose_cost"])
    assert np.all(perr <= ptol), f"pose cost: max err {perr.max():.3e}, ratio {(perr / ptol).max():.3f}"
    ctol = cost_tolerance(ref, wl.robot.n_pairs, 1) + ptol
    cerr = np.abs(cost - ref["cost_traj"])
    assert np.all(cerr <= ctol), f"cost: max err {cerr.max():.3e}, ratio {(cerr / ctol).max():.3f}"
    ok = kink_free(ref)
    gerr = np.abs(grad - ref["grad_q"])
    bad = (gerr > grad_tolerance(ref)).any(axis=1) & ok
    assert not bad.any(), f"grad: {int(bad.sum())} configs out of tolerance, max err {gerr[ok].max():.3e}"
    assert ok.mean() > 0.5


@pytest.mark.parametrize("seeds,n_worlds", [(100, 3), (37, 2), (64, 1)])
def test_ik_fp32_parity(seeds, n_worlds):
    need_gpu()
    wl, goals = ik_workload(seeds=seeds, n_worlds=n_worlds)
    ctx, ws, shape, cost, grad, ref = run(wl, goals)
    assert np.all(ref["pose_cost"] > 0)
    check(wl, goals, ctx, ws, shape, cost, grad, ref)


@pytest.mark.parametrize("prec,recompute", [
    ({"link_poses": "f16", "sphere_pos": "f16", "sphere_dist": ("e4m3", -10), "sphere_grad": ("e4m3", -2),
      "joint_grad": ("e4m3", 2)}, False),
    ({"link_poses": "bf16", "sphere_pos": "bf16"}, False),
    ({"sphere_pos": "f16", "joint_grad": ("e5m2", 0)}, True),
])
def test_ik_quantised_and_recompute(prec, recompute):
    """The pose wrench of the backward pass comes from the poses the backward pass reads: stored
    (quantised) link poses, or poses recomputed from q, exactly as in the oracle's emulation.  The
    stored joint gradient then goes through its own format: compared through the decoded values."""
    need_gpu()
    wl, goals = ik_workload(seed=32, seeds=80, n_worlds=2)
    ctx, ws, shape, cost, grad, ref = run(wl, goals, prec, recompute)
    ptol = pose_tolerance(wl, goals, ref)
    pc = ctx.ws_export("pose_cost", ws, shape).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(pc - ref["pose_cost"]) <= ptol)
    ok = kink_free(ref)
    # a stored pose or position within FP32 error of a rounding boundary may take the neighbouring
    # code on the GPU (the stage tests bound which); its configuration then reads a different stored
    # value, so the gradient is compared where every stored L and S code equals the oracle's
    same = np.ones(shape.B, dtype=bool)
    for name, key in (("link_poses", "L_codes"), ("sphere_pos", "S_codes")):
        if name == "link_poses" and recompute:
            continue
        codes = export_codes(ctx, name, ws, shape).reshape(shape.B, -1)
        same &= np.all(codes == np.asarray(ref[key]).reshape(shape.B, -1).astype(codes.dtype), axis=1)
    # per value the chance of a flip is about twice the FP32 error over the code step: with 276
    # stored values per configuration that leaves about 87 % of configurations untouched at FP16
    assert same.mean() > 0.75
    ok &= same
    fmt = prec.get("joint_grad", "f32")
    fmt, k = (fmt, 0) if isinstance(fmt, str) else fmt
    # value band: the FP32 computation bound, widened by one code step of the joint-gradient format
    # where the value sits near a rounding boundary
    tol = grad_tolerance(ref)
    lo = F.roundtrip(ref["J"] - tol, fmt, k)[1]
    hi = F.roundtrip(ref["J"] + tol, fmt, k)[1]
    inside = (grad >= np.minimum(lo, hi) - 1e-30) & (grad <= np.maximum(lo, hi) + 1e-30)
    bad = ~inside.all(axis=1) & ok
    assert not bad.any(), f"{int(bad.sum())} configs outside the band"


def test_goals_required_and_cleared():
    need_gpu()
    from paper_2310_07854_amd import VaprError

    wl, goals = ik_workload(seed=33, seeds=10, n_worlds=3)
    ctx = make_context(wl, {})
    ctx.set_goals(goals[:2])  # fewer goals than worlds in the pass
    with pytest.raises(VaprError):
        ctx.cost_fwd(dev(wl.q, torch.float32), shape_of(wl))
    bad = goals.copy()
    bad[0, 0, 0] = 2.0
    with pytest.raises(VaprError):
        ctx.set_goals(bad)
    ctx.set_goals(None)
    cost, ws = ctx.cost_fwd(dev(wl.q, torch.float32), shape_of(wl))
    with pytest.raises(VaprError):
        ctx.ws_export("pose_cost", ws, shape_of(wl))


def test_ik_optimizer_step_with_free_rows_matches_oracle():
    """One optimiser iteration on one-configuration trajectories with free rows: the accepted
    candidate, the new point and gradient equal the oracle's step bit for bit, and the direction
    agrees to FP64-dot rounding."""
    need_gpu()
    from paper_2310_07854_amd import Shape, _lib as L

    rng = np.random.default_rng(4)
    n_traj, T, n_ls, m, n = 9, 1, 4, 3, 7
    wl, _ = ik_workload(seed=34, seeds=4, n_worlds=1)
    ctx = make_context(wl, {})
    x = O.fp32(rng.normal(size=(n_traj, n)))
    g = O.fp32(rng.normal(size=(n_traj, n)))
    d = O.fp32(-g * rng.uniform(0.5, 1.5, size=(n_traj, n)))
    cost = rng.uniform(10, 20, size=n_traj)
    gd = np.einsum("tn,tn->t", g, d)
    cc = cost[:, None] + 1e-4 * np.array(O.ALPHAS[:n_ls])[None] * gd[:, None] - rng.uniform(0, 1, size=(n_traj, n_ls))
    cc[3] = cost[3] + 1.0  # rejected
    cg = O.fp32(rng.normal(size=(n_traj, n_ls, n)))
    shape = Shape(n_traj, 1, T, n_ls)
    ws = ctx.new_workspace(shape)
    import_codes(ctx, "joint_grad", ws, shape, F.quantize(cg.reshape(-1, 7), "f32"))
    f32 = lambda a: dev(a, torch.float32)
    z = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda:0")
    bufs = dict(x=f32(x), g=f32(g), d=f32(d), cost=dev(cost, torch.float64), s=z(n_traj, m, n), y=z(n_traj, m, n),
                rho=torch.zeros(n_traj, m, dtype=torch.float64, device="cuda:0"),
                hl=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"),
                hh=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"),
                acc=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"),
                fl=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"))
    st = L.LbfgsStateC(n_traj, T, n_ls, m, O.MAX_STEP, *[bufs[k].data_ptr() for k in
                                              ("x", "g", "d", "cost", "s", "y", "rho", "hl", "hh", "acc", "fl")], 1)
    ccd = dev(cc.reshape(-1), torch.float64)
    qn = torch.zeros(n_traj * n_ls, 7, device="cuda:0")
    ctx._call("vapr_optimizer_step", ctypes.byref(st), ws.data_ptr(), ws.numel(), ccd.data_ptr(), qn.data_ptr())
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in bufs.items()}
    for t in range(n_traj):
        ost = O.TrajState(x=x[t].copy(), g=g[t].copy(), d=d[t].copy(), cost=float(cost[t]))
        info = O.step(ost, cc[t], cg[t], T, m, pin=False)
        assert got["acc"][t] == info["accepted"], t
        np.testing.assert_array_equal(got["x"][t], ost.x)
        np.testing.assert_array_equal(got["g"][t], ost.g)
        np.testing.assert_allclose(got["d"][t], ost.d, rtol=1e-5, atol=1e-6 * np.abs(ost.d).max())
    assert (got["acc"] >= 0).sum() >= 7 and np.any(got["g"] != 0)


def test_ik_optimizer_descends():
    need_gpu()
    from paper_2310_07854_amd import TrajectoryOptimizer

    wl, goals = ik_workload(seed=35, seeds=256, n_worlds=2, n_cuboids=10)
    ctx = make_context(wl, {}, params={"w_goal_pos": W_GP, "w_goal_rot": W_GR})
    ctx.set_goals(goals)
    opt = TrajectoryOptimizer(ctx, wl.n_worlds, wl.traj_per_world, 1, n_ls=4, m=8, pin_ends=False)
    x0 = dev(wl.q.reshape(-1, 1, 7), torch.float32)
    opt.init(x0)
    c0 = opt.cost.clone()
    c_prev = c0.clone()
    for _ in range(30):
        opt.step()
        c = opt.cost.clone()
        assert bool(torch.all(c <= c_prev))
        c_prev = c
    torch.cuda.synchronize()
    assert float(opt.cost.sum()) < 0.3 * float(c0.sum())
    assert not torch.equal(opt.x.reshape(-1, 7), x0.reshape(-1, 7))
