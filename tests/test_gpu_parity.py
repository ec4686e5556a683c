"""GPU cost path against the FP64 oracle.

* FP32 end to end (tiny and batched workloads): trajectory costs within the derived cost tolerance,
  joint gradients within the gradient tolerance on kink-free configurations.
* Every stage under reduced formats, each fed the oracle's own stored inputs through workspace
  import: stored codes equal the oracle's except, by at most one step, where the oracle value lies
  within float32 computation error of a rounding boundary.
* Ragged and degenerate shapes, the full 196,608-configuration batch on sampled trajectories,
  determinism, the autograd Function, and error paths.
"""
import dataclasses

import numpy as np
import pytest

from oracle import cost as OC
from oracle import formats as F
from oracle.geometry import obb_signed_distance
from synthetic import Worlds, make_configs, make_robot, make_workload, make_worlds
from synthetic.generators import Workload
from tests.gpu_helpers import (ORACLE_KEY, TENSORS, cfg_cost_tolerance, compare_codes, cost_tolerance, dev, export_codes, grad_tolerance,
                               import_codes, kink_free, make_context, need_gpu, oracle_precision, shape_of, torch)

pytestmark = pytest.mark.gpu

PRECISIONS = {
    # FP32 codes are the computed values: the code tests then report how much of each band the FP32
    # arithmetic uses
    "f32": {t: "f32" for t in TENSORS},
    "f16": {t: "f16" for t in TENSORS},
    "bf16": {t: "bf16" for t in TENSORS},
    "fp8": {"link_poses": ("e4m3", -7), "sphere_pos": ("e4m3", -7), "sphere_dist": ("e4m3", -10),
            "sphere_grad": ("e5m2", -9), "joint_grad": ("e5m2", -5)},
    "fp6": {"link_poses": ("e3m2", -3), "sphere_pos": ("e3m2", -3), "sphere_dist": ("e3m2", -6),
            "sphere_grad": ("e3m2", 2), "joint_grad": ("e3m2", 6)},
    "mixed_fp4": {"link_poses": ("e4m3", -7), "sphere_pos": ("e4m3", -7), "sphere_dist": ("e2m1", -3),
                  "sphere_grad": ("e2m1", 5), "joint_grad": ("e4m3", 2)},
    # FP16 poses and positions with FP4 distances and sphere gradients
    "f16_fp4": {"link_poses": "f16", "sphere_pos": "f16", "sphere_dist": ("e2m1", -3),
                "sphere_grad": ("e2m1", 5), "joint_grad": ("e4m3", 2)},
    # the benchmark's headline assignment with the scales it calibrates on the 196,608-configuration
    # batch: poses and positions from the arm's reach, the rest from their FP32 magnitude
    "paper_like": {"link_poses": ("f16", -15), "sphere_pos": ("f16", -15), "sphere_dist": ("e4m3", -10),
                   "sphere_grad": ("e4m3", -1), "joint_grad": ("e4m3", 0)},
}


def dense_workload(seed=11, n_worlds=2, tpw=8, T=8, n_ls=4, n_spheres=60, n_cuboids=40, n_pairs=300):
    """Collision-rich variant: cuboids twice the standard size and joint angles reaching past the
    limits, so that many spheres, pairs and limits are active."""
    robot = make_robot(n_spheres, n_pairs, seed=seed)
    w = make_worlds(n_worlds, n_cuboids, seed=seed)
    w = Worlds(pose=w.pose, half_ext=(w.half_ext * 2.0).astype(np.float32).astype(np.float64))
    B = n_worlds * tpw * n_ls * T
    q = make_configs(B, seed=seed, lo=-3.2, hi=3.2)
    return Workload("dense", robot, w, tpw, T, n_ls, q)


def run_gpu(ctx, wl, upstream=None):
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    cost, ws = ctx.cost_fwd(q, shape)
    up = dev(upstream, torch.float64) if upstream is not None else None
    grad = ctx.cost_bwd(q, ws, up)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), grad.cpu().numpy(), ws, shape, q


def run_oracle(wl, prec=None, recompute=False, upstream=None):
    return OC.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls,
                      prec=oracle_precision(prec, recompute), upstream=upstream)


def check_fp32(wl, ref, cost, grad, min_checked=0.5):
    """Costs within the FP32 bound everywhere; gradients within it on every kink-free
    configuration, which must be at least `min_checked` of them."""
    tol = cost_tolerance(ref, wl.robot.n_pairs, wl.T)
    err = np.abs(cost - ref["cost_traj"])
    assert np.all(err <= tol), f"cost: max err {err.max():.3e}, worst ratio {(err / tol).max():.3f}"
    ok = kink_free(ref)
    gerr = np.abs(grad - ref["grad_q"])
    gtol = grad_tolerance(ref)
    bad = (gerr > gtol).any(axis=1) & ok
    assert not bad.any(), f"grad: {int(bad.sum())} configs out of tolerance, max err {gerr[ok].max():.3e}"
    assert ok.mean() > min_checked
    # the acceptance band 1e-4 (|g|_inf + 1e-3) per configuration, reported beside the test's band
    acc = 1e-4 * (np.abs(ref["grad_q"]).max(axis=1, keepdims=True) + 1e-3)
    print(f"[fp32] cost err/bound {(err / tol).max():.3f}; grad err/band {(gerr / gtol)[ok].max():.3f}, "
          f"err/acceptance {(gerr / acc)[ok].max():.3f} over {int(ok.sum())} configurations")


@pytest.mark.parametrize("name", ["tiny", "batched"])
def test_fp32_end_to_end(name):
    need_gpu()
    wl = make_workload(name)
    ctx = make_context(wl)
    cost, grad, ws, shape, _ = run_gpu(ctx, wl)
    ref = run_oracle(wl, {})
    check_fp32(wl, ref, cost, grad)
    # stored FP32 tensors: positions and poses to float32 computation accuracy
    S = export_codes(ctx, "sphere_pos", ws, shape).view(np.float32).reshape(ref["S"].shape)
    assert np.abs(S - ref["S"]).max() < 4e-6
    Lv = export_codes(ctx, "link_poses", ws, shape).view(np.float32).reshape(ref["L"].shape)
    assert np.abs(Lv - ref["L"]).max() < 4e-6
    D = export_codes(ctx, "sphere_dist", ws, shape).view(np.float32).reshape(ref["D"].shape)
    assert np.abs(D - ref["D"]).max() < 8e-6


def test_fp32_dense_with_upstream_and_recompute():
    need_gpu()
    wl = dense_workload()
    up = np.random.default_rng(3).uniform(-2, 2, size=wl.B // wl.T)
    for recompute in (False, True):
        ctx = make_context(wl, {}, recompute)
        cost, grad, _, _, _ = run_gpu(ctx, wl, up)
        ref = run_oracle(wl, {}, recompute, up)
        assert (ref["D"] > 0).mean() > 0.05
        check_fp32(wl, ref, cost, grad)


def _eligible_pairs(robot):
    link = robot.sphere_link
    n = link.shape[0]
    return np.array([(a, b) for a in range(n) for b in range(a + 1, n) if abs(int(link[a]) - int(link[b])) >= 2],
                    dtype=np.int32)


@pytest.mark.parametrize("kind", ["hubs", "all_eligible"])
def test_self_pair_tables(kind):
    """Robots whose self-pair lists are far from the benchmark's: three hub spheres paired with every
    eligible partner (about 50 each) plus 200 random pairs, and every eligible pair (about 1,250).
    Against the FP32 oracle."""
    need_gpu()
    wl = dense_workload(seed=13, n_worlds=1, tpw=4, T=8, n_ls=2)
    el = _eligible_pairs(wl.robot)
    if kind == "hubs":
        rng = np.random.default_rng(2)
        hub = el[(el[:, 0] == 0) | (el[:, 1] == 59) | (el[:, 0] == 30) | (el[:, 1] == 30)]
        rest = el[rng.choice(len(el), 200, replace=False)]
        pairs = np.unique(np.concatenate([hub, rest]), axis=0)
    else:
        pairs = el
    wl = dataclasses.replace(wl, robot=dataclasses.replace(wl.robot, pairs=pairs.astype(np.int32)))
    ctx = make_context(wl)
    cost, grad, _, _, _ = run_gpu(ctx, wl)
    ref = run_oracle(wl, {})
    assert ref["self_cost"].max() > 0
    check_fp32(wl, ref, cost, grad)
    print(f"[self pairs] {kind}: {len(pairs)} pairs")
    ctx.close()


@pytest.mark.parametrize("pname", list(PRECISIONS))
def test_stage_fk_codes(pname):
    need_gpu()
    prec = PRECISIONS[pname]
    wl = dense_workload()
    ctx = make_context(wl, prec)
    _, _, ws, shape, _ = run_gpu(ctx, wl)
    ref = run_oracle(wl, prec)
    for name in ("link_poses", "sphere_pos"):
        fmt, k = ctx.precision[name]
        got = export_codes(ctx, name, ws, shape)
        compare_codes(name, fmt, k, got, ref[ORACLE_KEY[name] + "_codes"], ref[ORACLE_KEY[name]])


@pytest.mark.parametrize("pname", list(PRECISIONS))
def test_stage_sphere_cost_codes(pname):
    need_gpu()
    prec = PRECISIONS[pname]
    wl = dense_workload()
    ctx = make_context(wl, prec)
    ref = run_oracle(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    ws = ctx.new_workspace(shape)
    import_codes(ctx, "sphere_pos", ws, shape, ref["S_codes"])
    ctx.ws_import("bound_cost", ws, shape, dev(ref["bound_cost"], torch.float32))
    cost, _ = ctx.cost_fwd(q, shape, ws=ws, first=2)
    torch.cuda.synchronize()
    # spheres whose closest cuboid or inside axis is within 1e-4 of switching have a set-valued
    # gradient; their G is not compared
    kink = (ref["D"] > 0) & (ref["margin"] < 1e-4)
    for name in ("sphere_dist", "sphere_grad"):
        fmt, k = ctx.precision[name]
        got = export_codes(ctx, name, ws, shape)
        ex = np.repeat(kink[..., None], 3, axis=2) if name == "sphere_grad" else None
        compare_codes(name, fmt, k, got, ref[ORACLE_KEY[name] + "_codes"], ref[ORACLE_KEY[name]], ex)
    sc = ctx.ws_export("self_cost", ws, shape).cpu().numpy()
    np.testing.assert_allclose(sc, ref["self_cost"], rtol=2e-5, atol=2e-4)


@pytest.mark.parametrize("pname", ["f16", "fp8", "mixed_fp4"])
def test_stage_reduce(pname):
    need_gpu()
    prec = PRECISIONS[pname]
    wl = dense_workload()
    ctx = make_context(wl, prec)
    ref = run_oracle(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    ws = ctx.new_workspace(shape)
    import_codes(ctx, "sphere_dist", ws, shape, ref["D_codes"])
    ctx.ws_import("self_cost", ws, shape, dev(ref["self_cost"], torch.float32))
    ctx.ws_import("bound_cost", ws, shape, dev(ref["bound_cost"], torch.float32))
    cfg = torch.empty(shape.B, dtype=torch.float32, device="cuda:0")
    cost, _ = ctx.cost_fwd(q, shape, ws=ws, first=3, cost_cfg=cfg)
    # identical stored inputs: only FP64 summation order and the FP32 q differences remain
    np.testing.assert_allclose(cost.cpu().numpy(), ref["cost_traj"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(cfg.cpu().numpy(), ref["cfg_cost"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("pname", list(PRECISIONS))
@pytest.mark.parametrize("recompute", [False, True])
def test_stage_adjoint_codes(pname, recompute):
    need_gpu()
    prec = PRECISIONS[pname]
    wl = dense_workload()
    up = np.random.default_rng(5).uniform(0.5, 2.0, size=wl.B // wl.T)
    ctx = make_context(wl, prec, recompute)
    ref = run_oracle(wl, prec, recompute, up)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    ws = ctx.new_workspace(shape)
    if not recompute:
        import_codes(ctx, "link_poses", ws, shape, ref["L_codes"])
    import_codes(ctx, "sphere_grad", ws, shape, ref["G_codes"])
    grad = ctx.cost_bwd(q, ws, dev(up, torch.float64))
    torch.cuda.synchronize()
    fmt, k = ctx.precision["joint_grad"]
    got = export_codes(ctx, "joint_grad", ws, shape)
    compare_codes("joint_grad", fmt, k, got, ref["J_codes"], ref["J"])
    # grad_q is the dequantised stored gradient
    np.testing.assert_array_equal(grad.cpu().numpy().astype(np.float64).reshape(-1),
                                  F.dequantize(got, fmt, k))


def shuffled_robot(robot, seed):
    """The same robot with its spheres listed in a seeded random order (links interleaved), so
    consecutive spheres change link often and every link's spheres span several groups."""
    perm = np.random.default_rng(seed).permutation(robot.n_spheres)  # new sphere i is old perm[i]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    pairs = np.sort(inv[robot.pairs], axis=1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))].astype(np.int32)
    return dataclasses.replace(robot, sphere_center=robot.sphere_center[perm],
                               sphere_radius=robot.sphere_radius[perm],
                               sphere_link=robot.sphere_link[perm].astype(np.int32), pairs=pairs)


@pytest.mark.parametrize("case", ["ragged", "no_cuboids", "no_pairs", "one_sphere", "worlds_in_wave",
                                  "many_spheres", "shuffled_links", "shuffled_many_spheres", "many_cuboids",
                                  "max_sizes", "staged_blocks"])
def test_edge_shapes(case):
    need_gpu()
    kw = dict(seed=21, n_worlds=3, tpw=3, T=5, n_ls=2, n_spheres=37, n_cuboids=7, n_pairs=40)
    if case == "max_sizes":  # the largest robot and world the boundary accepts
        kw.update(n_worlds=2, tpw=2, T=4, n_spheres=256, n_pairs=4096, n_cuboids=256)
    if case in ("many_spheres", "shuffled_many_spheres"):
        # more than 8 sphere groups: the kernel that reads positions from HBM
        kw.update(n_spheres=150, n_pairs=400)
    if case == "no_cuboids":
        kw["n_cuboids"] = 0
    if case == "many_cuboids":  # more than 64 cuboids: more than two culling mask words per voxel
        kw["n_cuboids"] = 100
    if case == "no_pairs":
        kw["n_pairs"] = 0
    if case == "one_sphere":
        kw.update(n_spheres=1, n_pairs=0)
    if case == "worlds_in_wave":
        kw.update(n_worlds=9, tpw=1, T=4, n_ls=1)
    if case == "staged_blocks":
        # 96 configurations per world: of the six 64-configuration blocks, four lie in one world and
        # read its cuboids from their LDS copy, two straddle a world boundary and read them from memory
        kw.update(n_worlds=4, tpw=2, T=24, n_ls=2, n_cuboids=40)
    wl = dense_workload(**kw)
    if case.startswith("shuffled"):
        wl = dataclasses.replace(wl, robot=shuffled_robot(wl.robot, seed=5))
        assert np.any(np.diff(wl.robot.sphere_link) < 0)
    ctx = make_context(wl, {})
    cost, grad, _, _, _ = run_gpu(ctx, wl)
    ref = run_oracle(wl, {})
    # 256 spheres against 256 doubled cuboids and 4,096 pairs put about half of the configurations
    # within the kink margin of some sphere or pair; the rest are still checked exactly
    check_fp32(wl, ref, cost, grad, min_checked=0.3 if case == "max_sizes" else 0.5)


def _sampled_oracle(wl, tcs, prec):
    """Oracle on whole trajectory candidates `tcs` of a workload, each in its own world."""
    T = wl.T
    rows = np.concatenate([np.arange(tc * T, (tc + 1) * T) for tc in tcs])
    worlds = [(tc // wl.n_ls) // wl.traj_per_world for tc in tcs]
    sub = Worlds(pose=wl.worlds.pose[worlds], half_ext=wl.worlds.half_ext[worlds])
    ref = OC.fwd_bwd(wl.robot, sub, wl.q[rows], 1, T, 1, prec=oracle_precision(prec))
    return ref, rows


@pytest.mark.parametrize("pname", ["f32", "paper_like"])
def test_large_batch_sampled(pname):
    """The full 196,608-configuration batch in the benchmark's launch configuration, compared on 12
    sampled trajectories (the last one included) with the oracle.  FP32: costs and gradients within
    the FP32 bounds.  Headline assignment: every stored code of all five tensors, stage by stage --
    S everywhere, D and G on configurations whose S codes equal the oracle's, J where L, S and G
    do -- then costs where S and D agree and gradients (the dequantised J) as codes."""
    need_gpu()
    prec = {} if pname == "f32" else PRECISIONS[pname]
    wl = make_workload("large")
    ctx = make_context(wl, prec)
    cost, grad, ws, shape, _ = run_gpu(ctx, wl)
    rng = np.random.default_rng(7)
    tcs = np.sort(rng.choice(shape.n_tc, size=12, replace=False))
    tcs[-1] = shape.n_tc - 1
    ref, rows = _sampled_oracle(wl, tcs, prec)
    if pname == "f32":
        sub = dataclasses.replace(wl, q=wl.q[rows])
        check_fp32(sub, ref, cost[tcs], grad[rows])
        ctx.close()
        return
    B = len(rows)
    codes = {name: export_codes(ctx, name, ws, shape).reshape(shape.B, -1)[rows] for name in TENSORS}
    same = {}
    for name in TENSORS:
        key = ORACLE_KEY[name]
        fmt, k = ctx.precision[name]
        want = ref[key + "_codes"].reshape(B, -1)
        if name in ("link_poses", "sphere_pos"):
            rows_ok = np.ones(B, dtype=bool)
        elif name in ("sphere_dist", "sphere_grad"):
            rows_ok = same["sphere_pos"]
        else:
            rows_ok = same["sphere_pos"] & same["sphere_grad"] & same["link_poses"]
        kink = np.repeat(((ref["D"] > 0) & (ref["margin"] < 1e-4))[..., None], 3, axis=2).reshape(B, -1)
        ex = (kink if name == "sphere_grad" else np.zeros_like(want, dtype=bool)) | ~rows_ok[:, None]
        compare_codes(name, fmt, k, codes[name], want, ref[key].reshape(B, -1), ex)
        same[name] = np.all(codes[name] == want, axis=1) & rows_ok
        assert rows_ok.mean() > 0.5, (name, rows_ok.mean())
    # configuration costs where the configuration's S and D codes all equal the oracle's: FP32 bound
    cfg = torch.empty(shape.B, dtype=torch.float32, device="cuda:0")
    ctx.cost_fwd(dev(wl.q, torch.float32), shape, ws=ws, cost_cfg=cfg)
    cfg = cfg.cpu().numpy()[rows].astype(np.float64)
    c_ok = same["sphere_pos"] & same["sphere_dist"]
    tol = cfg_cost_tolerance(ref, wl.robot.n_pairs)
    err = np.abs(cfg - ref["cfg_cost"])
    assert c_ok.mean() > 0.5 and np.all(err[c_ok] <= tol[c_ok]), (c_ok.mean(), (err / tol)[c_ok].max())
    print(f"[large/{pname}] configuration cost error / bound max {(err / tol)[c_ok].max():.3f} over "
          f"{int(c_ok.sum())}/{B}; J rows compared {int(same['joint_grad'].sum())}/{B}")
    # the gradient handed to torch is the dequantised stored J
    fmt, k = ctx.precision["joint_grad"]
    np.testing.assert_array_equal(grad[rows].astype(np.float64).reshape(-1),
                                  F.dequantize(codes["joint_grad"].reshape(-1), fmt, k))
    assert np.all(np.isfinite(cost)) and np.all(np.isfinite(grad))
    ctx.close()


def test_deterministic():
    need_gpu()
    wl = dense_workload()
    ctx = make_context(wl, PRECISIONS["mixed_fp4"])
    c1, g1, ws1, shape, _ = run_gpu(ctx, wl)
    c2, g2, ws2, _, _ = run_gpu(ctx, wl)
    assert np.array_equal(c1, c2) and np.array_equal(g1, g2)
    for name in TENSORS:
        assert np.array_equal(export_codes(ctx, name, ws1, shape), export_codes(ctx, name, ws2, shape))


def test_autograd_function():
    need_gpu()
    from paper_2310_07854_amd import trajectory_cost

    wl = dense_workload()
    ctx = make_context(wl, {})
    shape = shape_of(wl)
    w = np.random.default_rng(9).uniform(0.5, 1.5, size=shape.n_tc)
    q = dev(wl.q, torch.float32).requires_grad_(True)
    loss = (trajectory_cost(q, ctx, shape) * dev(w)).sum()
    loss.backward()
    ref = run_oracle(wl, {}, False, w)
    ok = kink_free(ref)
    g = q.grad.cpu().numpy()
    assert np.all(np.abs(g - ref["grad_q"])[ok] <= grad_tolerance(ref)[ok])
    # central differences of the GPU cost itself on a few coordinates
    rng = np.random.default_rng(10)
    for b in rng.choice(np.nonzero(ok)[0], size=6, replace=False):
        j = int(rng.integers(0, 7))
        h = 1e-3
        qp, qm = q.detach().clone(), q.detach().clone()
        qp[b, j] += h
        qm[b, j] -= h
        fd = ((trajectory_cost(qp, ctx, shape) - trajectory_cost(qm, ctx, shape)) * dev(w)).sum().item() / (2 * h)
        assert fd == pytest.approx(g[b, j], rel=2e-2, abs=0.5)


def test_error_paths():
    need_gpu()
    from paper_2310_07854_amd import VaprError, _lib as L

    wl = make_workload("tiny")
    ctx = make_context(wl, {})
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    cost, ws = ctx.cost_fwd(q, shape)
    ctx.set_precision({"sphere_pos": "f16"})
    with pytest.raises(VaprError) as e:
        ctx.cost_bwd(q, ws)
    assert e.value.status == L.E_STATE
    with pytest.raises(VaprError) as e:
        ctx.cost_fwd(q, shape, ws=ws[:16])
    assert e.value.status == L.E_INVALID
    bad = dataclasses.replace(wl.robot, fixed_tf=wl.robot.fixed_tf * 2.0)
    with pytest.raises(VaprError) as e:
        ctx.set_robot(bad)
    assert e.value.status == L.E_INVALID
    fresh = ctx.new_workspace(shape)
    with pytest.raises(VaprError) as e:
        ctx.cost_bwd(q, fresh)
    assert e.value.status == L.E_STATE


def test_workspace_state():
    """The workspace's forward-pass record: a freed workspace whose address torch hands out again is
    not mistaken for the forward pass it held; changed cost parameters invalidate it; a header
    overwritten behind the library's back
    makes the backward kernel write NaN and vapr_sync report it; a call rejected for its arguments leaves
    the record as it was."""
    need_gpu()
    from paper_2310_07854_amd import VaprError, _lib as L

    wl = make_workload("tiny")
    ctx = make_context(wl, {})
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    ws = ctx.new_workspace(shape)
    ctx.cost_fwd(q, shape, ws=ws)
    good = ctx.cost_bwd(q, ws)
    torch.cuda.synchronize()
    assert torch.isfinite(good).all()
    # recycled address: same size, same place under the caching allocator
    ptr = ws.data_ptr()
    del ws
    ws2 = ctx.new_workspace(shape)
    assert ws2.data_ptr() == ptr
    with pytest.raises(VaprError) as e:
        ctx.cost_bwd(q, ws2)
    assert e.value.status == L.E_STATE
    # cost parameters changed between the passes
    ctx.cost_fwd(q, shape, ws=ws2)
    ctx.set_cost_params(w_smooth=2.0)
    with pytest.raises(VaprError) as e:
        ctx.cost_bwd(q, ws2)
    assert e.value.status == L.E_STATE
    ctx.set_cost_params()
    # a forward pass into a workspace that already held one, with an argument error: no record left
    ctx.cost_fwd(q, shape, ws=ws2)
    with pytest.raises(VaprError) as e:
        ctx.cost_fwd(q, shape, ws=ws2[:16])  # same address, too small: rejected before any change
    assert e.value.status == L.E_INVALID
    ctx.cost_bwd(q, ws2)
    # header overwritten behind the library's back: NaN gradients, flag reported by sync
    ctx.cost_fwd(q, shape, ws=ws2)
    ws2[:64].zero_()
    grad = ctx.cost_bwd(q, ws2)
    with pytest.raises(VaprError) as e:
        ctx.sync()
    assert e.value.status == L.E_STATE
    assert torch.isnan(grad).all()
    ctx.sync()  # reported once
    ctx.cost_fwd(q, shape, ws=ws2)
    again = ctx.cost_bwd(q, ws2)
    ctx.sync()
    assert torch.equal(again, good)
    ctx.close()


@pytest.mark.parametrize("wname,pname", [("dense", "f32"), ("dense", "mixed_fp4"), ("batched", "f32"),
                                         ("large", "paper_like"), ("edge", "f32"), ("dense_k32", "f32"),
                                         ("dense_k100", "paper_like")])
def test_culling_is_exact(wname, pname):
    """Skipping cuboids that are out of reach changes nothing: stored codes, self costs and
    trajectory costs are bit-identical with and without culling (32, 40, 64 and 100 cuboids cover
    one, two and more mask words per voxel)."""
    need_gpu()
    prec = {} if pname == "f32" else PRECISIONS[pname]
    if wname == "dense":
        wl = dense_workload()
    elif wname.startswith("dense_k"):
        wl = dense_workload(n_cuboids=int(wname[len("dense_k"):]))
    elif wname == "edge":
        wl = dense_workload(seed=21, n_worlds=9, tpw=1, T=4, n_ls=1, n_spheres=37, n_cuboids=7, n_pairs=40)
    else:
        wl = make_workload(wname)
    ctx = make_context(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    out = []
    for cull in (True, False):
        ctx.set_culling(cull)
        cost, ws = ctx.cost_fwd(q, shape)
        torch.cuda.synchronize()
        out.append((cost.cpu().numpy(), {n: export_codes(ctx, n, ws, shape) for n in ("sphere_dist", "sphere_grad")},
                    ctx.ws_export("self_cost", ws, shape).cpu().numpy()))
    (c1, t1, s1), (c2, t2, s2) = out
    assert np.array_equal(c1, c2)
    assert np.array_equal(s1, s2)
    for n in t1:
        assert np.array_equal(t1[n], t2[n]), n


@pytest.mark.parametrize("wname", ["dense", "large"])
def test_culling_grid_is_conservative(wname):
    """The culling grid the kernels read never drops a cuboid that can matter: at random points
    (float32, assigned to voxels with the kernels' float32 arithmetic), every cuboid whose bit is
    clear, and every cuboid at points outside the grid, is at least eta + the largest sphere radius
    away (FP64 signed distance)."""
    need_gpu()
    wl = dense_workload() if wname == "dense" else make_workload(wname)
    ctx = make_context(wl, {})
    reach = OC.CostParams().eta + float(wl.robot.sphere_radius.max())
    rng = np.random.default_rng(7)
    for w in range(min(3, wl.worlds.pose.shape[0])):
        info, mask = ctx.culling_grid(w)
        n = info["n"]
        assert n > 0 and mask is not None and mask.shape == (n ** 3, info["mask_words"])
        o = np.array(info["origin"], dtype=np.float32)
        inv = np.float32(info["inv_cell"])
        span = n / float(inv)
        p = (o.astype(np.float64) - 0.1 * span + rng.random((20000, 3)) * 1.2 * span).astype(np.float32)
        f = (p - o) * inv                                            # float32, as in the kernels
        inside = np.all((f >= 0) & (f < np.float32(n)), axis=1)
        v = np.floor(f).astype(np.int64)
        vid = np.where(inside, (v[:, 2] * n + v[:, 1]) * n + v[:, 0], 0)
        for k in range(wl.worlds.pose.shape[1]):
            P = wl.worlds.pose[w, k]
            sd, _, _ = obb_signed_distance(p.astype(np.float64), P[:, :3], P[:, 3], wl.worlds.half_ext[w, k])
            bit = (mask[vid, k // 32] >> np.uint32(k % 32)) & np.uint32(1)
            dropped = ~inside | (bit == 0)
            assert np.all(sd[dropped] >= reach), (w, k, float(sd[dropped].min()))


@pytest.mark.parametrize("wname", ["tiny", "dense", "tiny_no_pairs"])
def test_collision_free(wname):
    """vapr_collision_free against the oracle's clearances: a configuration is free when every
    sphere clears every cuboid, every self pair is apart and the joints are within their limits.
    Configurations whose smallest clearance is within FP32 rounding of zero may go either way."""
    need_gpu()
    if wname == "dense":
        wl = dense_workload()
    else:
        wl = make_workload("tiny")
        if wname == "tiny_no_pairs":
            wl = dataclasses.replace(wl, robot=dataclasses.replace(wl.robot, pairs=wl.robot.pairs[:0]))
    ctx = make_context(wl, {})
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    _, ws = ctx.cost_fwd(q, shape)
    got = ctx.collision_free(ws, shape).cpu().numpy()
    ref = run_oracle(wl)
    r = wl.robot.sphere_radius.astype(np.float64)
    S = ref["S"]
    a, b = wl.robot.pairs[:, 0], wl.robot.pairs[:, 1]
    pair_clear = np.linalg.norm(S[:, a] - S[:, b], axis=-1) - r[a] - r[b]
    world_clear = OC.CostParams().eta - ref["D"].max(axis=1)  # the smallest clearance when it is < eta
    min_clear = np.minimum(world_clear, pair_clear.min(axis=1)) if pair_clear.shape[1] else world_clear
    want = (min_clear > 0) & (ref["bound_cost"] == 0)
    sure = np.abs(min_clear) > 1e-5
    assert np.array_equal(got[sure].astype(bool), want[sure])
    print(f"[collision_free] {wname}: {int(want.sum())} of {want.size} free, {int((~sure).sum())} undecided")
    ctx.close()


def test_seed_deviations_invert_trajectories():
    need_gpu()
    from paper_2310_07854_amd import seeding

    rng = np.random.default_rng(3)
    n = 5
    start = dev(rng.uniform(-2, 2, (n, 7)), torch.float32)
    goal = dev(rng.uniform(-2, 2, (n, 7)), torch.float32)
    y = dev(rng.normal(0, 0.3, (n, 8 * 32 * 7)), torch.float32)
    traj = seeding.trajectories(y, start, goal)
    got = seeding.deviations(traj, start, goal).cpu().numpy().reshape(n, 8, 32, 7)
    want = y.cpu().numpy().reshape(n, 8, 32, 7).astype(np.float64)
    want[:, :, 0] = 0.0
    want[:, :, 31] = 0.0
    # line + y rounded to FP32 and the line subtracted again: within one ulp of |line + y|
    tr = traj.cpu().numpy().reshape(n, 8, 32, 7).astype(np.float64)
    assert np.all(np.abs(got - want) <= np.spacing(np.abs(tr).astype(np.float32)).astype(np.float64) * 1.01)
    assert np.all(got[:, :, 0] == 0) and np.all(got[:, :, 31] == 0)


def test_scale_overflow_guard_and_far_reach():
    """FP16 sphere positions at a scale the arm can leave (2^-16, what a sampled calibration picks
    for the benchmark arm: at most 0.9995 m) are refused before any launch; at the scale of the
    arm's reach, configurations beyond that range are stored finite, and the cuboids placed on their
    farthest spheres cost what the oracle's emulation gives."""
    need_gpu()
    from oracle.kinematics import forward_kinematics, sphere_positions
    from paper_2310_07854_amd import Shape, VaprError, _lib as L

    from paper_2310_07854_amd.search import scale_for

    # the benchmark arm with its links stretched by 40 %: some configurations pass 1 m
    robot = make_workload("batched").robot
    stretched = robot.fixed_tf.copy()
    stretched[:, :, 3] *= 1.4
    robot = dataclasses.replace(robot, fixed_tf=F.fp32(stretched).astype(np.float64))
    rng = np.random.default_rng(12)
    q = rng.uniform(-2.9, 2.9, size=(20000, 7))
    P = sphere_positions(forward_kinematics(robot.fixed_tf, q), robot.sphere_center, robot.sphere_link)
    far = np.abs(P).max(axis=(1, 2))
    pick = np.argsort(far)[-8:]
    assert far[pick].min() > 65504.0 * 2.0 ** -16, far[pick]
    qs = F.fp32(q[pick]).astype(np.float64)
    # one world, a cuboid on each configuration's farthest sphere
    Ps = sphere_positions(forward_kinematics(robot.fixed_tf, qs), robot.sphere_center, robot.sphere_link)
    idx = np.abs(Ps).max(axis=2).argmax(axis=1)
    pose = np.zeros((1, 8, 3, 4))
    pose[0, :, :, :3] = np.eye(3)
    pose[0, :, :, 3] = Ps[np.arange(8), idx]
    worlds = Worlds(pose=F.fp32(pose).astype(np.float64), half_ext=np.full((1, 8, 3), 0.05))
    wl2 = Workload("far", robot, worlds, 1, 8, 1, qs)
    ctx = make_context(wl2)
    lp, sp = ctx.reach()
    assert sp >= far.max()
    shape = Shape(1, 1, 8, 1)
    qd = dev(qs, torch.float32)
    ctx.set_precision({"sphere_pos": ("f16", -16)})
    with pytest.raises(VaprError) as e:
        ctx.cost_fwd(qd, shape)
    assert e.value.status == L.E_INVALID and "reach" in str(e.value)
    ks = scale_for("f16", sp)
    prec = {"link_poses": ("f16", scale_for("f16", lp)), "sphere_pos": ("f16", ks), "sphere_dist": ("e4m3", -10),
            "sphere_grad": ("e4m3", -1), "joint_grad": ("e4m3", 0)}
    ctx.set_precision(prec)
    cost, ws = ctx.cost_fwd(qd, shape)
    grad = ctx.cost_bwd(qd, ws)
    torch.cuda.synchronize()
    S = ctx.ws_export("sphere_pos", ws, shape)
    Sv = F.dequantize(F.unpack(S.cpu().numpy(), "f16", shape.B * robot.sphere_radius.shape[0] * 3), "f16", ks)
    assert np.all(np.isfinite(Sv)) and np.abs(Sv).max() > 0.9995
    ref = run_oracle(wl2, prec)
    Dg = export_codes(ctx, "sphere_dist", ws, shape).reshape(shape.B, -1)
    assert np.all(F.dequantize(Dg[np.arange(8), idx], "e4m3", -10) > 0)   # the far spheres collide
    tol = cost_tolerance(ref, robot.n_pairs, 8)
    c = cost.cpu().numpy()
    assert np.all(np.abs(c - ref["cost_traj"]) <= tol) and np.all(np.isfinite(grad.cpu().numpy()))
    ctx.close()
