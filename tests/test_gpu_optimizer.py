"""GPU line-search + L-BFGS kernel against the oracle's step, and the optimiser end to end."""
import ctypes

import numpy as np
import pytest

from oracle import formats as F
from oracle import optimizer as O
from synthetic import make_workload
from tests.gpu_helpers import dev, import_codes, make_context, need_gpu, torch

pytestmark = pytest.mark.gpu


def _state_case(n_traj=7, T=8, n_ls=4, m=3, seed=0):
    """Synthetic optimiser states and candidate results covering: Armijo at alpha=1, Armijo at a
    smaller alpha, no Armijo but a cheaper candidate, rejection, a skipped curvature pair, a full
    history ring, and an empty history."""
    rng = np.random.default_rng(seed)
    n = T * 7
    x = O.fp32(rng.normal(size=(n_traj, n)))
    g = O.pin_rows(O.fp32(rng.normal(size=(n_traj, n))), T)
    d = O.fp32(-g * rng.uniform(0.5, 1.5, size=(n_traj, n)))
    cost = rng.uniform(10, 20, size=n_traj)
    hist_len = np.array([2, 2, 2, 1, 2, m, 0])[:n_traj]  # trajectory 5: a full ring
    hist_head = np.array([2, 2, 2, 1, 2, 1, 0])[:n_traj]
    S = O.fp32(O.pin_rows(rng.normal(size=(n_traj, m, n)) * 0.1, T))
    Y = O.fp32(S * rng.uniform(0.5, 2.0, size=(n_traj, m, n)))  # positive curvature
    rho = 1.0 / np.einsum("tmn,tmn->tm", S, Y)
    gd = np.einsum("tn,tn->t", g, d)
    cc = np.empty((n_traj, n_ls))
    for t in range(n_traj):
        armijo = cost[t] + 1e-4 * np.array(O.ALPHAS[:n_ls]) * gd[t]
        if t == 0:
            cc[t] = armijo - 1.0
        elif t == 1:
            cc[t] = armijo + np.array([1.0, 0.5, -0.5, -1.0])
        elif t == 2:
            cc[t] = cost[t] + np.array([0.5, -1e-9, 0.3, 0.2])  # below cost, above Armijo line
        elif t == 3:
            cc[t] = cost[t] + 1.0
        else:
            cc[t] = armijo - np.array([2.0, 1.0, 0.5, 0.1])
    cg = O.fp32(rng.normal(size=(n_traj, n_ls, n)))
    cg[4] = g[4][None]  # y = 0 -> curvature pair skipped
    return dict(T=T, n_ls=n_ls, m=m, x=x, g=g, d=d, cost=cost, hist_len=hist_len, hist_head=hist_head, S=S, Y=Y,
                rho=rho, cand_cost=cc, cand_grad=cg)


def _oracle_step(case, t):
    m = case["m"]
    L, H = int(case["hist_len"][t]), int(case["hist_head"][t])
    slots = [(H - L + i) % m for i in range(L)]  # oldest first
    st = O.TrajState(x=case["x"][t].copy(), g=case["g"][t].copy(), d=case["d"][t].copy(), cost=float(case["cost"][t]),
                     hist=[(case["S"][t, s].copy(), case["Y"][t, s].copy(), float(case["rho"][t, s])) for s in slots])
    info = O.step(st, case["cand_cost"][t], case["cand_grad"][t], case["T"], m)
    return st, info


@pytest.mark.parametrize("T,m", [(8, 3), (19, 3), (48, 8), (64, 8)])
def test_step_matches_oracle(T, m):
    """Every variables-per-lane instantiation class: 7T = 56 (one per lane), 133 (ragged, three per
    lane), 336 (six, the benchmark's horizon) and 448 (seven, the longest horizon), with a short and
    the full eight-pair history."""
    need_gpu()
    from paper_2310_07854_amd import Shape, _lib as L

    case = _state_case(T=T, m=m, seed=T + m)
    T, n_ls, m = case["T"], case["n_ls"], case["m"]
    n_traj, n = case["x"].shape
    wl = make_workload("tiny")
    ctx = make_context(wl, {})
    shape = Shape(n_traj, 1, T, n_ls)
    ws = ctx.new_workspace(shape)
    # candidate gradients as the stored joint gradient of configuration ((traj*n_ls + i)*T + t)
    J = case["cand_grad"].reshape(n_traj * n_ls * T, 7)
    import_codes(ctx, "joint_grad", ws, shape, F.quantize(J, "f32"))
    f32 = lambda a: dev(a, torch.float32)
    bufs = dict(x=f32(case["x"]), g=f32(case["g"]), d=f32(case["d"]), cost=dev(case["cost"], torch.float64),
                s=f32(case["S"]), y=f32(case["Y"]), rho=dev(case["rho"], torch.float64),
                hl=dev(case["hist_len"], torch.int32), hh=dev(case["hist_head"], torch.int32),
                acc=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"),
                fl=torch.zeros(n_traj, dtype=torch.int32, device="cuda:0"))
    st = L.LbfgsStateC(n_traj, T, n_ls, m, O.MAX_STEP, *[bufs[k].data_ptr() for k in
                                              ("x", "g", "d", "cost", "s", "y", "rho", "hl", "hh", "acc", "fl")])
    cc = dev(case["cand_cost"].reshape(-1), torch.float64)
    qn = torch.zeros(n_traj * n_ls * T, 7, device="cuda:0")
    ctx._call("vapr_optimizer_step", ctypes.byref(st), ws.data_ptr(), ws.numel(), cc.data_ptr(), qn.data_ptr())
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in bufs.items()}
    qn = qn.cpu().numpy().reshape(n_traj, n_ls, n)
    expect_acc = [0, 2, 1, -1, 0, 0, 0]
    for t in range(n_traj):
        ost, info = _oracle_step(case, t)
        assert got["acc"][t] == info["accepted"] == expect_acc[t], t
        assert got["hl"][t] == len(ost.hist), t
        assert bool(got["fl"][t] & 1) == info["curvature_ok"], t
        assert bool(got["fl"][t] & 2) == info["reset"], t
        np.testing.assert_array_equal(got["x"][t], ost.x)
        np.testing.assert_array_equal(got["g"][t], ost.g)
        assert got["cost"][t] == ost.cost
        np.testing.assert_allclose(got["d"][t], ost.d, rtol=1e-5, atol=1e-6 * np.abs(ost.d).max())
        for i in range(n_ls):
            np.testing.assert_allclose(qn[t, i], O.fp32(ost.x + O.ALPHAS[i] * got["d"][t]), rtol=0, atol=0)
        if info["curvature_ok"]:
            slot = (int(case["hist_head"][t]) if info["accepted"] >= 0 else 0) % m
            np.testing.assert_array_equal(got["s"][t, slot], ost.hist[-1][0])
            np.testing.assert_array_equal(got["y"][t, slot], ost.hist[-1][1])


def test_optimizer_descends_on_batched_workload():
    need_gpu()
    from paper_2310_07854_amd import TrajectoryOptimizer

    wl = make_workload("batched")
    ctx = make_context(wl, {})
    T = wl.T
    opt = TrajectoryOptimizer(ctx, wl.n_worlds, wl.traj_per_world, T, n_ls=wl.n_ls, m=8)
    x0 = dev(wl.q.reshape(wl.n_traj, wl.n_ls, T, 7)[:, 0], torch.float32)
    opt.init(x0)
    c_prev = opt.cost.clone()
    c0 = c_prev.clone()
    for _ in range(15):
        opt.step()
        c = opt.cost.clone()
        assert bool(torch.all(c <= c_prev))  # accepted steps never raise a trajectory's cost
        c_prev = c
    torch.cuda.synchronize()
    x = opt.x.reshape(wl.n_traj, T, 7)
    assert torch.equal(x[:, 0], x0[:, 0]) and torch.equal(x[:, -1], x0[:, -1])  # pinned start/goal
    assert float(opt.cost.sum()) < 0.7 * float(c0.sum())


def test_graph_replays_match_eager_steps():
    """One captured iteration replayed many times, with eager work and synchronisation in between,
    equals the same number of eager iterations bit for bit at every step."""
    need_gpu()
    from paper_2310_07854_amd import TrajectoryOptimizer

    wl = make_workload("batched")
    ctx = make_context(wl, {"sphere_pos": "f16", "sphere_dist": ("e4m3", -10), "sphere_grad": ("e4m3", -1)})
    T = wl.T
    x0 = dev(wl.q.reshape(wl.n_traj, wl.n_ls, T, 7)[:, 0], torch.float32)
    eager = TrajectoryOptimizer(ctx, wl.n_worlds, wl.traj_per_world, T, n_ls=wl.n_ls, m=8)
    graph = TrajectoryOptimizer(ctx, wl.n_worlds, wl.traj_per_world, T, n_ls=wl.n_ls, m=8)
    eager.init(x0)
    graph.init(x0)
    graph.capture()
    for it in range(6):
        eager.step()
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda:0").sum().item()  # unrelated eager work between replays
        assert torch.equal(eager.x, graph.x), it
        assert torch.equal(eager.cost, graph.cost), it
        assert torch.equal(eager.d, graph.d), it
        assert torch.equal(eager.hist_len, graph.hist_len), it


@pytest.mark.parametrize("parts", [2, 3, 4])
def test_partitioned_optimizer_matches_one_optimizer(parts):
    """The batch split by worlds over contexts and streams (uneven splits included: 4 worlds in 3
    parts) gives the single optimiser's iterates, costs and flags bit for bit, with a stored-mode
    reduced-precision assignment and the swept term off."""
    need_gpu()
    from paper_2310_07854_amd import PartitionedOptimizer, TrajectoryOptimizer

    wl = make_workload("batched")
    prec = {"link_poses": ("f16", -15), "sphere_pos": ("f16", -15), "sphere_dist": ("e4m3", -10),
            "sphere_grad": ("e4m3", -1), "joint_grad": ("e4m3", 0)}
    ctx = make_context(wl, prec)
    T = wl.T
    x0 = dev(wl.q.reshape(wl.n_traj, wl.n_ls, T, 7)[:, 0], torch.float32)
    one = TrajectoryOptimizer(ctx, wl.n_worlds, wl.traj_per_world, T, n_ls=wl.n_ls, m=8)
    split = PartitionedOptimizer(ctx, wl.n_worlds, wl.traj_per_world, T, n_ls=wl.n_ls, m=8, parts=parts)
    assert len(split.parts) == min(parts, wl.n_worlds)
    one.init(x0)
    split.init(x0)
    for it in range(6):
        one.step()
        split.step()
        if it % 2 == 1:
            assert torch.equal(split.x, one.x), it
            assert torch.equal(split.cost, one.cost), it
            assert torch.equal(split.flags, one.flags), it
    prof_parts = split.parts
    assert all(c.precision == ctx.precision for c, _, _ in prof_parts)
    split.close()


def test_stream_concurrency_probe():
    """The probe behind PartitionedOptimizer's streams: a stream is not concurrent with itself, and
    the streams concurrent_streams returns are concurrent."""
    need_gpu()
    from paper_2310_07854_amd.optim import concurrent_streams, streams_run_concurrently

    s = torch.cuda.Stream()
    assert not streams_run_concurrently([s, s])
    got = concurrent_streams(3)
    assert len(got) == 3 and streams_run_concurrently(got)
