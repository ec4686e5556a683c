"""The allocation-free forward + backward entry point (vapr_cost_fwd_bwd_noalloc, stored tensors in
the library's static per-device workspace) against vapr_cost_fwd + vapr_cost_bwd with a caller
workspace: the same kernels on the same inputs, so every output must be bit-identical.  Two calls in
a row, the second on a smaller batch, under FP32 and under a reduced-precision assignment."""
import numpy as np
import pytest

from synthetic import make_workload
from tests.gpu_helpers import dev, make_context, need_gpu, torch

pytestmark = pytest.mark.gpu

PAPER_LIKE = {"link_poses": ("f16", -15), "sphere_pos": ("f16", -15), "sphere_dist": ("e4m3", -10),
              "sphere_grad": ("e4m3", -1), "joint_grad": ("e4m3", 0)}


def reference(ctx, q, shape, up):
    cfg = torch.empty(shape.B, dtype=torch.float32, device=q.device)
    cost, ws = ctx.cost_fwd(q, shape, cost_cfg=cfg)
    grad = ctx.cost_bwd(q, ws, up)
    return cost, cfg, grad


def static_path(ctx, q, shape, up):
    cost = torch.full((shape.n_tc,), float("nan"), dtype=torch.float64, device=q.device)
    cfg = torch.full((shape.B,), float("nan"), dtype=torch.float32, device=q.device)
    grad = torch.full((shape.B, 7), float("nan"), dtype=torch.float32, device=q.device)
    ctx.cost_fwd_bwd_noalloc(q, shape, cost, grad, grad_cost_traj=up, cost_cfg=cfg)
    return cost, cfg, grad


@pytest.mark.parametrize("prec", [{}, PAPER_LIKE], ids=["f32", "paper_like"])
def test_noalloc_matches_workspace_path(prec):
    need_gpu()
    from paper_2310_07854_amd import Shape

    wl = make_workload("batched")  # 4 worlds x 32 seeds x 32 timesteps x 4 candidates, 40 cuboids
    ctx = make_context(wl, prec)
    full = Shape(wl.n_worlds, wl.traj_per_world, wl.T, wl.n_ls)
    small = Shape(2, 8, wl.T, wl.n_ls)
    q_all = dev(wl.q, torch.float32)
    # the smaller batch: the first 8 trajectories of worlds 0 and 1
    per_world = wl.traj_per_world * wl.n_ls * wl.T
    rows = np.concatenate([np.arange(w * per_world, w * per_world + small.B // 2) for w in range(2)])
    q_small = q_all[torch.as_tensor(rows, device=q_all.device)].contiguous()
    rng = np.random.default_rng(5)
    cases = [(full, q_all, dev(rng.uniform(0.5, 2.0, full.n_tc), torch.float64)), (small, q_small, None)]
    ctx.cost_fwd(q_all, full)  # builds the lookup tables
    for shape, q, up in cases:
        print(f"[noalloc] {list(prec) and 'paper_like' or 'f32'} B={shape.B}", flush=True)
        got = static_path(ctx, q, shape, up)
        want = reference(ctx, q, shape, up)
        torch.cuda.synchronize()
        for name, g, w in zip(("cost_traj", "cost_cfg", "grad_q"), got, want):
            assert torch.isfinite(w).all(), name
            assert torch.equal(g, w), (name, (g - w).abs().max().item())
    ctx.sync()
    ctx.close()


def test_noalloc_rejects_what_it_cannot_do():
    need_gpu()
    from paper_2310_07854_amd import Shape, VaprError, _lib as L

    wl = make_workload("tiny")
    ctx = make_context(wl, {})
    shape = Shape(wl.n_worlds, wl.traj_per_world, wl.T, wl.n_ls)
    q = dev(wl.q, torch.float32)
    cost = torch.empty(shape.n_tc, dtype=torch.float64, device=q.device)
    grad = torch.empty(shape.B, 7, dtype=torch.float32, device=q.device)
    # the lookup tables are built by the first ordinary forward pass
    with pytest.raises(VaprError) as e:
        ctx.cost_fwd_bwd_noalloc(q, shape, cost, grad)
    assert e.value.status == L.E_STATE
    ctx.cost_fwd(q, shape)
    ctx.cost_fwd_bwd_noalloc(q, shape, cost, grad)
    # a batch whose workspace exceeds the static 64 MiB: refused before any launch
    big = Shape(1, 4096, 48, 1)
    assert ctx.workspace_size(big) > 64 << 20
    qb = torch.zeros(big.B, 7, dtype=torch.float32, device=q.device)
    gb = torch.empty_like(qb)
    cb = torch.empty(big.n_tc, dtype=torch.float64, device=q.device)
    with pytest.raises(VaprError) as e:
        ctx.cost_fwd_bwd_noalloc(qb, big, cb, gb)
    assert e.value.status == L.E_INVALID
    assert "static workspace" in str(e.value)
    ctx.sync()
    ctx.close()
