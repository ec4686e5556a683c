"""Training data, training and evaluation of the learned seeder around the batched optimiser.

Problems come as arrays: worlds (already uploaded to the context, one per problem), start and goal
[W, 7], and initial trajectories [W, S, T, 7].
  endpoints_free      start and goal are collision-free: no sphere penetrates a cuboid (clearance
                      > 0), no self pair overlaps and the joint limits hold
  trajectories_free   every timestep of a trajectory is collision-free
  solve               run the optimiser from the initial trajectories; final trajectories and costs,
                      collision-free flags and, per problem, the first iteration at which any of its
                      trajectories was collision-free
  select_targets      the 8 lowest-cost collision-free solutions of each problem as deviations from
                      the straight line (fewer than 8: the rest marked invalid)
  train               Adam on shuffled batches
All cost, gradient, optimiser and network arithmetic runs in libvapr's kernels; this module moves
tensors and picks rows (sorting, indexing).
"""
from __future__ import annotations

from typing import Dict, Tuple

import torch

from .context import Context, Shape
from .optim import TrajectoryOptimizer
from .seeding import N_SEEDS, SeedNet, deviations, features


def configs_free(ctx: Context, q: torch.Tensor, shape: Shape) -> torch.Tensor:
    """[B] bool: every sphere clears every cuboid, every self pair is apart and the joint limits
    hold (the library's collision check of the forward pass)."""
    ws = ctx.new_workspace(shape)
    ctx.cost_fwd(q.reshape(-1, 7).contiguous(), shape, ws=ws)
    return ctx.collision_free(ws, shape)


def endpoints_free(ctx: Context, start: torch.Tensor, goal: torch.Tensor) -> torch.Tensor:
    """[W] bool: start and goal of every problem are collision-free."""
    W = start.shape[0]
    q = torch.stack([start, goal], dim=1)  # [W, 2, 7]: one trajectory of 2 timesteps per world
    return configs_free(ctx, q, Shape(W, 1, 2, 1)).view(W, 2).all(dim=1)


def trajectories_free(ctx: Context, x: torch.Tensor) -> torch.Tensor:
    """[W, S] bool for trajectories x [W, S, T, 7]: every timestep collision-free."""
    W, S, T, _ = x.shape
    return configs_free(ctx, x, Shape(W, S, T, 1)).view(W, S, T).all(dim=2)


def solve(ctx: Context, x0: torch.Tensor, iters: int, n_ls: int = 4, check_every: int = 1
          ) -> Dict[str, torch.Tensor]:
    """Optimise x0 [W, S, T, 7] for `iters` iterations.  Returns x [W, S, T, 7], cost [W, S] (FP64),
    free [W, S], first_free [W] (iteration index, 0 = the initial trajectories, -1 = never within
    `iters`)."""
    W, S, T, _ = x0.shape
    opt = TrajectoryOptimizer(ctx, W, S, T, n_ls=n_ls)
    opt.init(x0)
    first = torch.full((W,), -1, dtype=torch.int64, device=x0.device)

    def mark(it):
        free = trajectories_free(ctx, opt.x.view(W, S, T, 7)).any(dim=1)
        first.masked_fill_(free & (first < 0), it)

    mark(0)
    for it in range(1, iters + 1):
        opt.step()
        if it % check_every == 0 or it == iters:
            mark(it)
    x = opt.x.view(W, S, T, 7).clone()
    return {"x": x, "cost": opt.cost.view(W, S).clone(), "free": trajectories_free(ctx, x), "first_free": first}


def select_targets(sol: Dict[str, torch.Tensor], start: torch.Tensor, goal: torch.Tensor, diverse: bool = False
                   ) -> Tuple[torch.Tensor, torch.Tensor]:
    """targets [W, 8, T, 7] (deviations from the straight line) and valid [W, 8] (float 0/1).
    diverse=False: the 8 lowest-cost collision-free solutions.  diverse=True: the lowest-cost one,
    then seven more picked one at a time as the collision-free solution farthest (L2 over the whole
    deviation) from those already picked, so that the network's slots learn different routes
    rather than near-copies of the cheapest one."""
    x, cost, free = sol["x"], sol["cost"], sol["free"]
    W, S, T, _ = x.shape
    masked = torch.where(free, cost, torch.full_like(cost, float("inf")))
    dev = deviations(x.contiguous(), start.contiguous(), goal.contiguous())
    if diverse:
        rows = torch.arange(W, device=x.device)
        flat = dev.reshape(W, S, T * 7)
        dist = torch.cdist(flat, flat)                                  # [W, S, S]
        first = torch.argmin(masked, dim=1)
        order = [first]
        ok = [torch.isfinite(masked[rows, first])]
        avail = free.clone()
        avail[rows, first] = False
        near = dist[rows, first]                                        # distance to the picked set
        for _ in range(1, N_SEEDS):
            score = torch.where(avail, near, torch.full_like(near, -1.0))
            nxt = torch.argmax(score, dim=1)
            ok.append(score[rows, nxt] >= 0)
            order.append(nxt)
            avail[rows, nxt] = False
            near = torch.minimum(near, dist[rows, nxt])
        order = torch.stack(order, dim=1)
        ok = torch.stack(ok, dim=1)
    else:
        order = torch.argsort(masked, dim=1, stable=True)[:, :N_SEEDS]
        ok = torch.isfinite(torch.gather(masked, 1, order))
    idx = order.view(W, N_SEEDS, 1, 1).expand(W, N_SEEDS, T, 7)
    picked = torch.gather(dev, 1, idx)
    return torch.where(ok.view(W, N_SEEDS, 1, 1), picked, torch.zeros_like(picked)), ok.float()


def train(net: SeedNet, data: Dict[str, torch.Tensor], steps: int, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log_every: int = 0):
    """Adam on batches drawn without replacement from shuffled epochs of `data` (start, goal, occ
    [N, 512], targets [N, 8, 32, 7], valid [N, 8]); returns the batch losses."""
    n = data["start"].shape[0]
    x_all = features(data["start"], data["goal"], data["occ"])
    tgt = data["targets"].reshape(n, -1).contiguous()
    valid = data["valid"].contiguous()
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    losses = []
    perm, pos = torch.randperm(n, generator=gen), 0
    for s in range(steps):
        if pos + batch > n:
            perm, pos = torch.randperm(n, generator=gen), 0
        idx = perm[pos:pos + batch].to(x_all.device)
        pos += batch
        vb = valid[idx].contiguous()
        nv = int(vb.sum().item())
        if nv == 0:
            continue
        loss = net.train_step(x_all[idx].contiguous(), tgt[idx].contiguous(), vb, nv, lr=lr)
        losses.append(loss)
        if log_every and (s + 1) % log_every == 0:
            print(f"# seeder step {s + 1}/{steps}: loss {float(loss.item()):.5f}", flush=True)
    return [float(l.item()) for l in losses]
