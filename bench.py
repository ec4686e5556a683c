"""Benchmark: one trajectory-optimisation iteration per step (candidate generation, kinematics,
sphere costs, aggregation, adjoint, line-search selection and L-BFGS update) over a batch of
64 worlds x 64 seeds x 48 timesteps = 196,608 configurations of a synthetic 7-joint arm with 60
spheres and 300 self pairs among 64 random cuboids per world.  Reports configuration evaluations
(cost + joint gradient) per second for a variable-precision assignment of the five stored tensors
and for FP32 on the same GPU.  The timed steps run on one stream by default; with --parts P > 1 the
batch is split by worlds over P contexts, each on a stream of its own (identical results; one
partition's kernels can fill the GPU while another's drain), and the same steps are also timed on
one stream.  The one-stream run gives the per-kernel times (HIP events recorded around each launch
on the stream the kernels run on) and the dominant kernel's roofline.  The FP64 oracle's rate on the host cores for a bounded sample is reported
beside it.

  python bench.py [--steps K] [--warmup W] [--precision NAME] [--parts P] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2
# (an FMA is two flops).  The 157.3 TFLOP/s figure needs packed FP32, which this build does not emit.
VALU_PEAK_TFLOPS = 78.6

# formats per stored tensor; power-of-two scales are calibrated per run (calibrate_scales)
PRECISIONS = {
    "f32": {},
    # the paper's per-tensor requirements: sphere positions FP16, distances and sphere gradients FP8;
    # link poses FP16 like the positions, joint gradients FP8
    "paper_like": {"link_poses": "f16", "sphere_pos": "f16", "sphere_dist": "e4m3", "sphere_grad": "e4m3",
                   "joint_grad": "e4m3"},
    "all_fp8": {"link_poses": "e4m3", "sphere_pos": "e4m3", "sphere_dist": "e4m3", "sphere_grad": "e5m2",
                "joint_grad": "e5m2"},
    "mixed_fp4": {"link_poses": "e4m3", "sphere_pos": "e4m3", "sphere_dist": "e2m1", "sphere_grad": "e2m1",
                  "joint_grad": "e4m3"},
}
TENSOR_NAMES = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad", "swept_grad")
BITS = {"f32": 32, "f16": 16, "bf16": 16, "e4m3": 8, "e5m2": 8, "e3m2": 6, "e2m1": 4}
N_WORLDS, TPW, T, N_LS, N_SPHERES, N_CUBOIDS, N_PAIRS = 64, 64, 48, 1, 60, 64, 300
HIST_M = 8
# world partitions (contexts on streams of their own) for the timed steps: with the sphere-cost
# kernel at three blocks per CU, one stream is the faster for the variable-precision assignments
PARTS = 1
# algorithmic FP32 operations of one sphere-cuboid test (FMA = 2): R^T p - R^T c (18),
# |u| - h (3), max(a, 0) (3), |max(a,0)|^2 (5), min(max_i a_i, 0) (3), key (1), running arg-min (2)
FLOPS_PER_SPHERE_CUBOID = 35
# one self pair: difference (3), squared norm (5), sqrt (1), clearance (2), activation (2)
FLOPS_PER_PAIR = 13


def fmt_of(prec, name):
    v = prec.get(name, "f32")
    return v if isinstance(v, str) else v[0]


def tensor_bytes(prec):
    """Algorithmic bytes per configuration of each stored tensor (no padding)."""
    vals = {"link_poses": 96, "sphere_pos": 3 * N_SPHERES, "sphere_dist": N_SPHERES,
            "sphere_grad": 3 * N_SPHERES, "joint_grad": 7}
    return {k: v * BITS[fmt_of(prec, k)] / 8.0 for k, v in vals.items()}


def optimizer_traj_bytes(jg_bytes, n, stats=None):
    """Algorithmic HBM bytes of one trajectory's optimiser update (mode 1, n variables, jg_bytes per
    stored joint-gradient element): x, g, d read and written; the selected candidate's gradient
    read when a candidate is accepted; the new (s, y) pair and its rho written when it is kept; the
    history pairs the two-loop recursion uses read (each 2 n FP32 values and an FP64 rho); n_ls
    candidates written; FP64 costs and the int32 state words.  `stats` holds the per-trajectory means
    over iterations (`accepted`, `pairs_written`, `pairs_read`); without it every candidate is taken
    as accepted with a full history of HIST_M pairs."""
    st = stats or {"accepted": 1.0, "pairs_written": 1.0, "pairs_read": float(HIST_M)}
    pair = 2 * n * 4 + 8
    return (3 * n * 4 * 2 + st["accepted"] * (n * jg_bytes + 8) + st["pairs_written"] * pair
            + st["pairs_read"] * pair + N_LS * n * 4 + N_LS * 8 + 8 + 8 + 16)


def optimizer_stats_add(torch, opt, prev_len, sums):
    """Adds, on the GPU, what one optimiser update touched per trajectory to `sums` (a float64
    tensor of four running totals: iterations, accepted candidates, kept (s, y) pairs, history pairs
    read by the two-loop recursion -- the history length after the update, or before the reset when
    the new direction was not a descent direction); `prev_len` is the history length before it."""
    a, f, ln = opt.accepted, opt.flags, opt.hist_len
    ok = a >= 0
    kept = ok & ((f & 1) != 0)
    reset = ok & ((f & 2) != 0)
    r = torch.where(reset, torch.clamp(prev_len + kept.to(prev_len.dtype), max=opt.m), ln)
    r = torch.where(ok, r, torch.zeros_like(r))
    n = float(ok.numel())
    sums += torch.stack([torch.ones((), device=ok.device, dtype=torch.float64), ok.double().sum() / n,
                         kept.double().sum() / n, r.double().sum() / n])
    return sums


def optimizer_stats(sums):
    it, acc, kept, reads = (float(v) for v in sums.cpu())
    k = max(it, 1.0)
    return {"accepted": acc / k, "pairs_written": kept / k, "pairs_read": reads / k, "iterations": int(it)}


def kernel_bytes(prec, recompute=False, opt_stats=None):
    """Algorithmic HBM bytes per configuration of each kernel (stored tensors, q, FP32 scalars); the
    optimiser's from the measured update statistics when given."""
    b = tensor_bytes(prec)
    L = 0.0 if recompute else b["link_poses"]
    n = T * 7
    k5_per_traj = optimizer_traj_bytes(b["joint_grad"] / 7, n, opt_stats)
    return {
        "fk": 28 + L + b["sphere_pos"] + 4,
        "sphere_cost": b["sphere_pos"] + b["sphere_dist"] + b["sphere_grad"] + 4,
        "reduce": b["sphere_dist"] + 8 + 28,
        "adjoint": b["sphere_grad"] + L + 28 + b["joint_grad"],
        "optimizer": k5_per_traj / (T * N_LS),
    }


def dense_flops_per_cfg():
    """Sphere-cost work without culling: every sphere against every cuboid, every pair once."""
    return N_SPHERES * N_CUBOIDS * FLOPS_PER_SPHERE_CUBOID + N_PAIRS * FLOPS_PER_PAIR


def traffic_from_profile(kernel_src_hash, formats):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernels and
    the same format assignment."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    same = rec.get("kernels_sha256") == kernel_src_hash and rec.get("formats") == formats
    return rec if same else None


def workload_traffic(name, formats, kernel):
    """HBM bytes per launch of `kernel` in another benchmark mode (`swept_k4`, `ik`), measured with
    rocprofv3 counters on the current kernels and the same format assignment, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernels_sha256") != kernels_hash():
        return None
    w = rec.get("workloads", {}).get(name)
    if not w or w.get("formats") != json.loads(json.dumps(formats)):
        return None
    return w.get("bytes_per_launch", {}).get(kernel)


def seed_traffic(kernel, problems):
    """HBM bytes per launch of the seeding network's `kernel` at `problems` problems, measured with
    rocprofv3 counters on the current seeding kernels, else None."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    except Exception:
        return None
    w = rec.get("workloads", {}).get("seed_infer")
    if not w or w.get("problems") != problems:
        return None
    h = hashlib.sha256()
    for f in ("seednet.hip", "seednet.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2310_07854_amd", "csrc", f), "rb").read())
    return w.get("bytes_per_launch", {}).get(kernel) if w.get("seednet_sha256") == h.hexdigest() else None


def kernels_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "codec.hpp", "layout.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2310_07854_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def culled_work(ctx, opt, prec):
    """Sphere-cuboid tests of one sphere-cost launch of the timed loop (its last one), from the
    sphere positions that launch read and the culling grid it used: `needed` counts, per
    configuration and sphere, the cuboids marked in the sphere's voxel (the tests the exact culling
    leaves); `issued` counts lane slots the kernel spends (each lane tests the union over
    CULL_SPHERES spheres of its candidates, a wavefront as often as its busiest lane)."""
    import torch

    from paper_2310_07854_amd.context import dequantize

    shape = opt.shape
    B = shape.B
    fmt = prec.get("sphere_pos", "f32")
    fmt, k = (fmt, 0) if isinstance(fmt, str) else fmt
    codes = ctx.ws_export("sphere_pos", opt.ws, shape)
    pos = dequantize(codes, fmt, B * N_SPHERES * 3, k).view(B, N_SPHERES, 3).cpu().numpy()
    cfg_per_world = B // N_WORLDS
    n_pad = (N_SPHERES + 15) // 16 * 16
    n_q = n_pad // CULL_SPHERES
    Bp = (B + 63) // 64 * 64
    cand = np.zeros((Bp, n_pad), dtype=np.uint64)   # candidate masks [cfg, sphere], padded
    for w in range(N_WORLDS):
        info, mask = ctx.culling_grid(w)
        sl = slice(w * cfg_per_world, (w + 1) * cfg_per_world)
        if mask is None:
            cand[sl, :N_SPHERES] = np.uint64(2 ** 64 - 1) if N_CUBOIDS >= 64 else np.uint64((1 << N_CUBOIDS) - 1)
            continue
        m64 = mask[:, 0].astype(np.uint64)
        if mask.shape[1] > 1:
            m64 |= mask[:, 1].astype(np.uint64) << np.uint64(32)
        n = info["n"]
        f = (pos[sl] - np.array(info["origin"], dtype=np.float32)) * np.float32(info["inv_cell"])
        inside = np.all((f >= 0) & (f < np.float32(n)), axis=-1)
        v = np.floor(np.where(inside[..., None], f, 0)).astype(np.int64)
        cand[sl, :N_SPHERES] = np.where(inside, m64[(v[..., 2] * n + v[..., 1]) * n + v[..., 0]], np.uint64(0))
    needed = int(np.bitwise_count(cand).sum())
    lists = np.bitwise_or.reduce(cand.reshape(-1, 64, n_q, CULL_SPHERES), axis=3)  # [wave, lane, list]
    issued = int(np.bitwise_count(lists).max(axis=1).sum()) * CULL_SPHERES * 64
    return {"needed_tests_per_cfg": needed / B, "issued_lane_tests_per_cfg": issued / B}


CULL_SPHERES = 8  # spheres per candidate list of the sphere-cost kernel
SWEPT_SPHERES, SWEPT_SAMPLES = 4, 2  # the swept kernel's candidate lists: 4 spheres x 2 samples


def swept_culled_work(ctx, opt, prec, k):
    """Sample-cuboid tests of one swept launch of the timed loop (its last one), counted like
    culled_work: `needed` sums, over segments, spheres and the k sample points, the cuboids marked in
    the point's voxel; `issued` counts the lane slots the kernel spends (each lane walks one list per
    4 spheres and chunk of 2 samples, the union of those 8 points' marks, testing all 8 points per
    entry; a wavefront of 64 segment lanes walks as often as its busiest lane).  Sample points are
    recomputed from the stored positions in FP32."""
    from paper_2310_07854_amd.context import dequantize

    shape = opt.shape
    B = shape.B
    fmt = prec.get("sphere_pos", "f32")
    fmt, kx = (fmt, 0) if isinstance(fmt, str) else fmt
    codes = ctx.ws_export("sphere_pos", opt.ws, shape)
    pos = dequantize(codes, fmt, B * N_SPHERES * 3, kx).view(B, N_SPHERES, 3).cpu().numpy()
    n_pad = (N_SPHERES + 15) // 16 * 16
    seg = (np.arange(B) % T) != T - 1
    seg[-1] = False
    p0 = pos
    dp = np.zeros_like(pos)
    dp[:-1] = pos[1:] - pos[:-1]
    needed = 0
    issued = 0
    n_waves = (B + 62) // 63
    lane_a = (63 * np.arange(n_waves)[:, None] - 1 + np.arange(64)[None, :])          # segment start per lane
    lane_ok = (lane_a >= 0) & (lane_a < B)
    lane_a = np.clip(lane_a, 0, B - 1)
    cfg_per_world = B // N_WORLDS
    grids = [ctx.culling_grid(w) for w in range(N_WORLDS)]
    n_lists = n_pad // SWEPT_SPHERES
    for j0 in range(1, k + 1, SWEPT_SAMPLES):
        chunk = range(j0, min(k, j0 + SWEPT_SAMPLES - 1) + 1)
        union = np.zeros((B, n_lists), dtype=np.uint64)
        for j in chunk:
            u = np.float32(j) / np.float32(k + 1)
            pts = (p0 + u * dp).astype(np.float32)
            cand = np.zeros((B, n_pad), dtype=np.uint64)
            for w in range(N_WORLDS):
                info, mask = grids[w]
                sl = slice(w * cfg_per_world, (w + 1) * cfg_per_world)
                if mask is None:
                    cand[sl, :N_SPHERES] = np.uint64((1 << N_CUBOIDS) - 1) if N_CUBOIDS < 64 else np.uint64(2 ** 64 - 1)
                    continue
                m64 = mask[:, 0].astype(np.uint64)
                if mask.shape[1] > 1:
                    m64 |= mask[:, 1].astype(np.uint64) << np.uint64(32)
                n = info["n"]
                f = (pts[sl] - np.array(info["origin"], dtype=np.float32)) * np.float32(info["inv_cell"])
                inside = np.all((f >= 0) & (f < np.float32(n)), axis=-1)
                v = np.floor(np.where(inside[..., None], f, 0)).astype(np.int64)
                cand[sl, :N_SPHERES] = np.where(inside, m64[(v[..., 2] * n + v[..., 1]) * n + v[..., 0]], np.uint64(0))
            cand[~seg] = 0
            needed += int(np.bitwise_count(cand).sum())
            union |= np.bitwise_or.reduce(cand.reshape(B, n_lists, SWEPT_SPHERES), axis=2)
        per_lane = np.bitwise_count(union).astype(np.int64)[lane_a] * lane_ok[..., None]  # [wave, lane, list]
        issued += int(per_lane.max(axis=1).sum()) * SWEPT_SPHERES * len(chunk) * 64
    return {"needed_tests_per_cfg": needed / B, "issued_lane_tests_per_cfg": issued / B}


def calibrate_scales(torch, ctx, x0):
    """amax of each stored tensor on the FP32 path over the run's initial trajectories."""
    from paper_2310_07854_amd import Shape

    ctx.set_precision({})
    shape = Shape(N_WORLDS, TPW, T, 1)
    q = x0.reshape(-1, 7).contiguous()
    _, ws = ctx.cost_fwd(q, shape)
    ctx.cost_bwd(q, ws, want_grad=False)
    names = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")
    if ctx.cost_params.get("swept_steps", 0) > 0:
        names += ("swept_grad",)
    return {t: float(ctx.ws_export(t, ws, shape).view(torch.float32).abs().max()) for t in names}


def with_scales(formats, amax, reach):
    """(format, k) per tensor: link poses and sphere positions from the robot's reach, the others
    from their FP32 magnitude on the calibration pass (one binade of headroom for FP16/BF16, which
    overflow to Inf); |k| <= 16, FP32 k = 0."""
    from paper_2310_07854_amd.search import spec

    return spec({t: fmt_of(formats, t) for t in TENSOR_NAMES if t in amax or t in formats}, amax, reach)


def fwd_bwd_timing(torch, ctx, x0, prec, recompute=False, warmup=20, runs=200):
    """The cost and gradient path alone (k_fk .. k_adjoint, FP32 joint gradients out) on the
    196,608 trajectory points: HIP events around each run on the stream the kernels use; median,
    10th and 90th percentile of the run durations."""
    from paper_2310_07854_amd import Shape

    ctx.set_precision(prec, recompute_poses=recompute)
    shape = Shape(N_WORLDS, TPW, T, 1)
    q = x0.reshape(-1, 7).contiguous()
    ws = ctx.new_workspace(shape)
    cost = torch.empty(shape.n_tc, dtype=torch.float64, device=q.device)
    grad = torch.empty_like(q)

    def once():
        ctx.cost_fwd(q, shape, ws=ws, cost_traj=cost)
        ctx.cost_bwd(q, ws, grad_q=grad)

    for _ in range(warmup):
        once()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        once()
        b.record()
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    med, p10, p90 = np.median(ms), np.percentile(ms, 10), np.percentile(ms, 90)
    return {"evals_per_s": shape.B / (med * 1e-3), "median_ms": float(med), "p10_ms": float(p10),
            "p90_ms": float(p90), "runs": runs, "recompute_poses": recompute}


def copy_bandwidth(torch, mib=1024, runs=20):
    """Achievable HBM bandwidth on this machine: a plain 1 GiB device-to-device copy (read + write
    bytes over the median duration)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    med = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    del a, b
    return 2.0 * mib * (1 << 20) / (med * 1e-3) / 1e9


def cold_kernels(torch, ctx, opt_cls, x0, prec, recompute=False, reps=10, flush_mib=1024):
    """Per-kernel durations with the caches emptied before each measured launch: a 1 GiB buffer is
    written first, so the kernel finds none of its inputs in the 4 MB L2 of each XCD or the 256 MB
    Infinity Cache and reads them from HBM.  Each kernel is reached through the call that launches it
    first: the forward pass from stage 1 (k_fk), 2 (k_sphere_cost) and 3 (k_reduce), the backward
    pass (k_adjoint) and the optimiser update after an evaluated iteration (k_optimizer).  HIP events
    around each launch; the mean over `reps`, cold and warm (the same call without the flush)."""
    ctx.set_precision(prec, recompute_poses=recompute)
    opt = opt_cls(ctx, N_WORLDS, TPW, T, n_ls=N_LS, m=HIST_M)
    opt.init(x0)
    for _ in range(3):
        opt.step()
    flush = torch.empty(flush_mib << 18, dtype=torch.float32, device="cuda:0")
    q, shape, ws, cost = opt.q_cand, opt.shape, opt.ws, opt.cost_cand
    calls = {
        "fk": (None, lambda: ctx.cost_fwd(q, shape, ws=ws, cost_traj=cost, first=1)),
        "sphere_cost": (None, lambda: ctx.cost_fwd(q, shape, ws=ws, cost_traj=cost, first=2)),
        "reduce": (None, lambda: ctx.cost_fwd(q, shape, ws=ws, cost_traj=cost, first=3)),
        "adjoint": (None, lambda: ctx.cost_bwd(q, ws, want_grad=False)),
        "optimizer": (opt.evaluate, opt.update),
    }
    out = {}
    for name, (before, call) in calls.items():
        res = {}
        for mode in ("cold", "warm"):
            total = 0.0
            for i in range(reps):
                if before is not None:
                    before()
                if mode == "cold":
                    flush.fill_(float(i))
                ctx.profile_enable(True)
                call()
                ms, n = ctx.profile_read()[name]
                ctx.profile_enable(False)
                total += ms / max(n, 1)
            res[mode + "_us"] = total / reps * 1e3
        out[name] = res
    del flush, opt
    return out


def run_variant(torch, ctx, opt_cls, x0, prec, steps, warmup, want_opt=False, recompute=False):
    """`warmup` untimed iterations, then `steps` timed ones with nothing but the iteration's own
    launches in the stream (the step time), then `steps` more with HIP events recorded around every
    launch on the library's stream (the per-kernel durations: the events add their own cost to the
    stream, about 15% of a step here, so they stay out of the step time)."""
    ctx.set_precision(prec, recompute_poses=recompute)
    opt = opt_cls(ctx, N_WORLDS, TPW, T, n_ls=N_LS, m=HIST_M)
    opt.init(x0)
    for _ in range(warmup):
        opt.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        opt.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the per-kernel window; the optimiser's update statistics are gathered over the same
    # iterations by small torch kernels between them (outside the events around each launch)
    sums = torch.zeros(4, dtype=torch.float64, device=x0.device)
    ctx.profile_enable(True)
    for _ in range(steps):
        prev = opt.hist_len.clone()
        opt.step()
        optimizer_stats_add(torch, opt, prev, sums)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    cost = float(opt.cost.sum())
    prof_stats = optimizer_stats(sums)
    return (t1 - t0), prof, cost, (opt if want_opt else None), prof_stats


def run_partitioned(torch, ctx, x0, prec, steps, warmup, parts, recompute=False):
    """The same iterations with the batch split by worlds over `parts` contexts and streams
    (PartitionedOptimizer: identical results, the kernels of one partition filling the GPU while
    another's drain).  Returns (seconds for `steps` timed iterations, total final cost)."""
    from paper_2310_07854_amd import PartitionedOptimizer

    ctx.set_precision(prec, recompute_poses=recompute)
    opt = PartitionedOptimizer(ctx, N_WORLDS, TPW, T, n_ls=N_LS, m=HIST_M, parts=parts)
    opt.init(x0)
    for _ in range(warmup):
        opt.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        opt.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cost = float(opt.cost.sum())
    opt.close()
    return t1 - t0, cost


def stored_tensor_report(torch, ctx, opt, prec):
    """After the timed steps of one assignment: per stored tensor the census of its codes (at the
    format's largest finite magnitude -- saturated --, and Inf/NaN), and the fraction of spheres
    with a nonzero distance and a nonzero gradient (how dense D and G are on this workload)."""
    from paper_2310_07854_amd.context import dequantize

    shape = opt.shape
    census = {}
    for t in ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad"):
        a, b = ctx.census(t, opt.ws, shape)
        census[t] = {"largest_magnitude": a, "inf_nan": b, "of": shape.B * ctx.tensor_count(t)}
    act = {}
    for t in ("sphere_dist", "sphere_grad"):
        fmt, k = prec.get(t, ("f32", 0)) if not isinstance(prec.get(t, "f32"), str) else (prec[t], 0)
        n = shape.B * ctx.tensor_count(t)
        v = dequantize(ctx.ws_export(t, opt.ws, shape), fmt, n, k).view(shape.B, N_SPHERES, -1)
        act[t] = float((v != 0).any(dim=2).float().mean())
    return census, act


def _oracle_trajectories(prec_kw, start, count):
    """One optimisation iteration of the FP64 oracle (quantisation emulated) over trajectories
    start .. start + count - 1 of the benchmark batch, each in its world; returns the seconds."""
    from threadpoolctl import threadpool_limits

    from oracle import cost as OC
    from oracle import optimizer as OO
    from synthetic import Worlds, make_robot, make_trajectories, make_worlds

    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    traj = make_trajectories(N_WORLDS, TPW, T).reshape(-1, T, 7)
    oprec = OC.Precision(**prec_kw)
    idx = np.arange(start, start + count)
    sub = Worlds(pose=worlds.pose[idx // TPW], half_ext=worlds.half_ext[idx // TPW])
    x = traj[idx]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        out = OC.fwd_bwd(robot, sub, x.reshape(-1, 7), 1, T, N_LS, prec=oprec)
        for i in range(count):
            st = OO.TrajState(x=x[i].reshape(-1), g=np.zeros(T * 7), d=-np.ones(T * 7) * 1e-3,
                              cost=float(out["cost_traj"][i]) + 1.0)
            OO.step(st, out["cost_traj"][i:i + 1], out["grad_q"].reshape(count, 1, -1)[i], T, HIST_M)
        return time.perf_counter() - t0


def _host_cpu():
    """(usable cores, CPU model) of this host."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(prec, budget_s=12.0, all_core_s=10.0, max_workers=16):
    """The FP64 oracle (quantisation emulated at the same five tensors) timed on the host for one
    optimisation iteration of a sample of whole trajectories: single-threaded, and on all usable
    cores (up to max_workers processes, one thread each, started fresh: no GPU state is inherited)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    prec_kw = {t: ((v, 0) if isinstance(v, str) else tuple(v)) for t, v in prec.items()}
    n, dt = timed_sample(lambda k: _oracle_trajectories(prec_kw, 0, k), N_WORLDS * TPW, budget_s)
    single = n * T * N_LS / dt
    cores, model = _host_cpu()
    workers = max(1, min(cores, max_workers))
    per_traj = dt / n
    chunk = max(4, int(0.5 / per_traj))  # about half a second per task
    n_all = int(min(N_WORLDS * TPW, all_core_s * workers / per_traj)) // chunk * chunk
    n_all = max(n_all, chunk)
    tasks = [(prec_kw, s0, chunk) for s0 in range(0, n_all, chunk)]
    # a worker that dies raises BrokenProcessPool here instead of leaving the map waiting
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        list(pool.map(_oracle_trajectories, *zip(*[(prec_kw, 0, 2)] * workers), timeout=300))  # imports
        t0 = time.perf_counter()
        list(pool.map(_oracle_trajectories, *zip(*tasks), timeout=600))
        wall = time.perf_counter() - t0
    return {"value": single, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} trajectories x {T} timesteps = {n * T} configurations, one iteration, "
                      f"{dt:.1f} s single-threaded",
            "all_cores": {"value": n_all * T * N_LS / wall, "unit": "evals/s", "cores": workers,
                          "host_cores": cores, "cpu_model": model,
                          "sample": f"{n_all} trajectories in {len(tasks)} tasks of {chunk}, {wall:.1f} s on "
                                    f"{workers} processes"}}


def error_vs_fp64(prec, gpu):
    """Error of the GPU's cost and gradient against the unquantised FP64 oracle on sampled
    trajectories of the benchmark batch (at its initial trajectories), with the oracle's first-order
    error budget of the assignment: cost error relative to |cost| (max, median) and to the budget;
    gradient error relative in L2 over the sample and, on configurations away from the kinks (where
    a rounding of the sphere centres cannot switch a branch of the cost), to the budget (max, 99th
    percentile)."""
    from oracle import budget as BG
    from oracle import cost as OC
    from synthetic import Worlds, make_robot, make_trajectories, make_worlds

    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    traj = make_trajectories(N_WORLDS, TPW, T).reshape(-1, T, 7)
    tr = gpu["traj"]
    sub = Worlds(pose=worlds.pose[tr // TPW], half_ext=worlds.half_ext[tr // TPW])
    oprec = OC.Precision(**{t: ((v, 0) if isinstance(v, str) else tuple(v)) for t, v in prec.items()})
    t0 = time.perf_counter()
    bud = BG.error_budget(robot, sub, traj[tr].reshape(-1, 7), 1, T, 1, oprec)
    ref = bud["ref"]
    dc = np.abs(gpu["cost"] - ref["cost_traj"])
    dg = np.abs(gpu["grad"] - ref["J"])
    ok = BG.smooth_configurations(robot, ref, sub.pose, sub.half_ext, BG.position_gap(oprec, ref))
    gr = (dg / bud["grad"])[ok]
    return {"trajectories": int(len(tr)), "configurations": int(len(tr) * T),
            "cost_max_rel": float(np.max(dc / np.abs(ref["cost_traj"]))),
            "cost_med_rel": float(np.median(dc / np.abs(ref["cost_traj"]))),
            "grad_rel_l2": float(np.linalg.norm(dg) / np.linalg.norm(ref["J"])),
            "budget_ratio": {"cost_max": float(np.max(dc / bud["cost"])),
                             "grad_max": float(gr.max()) if gr.size else None,
                             "grad_p99": float(np.percentile(gr, 99)) if gr.size else None,
                             "grad_configurations": int(ok.sum())},
            "oracle_seconds": time.perf_counter() - t0}


def timed_sample(one, n_max, budget_s):
    """(n, seconds) of one(n) single-threaded, with n sized from the slope between two small samples
    (a call has a fixed cost) so that it takes about budget_s."""
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        t8, t32 = one(8), one(32)
        per = max((t32 - t8) / 24.0, t32 / 64.0, 1e-6)
        n = int(max(8, min(n_max, budget_s / per)))
        dt = one(n)
        if dt < 0.5 * budget_s and n < n_max:  # the small samples overstated the per-item time
            n = int(min(n_max, n * budget_s / dt))
            dt = one(n)
        return n, dt


def swept_cpu_baseline(prec, k, budget_s=12.0):
    """The oracle with the swept term (k samples per segment, quantisation emulated at the six
    stored tensors) for one optimisation iteration of a sample of whole trajectories."""
    from oracle import cost as OC
    from oracle import optimizer as OO
    from synthetic import Worlds, make_robot, make_trajectories, make_worlds

    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    traj = make_trajectories(N_WORLDS, TPW, T)
    oprec = OC.Precision(**{t: ((v, 0) if isinstance(v, str) else tuple(v)) for t, v in prec.items()})
    params = OC.CostParams(swept_steps=k, w_swept=100.0)

    def one(n_traj):
        x = traj.reshape(-1, T, 7)[:n_traj]
        sub = Worlds(pose=worlds.pose[np.arange(n_traj) // TPW], half_ext=worlds.half_ext[np.arange(n_traj) // TPW])
        t0 = time.perf_counter()
        out = OC.fwd_bwd(robot, sub, x.reshape(-1, 7), 1, T, N_LS, prec=oprec, params=params)
        for i in range(n_traj):
            st = OO.TrajState(x=x[i].reshape(-1), g=np.zeros(T * 7), d=-np.ones(T * 7) * 1e-3,
                              cost=float(out["cost_traj"][i]) + 1.0)
            OO.step(st, out["cost_traj"][i:i + 1], out["grad_q"].reshape(n_traj, 1, -1)[i], T, HIST_M)
        return time.perf_counter() - t0

    n, dt = timed_sample(one, N_WORLDS * TPW, budget_s)
    return {"value": n * T / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} trajectories x {T} timesteps = {n * T} configurations with the swept term "
                      f"(k = {k}), one iteration, {dt:.1f} s single-threaded"}


def ik_cpu_baseline(prec, budget_s=12.0):
    """The oracle on the inverse-kinematics workload (pose, collision, self and bound costs, one
    configuration per trajectory, free rows) for one iteration of a sample of seeds against problem 0,
    with the goal computed by the oracle's own kinematics."""
    from oracle import cost as OC
    from oracle import optimizer as OO
    from oracle.kinematics import forward_kinematics
    from synthetic import Worlds, make_configs, make_robot, make_worlds

    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    qg = make_configs(N_WORLDS, seed=77)
    goals = forward_kinematics(robot.fixed_tf, qg[:1])[:, 8, :3, :]
    q = make_configs(N_WORLDS * IK_SEEDS, seed=78)  # the benchmark's seeds, all posed against problem 0
    oprec = OC.Precision(**{t: ((v, 0) if isinstance(v, str) else tuple(v)) for t, v in prec.items()})
    sub = Worlds(pose=worlds.pose[:1], half_ext=worlds.half_ext[:1])

    def one(n):
        t0 = time.perf_counter()
        out = OC.fwd_bwd(robot, sub, q[:n], n, 1, 1, prec=oprec, goals=goals)
        for i in range(n):
            st = OO.TrajState(x=q[i].copy(), g=np.zeros(7), d=-np.ones(7) * 1e-3, cost=float(out["cost_traj"][i]) + 1.0)
            OO.step(st, out["cost_traj"][i:i + 1], out["grad_q"][i:i + 1], 1, HIST_M, pin=False)
        return time.perf_counter() - t0

    n, dt = timed_sample(one, len(q), budget_s)
    return {"value": n / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} seeds against one problem (one configuration each), one iteration, {dt:.1f} s "
                      f"single-threaded"}


def seed_cpu_baseline(budget_s=12.0):
    """The oracle's seeding network inference (occupancy, features, three GELU layers, output layer
    and trajectory construction, FP64 with BF16 operands emulated) on a sample of problems."""
    from oracle import seeding as SD
    from synthetic import make_seed_problems, make_seednet_params

    params = make_seednet_params()
    pr = make_seed_problems(8192, 16, split=7)

    def one(n):
        t0 = time.perf_counter()
        occ = SD.occupancy(pr.worlds.pose[:n], pr.worlds.half_ext[:n])
        x = SD.features(pr.start[:n], pr.goal[:n], occ)
        y, _ = SD.forward(params, x, emulate=True)
        SD.seeds(y, pr.start[:n], pr.goal[:n])
        return time.perf_counter() - t0

    n, dt = timed_sample(one, 8192, budget_s)
    return {"value": n / dt, "unit": "problems/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} problems of 16 cuboids, inference, {dt:.1f} s single-threaded"}


class InfeasibleEnvironment(RuntimeError):
    pass


def seeding_study(args):
    """The learned seeder end to end on synthetic problems (one GPU), per environment: an environment
    is a base world of 16 cuboids whose problems jitter every cuboid centre by up to 5 cm and draw
    start and goal uniformly.  Keep problems with collision-free endpoints, solve each from 32 linear
    initial trajectories, train the network on the 8 lowest-cost collision-free solutions, then
    compare network, linear and random seeds (8 each) on held-out problems of the same environment
    by the first optimiser iteration at which a seed is collision-free.  The arm is the benchmark's
    without self pairs (its random sphere model overlaps itself in nearly every configuration)."""
    import dataclasses

    import torch

    from paper_2310_07854_amd import Context, seed_pipeline as SP, seeding as SG
    from synthetic import make_robot, make_seed_family, make_seed_inits, make_seednet_params

    K, T, S_TRAIN, S_EVAL = 16, 32, 32, 8
    dev = "cuda:0"
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=dev)
    log = lambda msg: print(f"# seeder: {msg}", file=sys.stderr, flush=True)
    robot = make_robot(N_SPHERES, N_PAIRS)
    robot = dataclasses.replace(robot, pairs=robot.pairs[:0])
    ctx = Context(0)
    ctx.set_robot(robot)
    ctx.set_precision({})
    ctx.set_culling(False)
    t_start = time.perf_counter()

    def feasible(family, n_want, split0):
        keep = {"pose": [], "half": [], "start": [], "goal": []}
        have, drawn, split = 0, 0, split0
        while have < n_want:
            pr = make_seed_family(16384, K, family, split=split)
            ctx.set_worlds(pr.worlds.pose, pr.worlds.half_ext)
            ok = SP.endpoints_free(ctx, d(pr.start), d(pr.goal)).cpu().numpy()
            for key, arr in (("pose", pr.worlds.pose), ("half", pr.worlds.half_ext), ("start", pr.start),
                             ("goal", pr.goal)):
                keep[key].append(arr[ok])
            have += int(ok.sum())
            drawn += 16384
            split += 1
            log(f"environment {family}: {have} of {n_want} feasible problems from {drawn} drawn")
            if drawn >= 64 * n_want:
                raise InfeasibleEnvironment(f"environment {family}: too few problems with collision-free endpoints")
        return {k: np.concatenate(v)[:n_want] for k, v in keep.items()}, drawn

    def dataset(family):
        p, drawn = feasible(family, args.seed_problems, 100)
        chunks = []
        for c0 in range(0, args.seed_problems, 4096):
            sl = slice(c0, min(c0 + 4096, args.seed_problems))
            ctx.set_worlds(p["pose"][sl], p["half"][sl])
            st, gl = d(p["start"][sl]), d(p["goal"][sl])
            if args.seed_train_inits == "linear":
                x0 = d(make_seed_inits(p["start"][sl], p["goal"][sl], S_TRAIN, T, "linear", split=1000 + c0))
            else:
                x0 = torch.cat([d(make_seed_inits(p["start"][sl], p["goal"][sl], S_TRAIN // 2, T, "linear",
                                                  split=1000 + c0)),
                                d(make_seed_inits(p["start"][sl], p["goal"][sl], S_TRAIN // 2, T, "random",
                                                  split=1000 + c0))], dim=1).contiguous()
            sol = SP.solve(ctx, x0, iters=args.seed_solve_iters, check_every=args.seed_solve_iters)
            tgt, valid = SP.select_targets(sol, st, gl, diverse=args.seed_targets == "diverse")
            occ = SG.occupancy(d(p["pose"][sl]), d(p["half"][sl]))
            chunks.append({"start": st, "goal": gl, "occ": occ, "targets": tgt, "valid": valid})
            log(f"environment {family}: solved {sl.stop} of {args.seed_problems}")
        data = {k: torch.cat([c[k] for c in chunks]) for k in chunks[0]}
        keep = data["valid"].sum(dim=1) > 0
        return {k: v[keep] for k, v in data.items()}, drawn

    # environments are drawn in turn; one whose base world leaves almost no start and goal
    # collision-free (fewer than 1 in 64 draws) is skipped and recorded
    envs, skipped, family = [], [], -1
    while len(envs) < args.seed_envs:
        family += 1
        if family >= 4 * args.seed_envs:
            raise RuntimeError("too many environments without collision-free problems")
        t0 = time.perf_counter()
        try:
            data, drawn = dataset(family)
        except InfeasibleEnvironment as e:
            log(str(e) + ": skipped")
            skipped.append(family)
            continue
        t_data = time.perf_counter() - t0
        n_data = int(data["start"].shape[0])
        net = SG.SeedNet(make_seednet_params())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = SP.train(net, data, steps=args.seed_train_steps, batch=256, lr=1e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        log(f"environment {family}: trained {args.seed_train_steps} steps in {t_train:.1f} s, "
            f"loss {np.mean(losses[:20]):.4f} -> {np.mean(losses[-20:]):.4f}")
        ev, _ = feasible(family, args.seed_eval, 1)
        ctx.set_worlds(ev["pose"], ev["half"])
        st, gl = d(ev["start"]), d(ev["goal"])
        occ = SG.occupancy(d(ev["pose"]), d(ev["half"]))
        inits = {"network": net.seeds(st, gl, occ),
                 "linear": d(make_seed_inits(ev["start"], ev["goal"], S_EVAL, T, "linear", split=1)),
                 "random": d(make_seed_inits(ev["start"], ev["goal"], S_EVAL, T, "random", split=1))}
        # the network's first four slots with four of the linear fallback seeds (those with a random
        # bend; the straight line is what the network's slots sit close to)
        inits["network+linear"] = torch.cat([inits["network"][:, :S_EVAL // 2], inits["linear"][:, 1:1 + S_EVAL // 2]],
                                            dim=1)
        # ... or with four random-via-point seeds, the family that reaches the hard problems soonest
        inits["network+random"] = torch.cat([inits["network"][:, :S_EVAL // 2], inits["random"][:, :S_EVAL // 2]],
                                            dim=1)
        # each network slot bent through a random via point: the slot plus the random seed's
        # deviation from the straight line (zero at the endpoints), so the learned route keeps the
        # random seeds' spread; alone, and its first four with the network's first four
        straight = inits["linear"][:, :1]
        inits["network bent"] = inits["network"] + (inits["random"] - straight)
        inits["network+bent"] = torch.cat([inits["network"][:, :S_EVAL // 2],
                                           inits["network bent"][:, :S_EVAL // 2]], dim=1)
        firsts, final_cost = {}, {}
        for kind, x0 in inits.items():
            sol = SP.solve(ctx, x0.contiguous(), iters=args.seed_eval_iters, check_every=1)
            firsts[kind] = sol["first_free"].cpu().numpy()
            masked = torch.where(sol["free"], sol["cost"], torch.full_like(sol["cost"], float("inf")))
            best = masked.min(dim=1).values.cpu().numpy()
            final_cost[kind] = float(np.median(best[np.isfinite(best)])) if np.isfinite(best).any() else None
            log(f"environment {family}, {kind} seeds: collision-free by iteration 0/1/5/20: "
                + " ".join(f"{np.mean((firsts[kind] >= 0) & (firsts[kind] <= i)):.3f}" for i in (0, 1, 5, 20)))
        envs.append({"environment": family, "problems_drawn": drawn, "problems_with_targets": n_data,
                     "targets_per_problem": float(data["valid"].sum().item()) / max(n_data, 1),
                     "data_s": t_data, "train_s": t_train, "loss_first": float(np.mean(losses[:20])),
                     "loss_last": float(np.mean(losses[-20:])), "firsts": firsts,
                     "median_final_cost": final_cost})

    # inference throughput of the network (features -> 8 seeds) at a large batch
    nb = 16384
    xb = SG.features(d(np.zeros((nb, 7))), d(np.ones((nb, 7))), torch.zeros(nb, 512, device=dev))
    for _ in range(3):
        net.forward(xb)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        net.forward(xb)
        b.record()
    torch.cuda.synchronize()
    fwd_ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    flops = 2.0 * nb * (544 * 256 + 256 * 256 * 2 + 256 * 1792)
    ctx.close()

    # pooled over environments: collision-free rate by iteration, and the iterations each kind of
    # seed needs to reach the rate that all three reach
    kinds = ("network", "linear", "random", "network+linear", "network+random", "network bent", "network+bent")
    pooled = {k: np.concatenate([e["firsts"][k] for e in envs]) for k in kinds}
    marks = sorted({0, 1, 2, 3, 5, 10, 20, args.seed_eval_iters})
    curves = {k: {str(i): float(np.mean((ff >= 0) & (ff <= i))) for i in marks} for k, ff in pooled.items()}
    rate = min(float(np.mean(ff >= 0)) for ff in pooled.values())
    need = {}
    for k, ff in pooled.items():
        srt = np.sort(np.where(ff >= 0, ff, 10 ** 9))
        need[k] = int(srt[int(np.ceil(rate * len(ff))) - 1]) if rate > 0 else None
    for e in envs:
        e.pop("firsts")
    line = {"metric": "learned seeding: collision-free rate by optimiser iteration (network vs linear vs random "
                      "seeds, 8 each; 4 network + 4 linear; 4 network + 4 random; network slots bent through "
                      "random via points, 8, and 4 network + 4 of those)",
            "data": "synthetic", "n_gpus": 1, "dtype": "bf16 GEMM operands, f32 accumulate",
            "config": {"workload": f"7-joint arm, 60 spheres, no self pairs; {args.seed_envs} environments of {K} "
                                   f"cuboids (centres jittered 5 cm per problem); T = {T}; "
                                   f"{args.seed_problems} training problems per environment solved from "
                                   f"{S_TRAIN} {args.seed_train_inits} seeds x {args.seed_solve_iters} iterations, "
                                   f"{args.seed_targets} targets; "
                                   f"{args.seed_eval} held-out problems per environment",
                       "train_steps": args.seed_train_steps, "batch": 256, "lr": 1e-3},
            "curves": curves, "common_rate": rate, "iterations_to_common_rate": need,
            "environments": envs, "environments_skipped": skipped,
            "network_forward": {"batch": nb, "ms": fwd_ms, "TFLOPs": flops / (fwd_ms * 1e-3) / 1e12,
                                "peak_bf16_TFLOPs": 2500.0},
            "total_s": time.perf_counter() - t_start}
    print(json.dumps(line), flush=True)


SEED_FLOPS_PER_PROBLEM = 2 * (544 * 256 + 2 * 256 * 256 + 256 * 1792)
# algorithmic HBM bytes per problem of each inference kernel (weights, read once per launch, excluded)
SEED_BYTES = {"k_features": 56 + 2048 + 1088, "gemm1": 1088 + 512, "gemm2": 512 + 512, "gemm3": 512 + 512,
              "head": 512 + 56 + 7168}


def seed_inference(args):
    """Throughput of the seeding network's inference (features -> 3 BF16 MFMA GEMMs with GELU ->
    output GEMM fused with the trajectory construction -> 8 seed trajectories) on a batch of problems
    resident in HBM; weights at their initial values (the work does not depend on them)."""
    import torch

    from paper_2310_07854_amd import seeding as SG
    from synthetic import make_seed_problems, make_seednet_params

    nb = args.seed_batch
    dev = "cuda:0"
    pr = make_seed_problems(nb, 16, split=7)
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=dev)
    st, gl = d(pr.start), d(pr.goal)
    occ = SG.occupancy(d(pr.worlds.pose), d(pr.worlds.half_ext))
    net = SG.SeedNet(make_seednet_params())
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        net.seeds(st, gl, occ)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.seeds(st, gl, occ)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # per-kernel durations with events around each launch on the launching stream
    x = SG.features(st, gl, occ)
    ev = {k: [] for k in SEED_BYTES}
    a = x
    reps = 10
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True); e0.record(stream)
        x = SG.features(st, gl, occ)
        e1 = torch.cuda.Event(enable_timing=True); e1.record(stream)
        ev["k_features"].append((e0, e1))
        a, k = x, 544
        for l in (1, 2, 3):
            a_next = torch.empty(nb, 256, dtype=torch.bfloat16, device=dev)
            e0 = torch.cuda.Event(enable_timing=True); e0.record(stream)
            SG.gemm(a, k, 1, net.view(net.w16, f"W{l}"), 256, 1, nb, 256, k, bias=net.view(net.w, f"b{l}"),
                    epilogue=SG.GELU, C16=a_next)
            e1 = torch.cuda.Event(enable_timing=True); e1.record(stream)
            ev[f"gemm{l}"].append((e0, e1))
            a, k = a_next, 256
        e0 = torch.cuda.Event(enable_timing=True); e0.record(stream)
        net.head(a, st, gl)
        e1 = torch.cuda.Event(enable_timing=True); e1.record(stream)
        ev["head"].append((e0, e1))
    torch.cuda.synchronize()
    kern = {}
    for k, lst in ev.items():
        us = float(np.mean([a.elapsed_time(b) for a, b in lst])) * 1e3
        kern[k] = {"us": us, "GBs": SEED_BYTES[k] * nb / (us * 1e-6) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["us"])
    ach = kern[dom]["GBs"]
    line = {"metric": "seeding network inference throughput", "value": nb / (ms * 1e-3), "unit": "problems/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16 operands, f32 accumulate", "data": "synthetic",
            "config": {"workload": f"{nb} problems: 7 + 7 + 512 inputs -> 3 x 256 GELU -> 8 seeds x 32 x 7"},
            "TFLOPs": SEED_FLOPS_PER_PROBLEM * nb / (ms * 1e-3) / 1e12,
            "kernels": kern,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": seed_traffic(dom, nb),
                         "bytes_per_problem": SEED_BYTES[dom]},
            "cpu_baseline": None if args.no_cpu_baseline else seed_cpu_baseline()}
    print(json.dumps(line), flush=True)


def swept_bench(args):
    """One optimiser iteration per step on the 196,608-configuration workload with the swept term
    on (k samples per segment between consecutive timesteps), FP32 and the paper-like assignment
    (the swept gradient X stored like G).  The swept kernel tests every sample against the cuboids
    its world's culling grid marks in the sample's voxel; its algorithmic work is those tests x 35
    FP32 operations (counted from the last launch's positions)."""
    import torch

    from paper_2310_07854_amd import Context, TrajectoryOptimizer
    from synthetic import make_robot, make_trajectories, make_worlds

    k = args.swept
    B = N_WORLDS * TPW * T * N_LS
    ctx = Context(0)
    ctx.set_robot(make_robot(N_SPHERES, N_PAIRS))
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    ctx.set_worlds(worlds.pose, worlds.half_ext)
    ctx.set_cost_params(swept_steps=k, w_swept=100.0)
    x0 = torch.tensor(make_trajectories(N_WORLDS, TPW, T).reshape(N_WORLDS * TPW, T, 7), dtype=torch.float32,
                      device="cuda:0")
    amax = calibrate_scales(torch, ctx, x0)
    out = {}
    for name in ("f32", "paper_like"):
        f = dict(PRECISIONS[name])
        f["swept_grad"] = f.get("sphere_grad", "f32")
        prec = with_scales(f, amax, ctx.reach())
        dt, prof, _, opt, _ = run_variant(torch, ctx, TrajectoryOptimizer, x0, prec, args.steps, args.warmup,
                                       want_opt=name == "paper_like")
        if opt is not None:
            work = swept_culled_work(ctx, opt, prec, k)
            del opt
        kern = {kk: v[0] / max(v[1], 1) * 1e3 for kk, v in prof.items() if v[1]}
        out[name] = {"value": B * args.steps / dt, "ms_per_step": dt / args.steps * 1e3, "kernels_us": kern,
                     "formats": {kk: list(v) for kk, v in prec.items()}}
        print(f"# swept k={k} {name}: {dt / args.steps * 1e3:.3f} ms/step, {B * args.steps / dt / 1e6:.1f} M evals/s, "
              + ", ".join(f"{kk} {v:.1f}us" for kk, v in kern.items()), file=sys.stderr, flush=True)
    ctx.close()
    dense_cfg = (T - 1) / T * N_SPHERES * k * N_CUBOIDS * FLOPS_PER_SPHERE_CUBOID
    flops_cfg = work["needed_tests_per_cfg"] * FLOPS_PER_SPHERE_CUBOID
    sw_us = out["paper_like"]["kernels_us"]["swept"]
    achieved = flops_cfg * B / (sw_us * 1e-6) / 1e12
    line = {"metric": "cost fwd+bwd evals/s with the swept collision term (one optimiser iteration per step)",
            "value": out["paper_like"]["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out["paper_like"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"64 worlds x 64 seeds x 48 timesteps = 196,608 configurations per step; "
                                   f"7-joint arm, 60 spheres, 300 self pairs, 64 oriented cuboids per world; swept "
                                   f"term with {k} samples per segment",
                       "precision": "paper_like", "formats": out["paper_like"]["formats"]},
            "fp32_value": out["f32"]["value"], "variants": out,
            "roofline": {"kernel": "k_swept", "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS, "flops_per_cfg": flops_cfg,
                         "culled_tests_per_cfg": work["needed_tests_per_cfg"],
                         "issued_lane_tests_per_cfg": work["issued_lane_tests_per_cfg"],
                         "dense_equivalent_TFLOPs": dense_cfg * B / (sw_us * 1e-6) / 1e12,
                         "traffic": workload_traffic(f"swept_k{k}", out["paper_like"]["formats"], "k_swept")},
            "cpu_baseline": None if args.no_cpu_baseline else swept_cpu_baseline(
                {kk: tuple(v) for kk, v in out["paper_like"]["formats"].items()}, k)}
    print(json.dumps(line), flush=True)


def batched_workload(torch, steps, warmup):
    """Optimiser iterations per second on the batched workload with a line search: 4 worlds x 32 seeds
    x 32 timesteps x 4 step-scale candidates = 16,384 configurations per iteration, 40 cuboids,
    FP32 and the paper-like assignment (scales calibrated on the batch's initial trajectories)."""
    from paper_2310_07854_amd import Context, Shape, TrajectoryOptimizer
    from synthetic import make_robot, make_trajectories, make_worlds

    W, S, Tn, nls, K = 4, 32, 32, 4, 40
    B = W * S * Tn * nls
    ctx = Context(0)
    ctx.set_robot(make_robot(N_SPHERES, N_PAIRS))
    worlds = make_worlds(W, K)
    ctx.set_worlds(worlds.pose, worlds.half_ext)
    x0 = torch.tensor(make_trajectories(W, S, Tn).reshape(W * S, Tn, 7), dtype=torch.float32, device="cuda:0")
    ctx.set_precision({})
    sh = Shape(W, S, Tn, 1)
    q = x0.reshape(-1, 7).contiguous()
    _, ws = ctx.cost_fwd(q, sh)
    ctx.cost_bwd(q, ws, want_grad=False)
    amax = {t: float(ctx.ws_export(t, ws, sh).view(torch.float32).abs().max()) for t in
            ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")}
    out = {"workload": "4 worlds x 32 seeds x 32 timesteps x 4 line-search candidates = 16,384 configurations "
                       "per iteration; 60 spheres, 300 self pairs, 40 cuboids per world"}
    for name in ("f32", "paper_like"):
        ctx.set_precision(with_scales(PRECISIONS[name], amax, ctx.reach()) if name != "f32" else {})
        opt = TrajectoryOptimizer(ctx, W, S, Tn, n_ls=nls, m=HIST_M)
        opt.init(x0)
        for _ in range(warmup):
            opt.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            opt.step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"iterations_per_s": 1.0 / dt, "ms_per_iteration": dt * 1e3, "evals_per_s": B / dt,
                     "cost_sum": float(opt.cost.sum())}
        del opt
    ctx.close()
    return out


def graph_bench(args):
    """Eager iterations against replays of one captured HIP graph of the iteration, on the batched
    FP32 workload (4 worlds x 32 seeds x 32 timesteps, 4 line-search candidates: 16,384
    configurations per step, 40 cuboids) and on the 196,608-configuration workload (paper-like)."""
    import torch

    from paper_2310_07854_amd import Context, TrajectoryOptimizer
    from synthetic import make_robot, make_trajectories, make_worlds

    out = {}
    cases = {"batched_4096x4_fp32": (4, 32, 32, 4, 40, "f32"),
             "large_196608_paper_like": (N_WORLDS, TPW, T, N_LS, N_CUBOIDS, "paper_like")}
    for name, (W, S, Tn, nls, K, prec) in cases.items():
        ctx = Context(0)
        ctx.set_robot(make_robot(N_SPHERES, N_PAIRS))
        worlds = make_worlds(W, K)
        ctx.set_worlds(worlds.pose, worlds.half_ext)
        x0 = torch.tensor(make_trajectories(W, S, Tn).reshape(W * S, Tn, 7), dtype=torch.float32, device="cuda:0")
        if prec == "paper_like":
            from paper_2310_07854_amd import Shape
            ctx.set_precision({})
            sh = Shape(W, S, Tn, 1)
            q = x0.reshape(-1, 7).contiguous()
            _, ws = ctx.cost_fwd(q, sh)
            ctx.cost_bwd(q, ws, want_grad=False)
            amax = {t: float(ctx.ws_export(t, ws, sh).view(torch.float32).abs().max()) for t in
                    ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")}
            ctx.set_precision(with_scales(PRECISIONS["paper_like"], amax, ctx.reach()))
        else:
            ctx.set_precision({})
        res = {}
        for mode in ("eager", "graph"):
            opt = TrajectoryOptimizer(ctx, W, S, Tn, n_ls=nls, m=HIST_M)
            opt.init(x0)
            if mode == "graph":
                opt.capture()
            run = opt.replay if mode == "graph" else opt.step
            for _ in range(args.warmup):
                run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                run()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            B = W * S * Tn * nls
            res[mode] = {"ms_per_step": dt * 1e3, "evals_per_s": B / dt}
            del opt
        ctx.close()
        res["graph_speedup"] = res["eager"]["ms_per_step"] / res["graph"]["ms_per_step"]
        out[name] = res
        print(f"# graph {name}: eager {res['eager']['ms_per_step']*1e3:.1f} us/step, graph "
              f"{res['graph']['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "optimiser iteration: eager launches vs one HIP graph replay", "data": "synthetic",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "results": out}), flush=True)


def search_study(args):
    """The variable-precision search on synthetic planning problems: problems drawn like the
    benchmark worlds (16 cuboids each, start and goal collision-free), 8 linear seeds of 32
    timesteps each, `search_iters` optimiser iterations per evaluation; an assignment succeeds on a
    problem when one of its final trajectories is collision-free, and must keep the FP32 success
    rate.  The arm is the benchmark's without self pairs (its random sphere model overlaps itself)."""
    import dataclasses
    from types import SimpleNamespace

    import torch

    from paper_2310_07854_amd import Context, search as SR, seed_pipeline as SP
    from synthetic import make_robot, make_seed_inits, make_seed_problems

    K, T_S, S_S = 16, 32, 8
    robot = make_robot(N_SPHERES, N_PAIRS)
    robot = dataclasses.replace(robot, pairs=robot.pairs[:0])
    ctx = Context(0)
    ctx.set_robot(robot)
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")
    keep = {"pose": [], "half": [], "start": [], "goal": []}
    have, split = 0, 200
    while have < args.search_problems:
        pr = make_seed_problems(4096, K, split=split)
        ctx.set_worlds(pr.worlds.pose, pr.worlds.half_ext)
        ok = SP.endpoints_free(ctx, d(pr.start), d(pr.goal)).cpu().numpy()
        for key, arr in (("pose", pr.worlds.pose), ("half", pr.worlds.half_ext), ("start", pr.start),
                         ("goal", pr.goal)):
            keep[key].append(arr[ok])
        have += int(ok.sum())
        split += 1
    n = args.search_problems
    p = {k: np.concatenate(v)[:n] for k, v in keep.items()}
    worlds = SimpleNamespace(pose=p["pose"], half_ext=p["half"])
    x0 = make_seed_inits(p["start"], p["goal"], S_S, T_S, "linear", split=5)
    task = SR.OptimizerTask(ctx, worlds, p["start"], p["goal"], x0, iters=args.search_iters, n_ls=4)
    evals = []

    def timed_eval(a):
        t0 = time.perf_counter()
        r = task(a)
        evals.append(time.perf_counter() - t0)
        print(f"# search: {r:.4f} " + " ".join(f"{t}={f}" for t, f in a.items()), file=sys.stderr, flush=True)
        return r

    # success counts move by a problem or two under changes that do not matter (the optimiser's
    # trajectories branch on tiny differences), so the target is the FP32 rate less one binomial
    # standard error of it
    p32 = task({t: "f32" for t in SR.TENSORS})
    tol = math.sqrt(max(p32 * (1.0 - p32), 0.0) / n)
    res = SR.Search(timed_eval, tolerance=tol).run(budget=args.search_budget, seed=0)
    ctx.close()
    line = {"metric": "variable-precision search: fewest stored-tensor bits at the FP32 collision-free rate",
            "data": "synthetic", "n_gpus": 1,
            "config": {"workload": f"{n} problems (worlds of {K} cuboids), {S_S} linear seeds x {T_S} timesteps, "
                                   f"{args.search_iters} optimiser iterations per evaluation; 21-type ladder",
                       "budget": args.search_budget},
            "fp32_rate": res.fp32_rate, "target": res.target, "tolerance": tol, "per_tensor": res.per_tensor,
            "best": res.best,
            "best_rate": res.best_rate, "best_bits": res.best_bits, "fp32_bits": 32 * len(res.best),
            "evaluations": res.evaluations, "seconds": res.seconds,
            "seconds_per_evaluation": float(np.median(evals)) if evals else None,
            "history": [[a, r] for a, r in res.history]}
    print(json.dumps(line), flush=True)


IK_SEEDS = 2000


def ik_bench(args):
    """Inverse kinematics: 64 problems (worlds of 64 cuboids) x 2,000 seeds, one configuration per
    trajectory (128,000 configurations per step), pose cost against each problem's goal (the link-8
    pose of a random configuration, so every goal is reachable) plus the collision, self and bound
    costs; one optimiser iteration per step with free rows.  FP32 and the paper-like assignment."""
    import torch

    from paper_2310_07854_amd import Context, TrajectoryOptimizer
    from synthetic import make_configs, make_robot, make_worlds

    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    B = N_WORLDS * IK_SEEDS
    ctx = Context(0)
    ctx.set_robot(robot)
    ctx.set_worlds(worlds.pose, worlds.half_ext)
    # goals: link-8 poses of random configurations, computed by the library's own kinematics
    qg = torch.tensor(make_configs(N_WORLDS, seed=77), dtype=torch.float32, device="cuda:0")
    from paper_2310_07854_amd import Shape

    ctx.set_precision({})
    sh_g = Shape(N_WORLDS, 1, 1, 1)
    _, wsg = ctx.cost_fwd(qg, sh_g)
    L = ctx.ws_export("link_poses", wsg, sh_g).view(torch.float32).view(N_WORLDS, 8, 12)
    goals = L[:, 7].reshape(N_WORLDS, 3, 4).cpu().numpy()
    ctx.set_goals(goals)
    x0 = torch.tensor(make_configs(B, seed=78), dtype=torch.float32, device="cuda:0").reshape(N_WORLDS * IK_SEEDS, 1, 7)
    ctx.set_precision({})
    shape = Shape(N_WORLDS, IK_SEEDS, 1, 1)
    q = x0.reshape(-1, 7).contiguous()
    _, ws = ctx.cost_fwd(q, shape)
    ctx.cost_bwd(q, ws, want_grad=False)
    names = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")
    amax = {t: float(ctx.ws_export(t, ws, shape).view(torch.float32).abs().max()) for t in names}
    out = {}
    for name in ("f32", "paper_like"):
        prec = with_scales(PRECISIONS[name], amax, ctx.reach())
        ctx.set_precision(prec)
        opt = TrajectoryOptimizer(ctx, N_WORLDS, IK_SEEDS, 1, n_ls=N_LS, m=HIST_M, pin_ends=False)
        opt.init(x0)
        c0 = float(opt.cost.sum())
        for _ in range(args.warmup):
            opt.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            opt.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # per-kernel durations from a second region with HIP events around every launch
        ctx.profile_enable(True)
        for _ in range(args.steps):
            opt.step()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        kern = {kk: v[0] / max(v[1], 1) * 1e3 for kk, v in prof.items() if v[1]}
        work = culled_work(ctx, opt, prec) if name == "paper_like" else None
        out[name] = {"value": B * args.steps / dt, "ms_per_step": dt / args.steps * 1e3, "kernels_us": kern,
                     "cost_first": c0, "cost_last": float(opt.cost.sum()),
                     "formats": {kk: list(v) for kk, v in prec.items()}}
        if work:
            out[name]["culled"] = work
        print(f"# ik {name}: {dt / args.steps * 1e3:.3f} ms/step, {B * args.steps / dt / 1e6:.1f} M evals/s, "
              + ", ".join(f"{kk} {v:.1f}us" for kk, v in kern.items()), file=sys.stderr, flush=True)
        del opt
    ctx.close()
    pl = out["paper_like"]
    kern = pl["kernels_us"]
    dom = max(kern, key=lambda k: kern[k])
    if dom == "sphere_cost":
        flops = FLOPS_PER_SPHERE_CUBOID * pl["culled"]["needed_tests_per_cfg"] + FLOPS_PER_PAIR * N_PAIRS
        achieved = flops * B / (kern[dom] * 1e-6) / 1e12
        roofline = {"kernel": "k_sphere_cost", "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS, "flops_per_cfg": flops}
    else:
        kb = kernel_bytes({kk: tuple(v) for kk, v in pl["formats"].items()})
        achieved = kb.get(dom, 0.0) * B / (kern[dom] * 1e-6) / 1e9
        roofline = {"kernel": "k_" + dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS}
    roofline["traffic"] = workload_traffic("ik", pl["formats"], roofline["kernel"])
    line = {"metric": "inverse-kinematics cost fwd+bwd evals/s (one optimiser iteration per step)",
            "value": pl["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": pl["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{N_WORLDS} problems x {IK_SEEDS} seeds = {B:,} configurations per step; 7-joint "
                                   f"arm, 60 spheres, 300 self pairs, 64 cuboids per world; pose cost + collision",
                       "precision": "paper_like", "formats": pl["formats"]},
            "fp32_value": out["f32"]["value"], "variants": out, "roofline": roofline,
            "cpu_baseline": None if args.no_cpu_baseline else ik_cpu_baseline(
                {kk: tuple(v) for kk, v in pl["formats"].items()})}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="paper_like", choices=[k for k in PRECISIONS if k != "f32"])
    ap.add_argument("--parts", type=int, default=PARTS,
                    help="world partitions, one context and stream each, for the timed steps (1: one stream)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seeding", action="store_true", help="run the learned-seeder study instead")
    ap.add_argument("--seed-infer", action="store_true", help="time the seeding network's inference instead")
    ap.add_argument("--swept", type=int, default=0, help="time the step with the swept term (k samples) instead")
    ap.add_argument("--ik", action="store_true", help="time the inverse-kinematics workload instead")
    ap.add_argument("--search", action="store_true", help="run the variable-precision search instead")
    ap.add_argument("--graph", action="store_true", help="time eager iterations against HIP graph replays instead")
    ap.add_argument("--search-problems", type=int, default=1024)
    ap.add_argument("--search-iters", type=int, default=60)
    ap.add_argument("--search-budget", type=int, default=60)
    ap.add_argument("--seed-batch", type=int, default=65536)
    ap.add_argument("--seed-envs", type=int, default=2)
    ap.add_argument("--seed-problems", type=int, default=32768)
    ap.add_argument("--seed-solve-iters", type=int, default=60)
    ap.add_argument("--seed-train-steps", type=int, default=8000)
    ap.add_argument("--seed-eval", type=int, default=1024)
    ap.add_argument("--seed-eval-iters", type=int, default=30)
    ap.add_argument("--seed-targets", choices=["lowest", "diverse"], default="lowest",
                    help="training targets: the 8 lowest-cost solutions, or 8 spread-out ones")
    ap.add_argument("--seed-train-inits", choices=["linear", "mixed"], default="linear",
                    help="initial trajectories of the training solves: linear, or half linear half random")
    ap.add_argument("--only", choices=list(PRECISIONS), default=None,
                    help="run one assignment's optimisation loop and nothing else (for profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB, 5 times (profiler calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_MiB": args.copy_calibration, "launches": 5}))
        return
    if args.seeding:
        seeding_study(args)
        return
    if args.seed_infer:
        seed_inference(args)
        return
    if args.swept:
        swept_bench(args)
        return
    if args.ik:
        ik_bench(args)
        return
    if args.search:
        search_study(args)
        return
    if args.graph:
        graph_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the cost path shards by world "
              "with no communication, so more GPUs are not exercised here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2310_07854_amd import Context, TrajectoryOptimizer
    from synthetic import make_robot, make_trajectories, make_worlds

    B = N_WORLDS * TPW * T * N_LS
    robot = make_robot(N_SPHERES, N_PAIRS)
    worlds = make_worlds(N_WORLDS, N_CUBOIDS)
    x0 = torch.tensor(make_trajectories(N_WORLDS, TPW, T).reshape(N_WORLDS * TPW, T, 7), dtype=torch.float32,
                      device="cuda:0")
    ctx = Context(0)
    ctx.set_robot(robot)
    ctx.set_worlds(worlds.pose, worlds.half_ext)

    amax = calibrate_scales(torch, ctx, x0)
    precs = {name: with_scales(f, amax, ctx.reach()) for name, f in PRECISIONS.items()}
    if args.only:
        dt, prof, _, _, st = run_variant(torch, ctx, TrajectoryOptimizer, x0, precs[args.only], args.steps,
                                         args.warmup)
        print(json.dumps({"only": args.only, "ms_per_step": dt / args.steps * 1e3,
                          "config": {"formats": {k: list(v) for k, v in precs[args.only].items()}},
                          "kernels_us": {k: v[0] / max(v[1], 1) * 1e3 for k, v in prof.items() if v[1]},
                          "optimizer_stats": st,
                          "optimizer_bytes_per_launch": kernel_bytes(precs[args.only], opt_stats=st)["optimizer"]
                          * N_WORLDS * TPW * T * N_LS}))
        ctx.close()
        return
    # every named assignment, stored poses and recomputed in the backward pass; FP32 only stored
    results = {}
    names = ["f32", args.precision] + [k for k in PRECISIONS if k not in ("f32", args.precision)]
    culled = None
    census = activity = None
    opt_stats = {}
    for name in names:
        for recompute in ((False,) if name == "f32" else (False, True)):
            main = name == args.precision and not recompute
            if args.parts > 1:
                dtp, costp = run_partitioned(torch, ctx, x0, precs[name], args.steps, args.warmup, args.parts,
                                             recompute)
                if not math.isfinite(costp):
                    raise RuntimeError(f"{name}: non-finite total cost after the partitioned steps")
            dt, prof, cost, opt, st = run_variant(torch, ctx, TrajectoryOptimizer, x0, precs[name], args.steps,
                                                  args.warmup, want_opt=main, recompute=recompute)
            opt_stats[name + ("_recompute" if recompute else "")] = st
            if args.parts <= 1:
                dtp = dt
            results[(name, recompute)] = {"seconds": dt, "prof": prof, "cost": cost, "seconds_parts": dtp}
            if main:
                culled = culled_work(ctx, opt, precs[name])
                census, activity = stored_tensor_report(torch, ctx, opt, precs[name])
                del opt
            print(f"# {name}{' recompute' if recompute else ''}: {dt / args.steps * 1e3:.3f} ms/step, "
                  f"{B * args.steps / dt / 1e6:.1f} M evals/s on one stream, "
                  f"{B * args.steps / dtp / 1e6:.1f} M evals/s on {args.parts}, kernels "
                  + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f}us" for k, v in prof.items() if v[1])
                  + "; optimiser per trajectory and iteration: "
                  + ", ".join(f"{k} {v:.3f}" for k, v in st.items() if k != "iterations"),
                  file=sys.stderr, flush=True)
            if not math.isfinite(cost):
                raise RuntimeError(f"{name}: non-finite total cost after the timed steps")

    fwd_bwd = {name: fwd_bwd_timing(torch, ctx, x0, precs[name]) for name in ("f32", args.precision)}
    fwd_bwd[args.precision + "_recompute"] = fwd_bwd_timing(torch, ctx, x0, precs[args.precision], True)
    copy_gbs = copy_bandwidth(torch)
    cold = {name: cold_kernels(torch, ctx, TrajectoryOptimizer, x0, precs[name]) for name in ("f32", args.precision)}
    print("# cold/warm us: " + "; ".join(f"{n} " + ", ".join(f"{k} {v['cold_us']:.1f}/{v['warm_us']:.1f}"
                                                          for k, v in c.items()) for n, c in cold.items()),
          file=sys.stderr, flush=True)

    # the headline assignment's cost and gradient at the initial trajectories, for the error of
    # sampled trajectories against the FP64 oracle (cpu_baseline leg)
    from paper_2310_07854_amd import Shape

    ctx.set_precision(precs[args.precision])
    shape1 = Shape(N_WORLDS, TPW, T, 1)
    q0 = x0.reshape(-1, 7).contiguous()
    c0, ws0 = ctx.cost_fwd(q0, shape1)
    g0 = ctx.cost_bwd(q0, ws0)
    err_tr = np.sort(np.random.default_rng(2310).choice(N_WORLDS * TPW, 16, replace=False))
    err_rows = (err_tr[:, None] * T + np.arange(T)[None, :]).reshape(-1)
    gpu_sample = {"traj": err_tr, "cost": c0.cpu().numpy()[err_tr], "grad": g0.cpu().numpy()[err_rows]}
    del ws0

    main_r = results[(args.precision, False)]
    f32_r = results[("f32", False)]
    rc_r = results[(args.precision, True)]
    dt = main_r["seconds_parts"]
    dt_rc = rc_r["seconds_parts"]
    prof_rc = rc_r["prof"]
    value = B * args.steps / dt
    value_f32 = B * args.steps / f32_r["seconds_parts"]
    value_1 = B * args.steps / main_r["seconds"]
    value_f32_1 = B * args.steps / f32_r["seconds"]
    prec = precs[args.precision]
    kb = kernel_bytes(prec, opt_stats=opt_stats.get(args.precision))
    per_kernel = {}
    for k, (ms, n) in main_r["prof"].items():
        if n == 0:
            continue
        avg_s = ms / n / 1e3
        entry = {"avg_us": avg_s * 1e6, "launches": n}
        if k in kb:
            entry["algorithmic_GBs"] = kb[k] * B / avg_s / 1e9
        if k in cold[args.precision]:
            cu = cold[args.precision][k]["cold_us"]
            entry["cold_us"] = cu
            if k in kb:
                entry["cold_algorithmic_GBs"] = kb[k] * B / (cu * 1e-6) / 1e9
                entry["cold_frac_of_peak"] = entry["cold_algorithmic_GBs"] / HBM_PEAK_GBS
                entry["cold_frac_of_copy"] = entry["cold_algorithmic_GBs"] / copy_gbs
        per_kernel[k] = entry
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"] * per_kernel[k]["launches"])
    dom_s = per_kernel[dom]["avg_us"] * 1e-6
    traffic = traffic_from_profile(kernels_hash(), {k: list(v) for k, v in prec.items()})
    if dom == "sphere_cost":
        # the tests exact culling leaves, plus every self pair once
        flops = FLOPS_PER_SPHERE_CUBOID * culled["needed_tests_per_cfg"] + FLOPS_PER_PAIR * N_PAIRS
        achieved = flops * B / dom_s / 1e12
        roofline = {"kernel": "k_sphere_cost", "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS,
                    "flops_per_cfg": flops, "culled_tests_per_cfg": culled["needed_tests_per_cfg"],
                    "issued_lane_tests_per_cfg": culled["issued_lane_tests_per_cfg"],
                    "dense_equivalent_TFLOPs": dense_flops_per_cfg() * B / dom_s / 1e12}
    else:
        achieved = kb[dom] * B / dom_s / 1e9
        roofline = {"kernel": "k_" + dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
    roofline["traffic"] = (traffic or {}).get("bytes_per_launch", {}).get(roofline["kernel"]) if traffic else None

    def kernels_us(prof):
        return {k: v[0] / max(v[1], 1) * 1e3 for k, v in prof.items() if v[1]}

    variants = {}
    for (name, recompute), r in results.items():
        v = B * args.steps / r["seconds_parts"]
        v1 = B * args.steps / r["seconds"]
        variants[name + ("_recompute" if recompute else "")] = {
            "value": v, "ms_per_step": r["seconds_parts"] / args.steps * 1e3,
            "speedup_vs_fp32_pct": (v / value_f32 - 1.0) * 100.0,
            "single_stream_value": v1, "single_stream_speedup_vs_fp32_pct": (v1 / value_f32_1 - 1.0) * 100.0,
            "formats": {k: list(f) for k, f in precs[name].items()}, "kernels_us": kernels_us(r["prof"])}
    step_bytes = sum(kb[k] for k in kb) * B
    line = {
        "metric": "cost fwd+bwd evals/s (one optimiser iteration per step), variable precision vs FP32",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 worlds x 64 seeds x 48 timesteps = 196,608 configurations per step; 7-joint "
                               "arm, 60 spheres, 300 self pairs, 64 oriented cuboids per world; 1 step scale",
                   "precision": args.precision, "formats": {k: list(v) for k, v in prec.items()},
                   "recompute_poses": False, "partitions": args.parts},
        # the same steps on one stream; per-kernel times and the roofline come from that run, where
        # each launch has the GPU to itself
        "single_stream": {"value": value_1, "ms_per_step": main_r["seconds"] / args.steps * 1e3,
                          "fp32_value": value_f32_1, "speedup_vs_fp32_pct": (value_1 / value_f32_1 - 1.0) * 100.0},
        "fp32_value": value_f32,
        # the paper's definition: (t_FP32 / t_X - 1) * 100 %
        "speedup_vs_fp32_pct": (value / value_f32 - 1.0) * 100.0,
        "hbm_algorithmic_GBs": step_bytes / (dt / args.steps) / 1e9,
        "kernels": per_kernel,
        "fp32_kernels": kernels_us(f32_r["prof"]),
        "roofline": roofline,
        # codes of the headline's stored tensors after the timed steps: saturated or Inf/NaN counts
        # (static scales outgrown), and how dense D and G are (the share of spheres with a nonzero value)
        "census": census,
        "active_fraction": activity,
        # per trajectory and iteration after the timed steps: accepted candidates, kept (s, y) pairs
        # and history pairs read by the two-loop recursion (the optimiser's algorithmic bytes use them)
        "optimizer_stats": opt_stats,
        "recompute_value": B * args.steps / dt_rc,
        "recompute_kernels": kernels_us(prof_rc),
        "variants": variants,
        "cold_kernels": cold,
        "fwd_bwd": fwd_bwd,
        "copy_GBs": copy_gbs,
        "copy_frac_of_peak": copy_gbs / HBM_PEAK_GBS,
    }
    ctx.close()
    line["batched"] = batched_workload(torch, max(args.steps, 50), args.warmup)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prec)
        line["error_vs_fp64"] = error_vs_fp64(prec, gpu_sample)
    else:
        line["cpu_baseline"] = None
        line["error_vs_fp64"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
