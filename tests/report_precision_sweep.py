"""Error of every precision assignment against the FP64 oracle (needs a GPU).

For the batched workload (60 spheres, 40 cuboids, 4 worlds x 32 seeds x 32 timesteps x 4
line-search candidates = 16,384 configurations) this runs the cost and gradient path once per
assignment of a format in {F32, F16, BF16, E4M3, E5M2, E3M2, E2M1} to each of the five stored
tensors (7^5 = 16,807 assignments, stored poses) and compares with the unquantised FP64 oracle:

  cost_max_rel   max over trajectory candidates of |c - c64| / |c64|
  cost_med_rel   median of the same
  grad_rel_l2    |g - g64|_2 / |g64|_2 over the whole batch of joint gradients

Scales are powers of two calibrated once on the FP32 run, per tensor and format:
k = ceil(log2(amax / max_finite)) clamped to [-16, 16] (F32: 0).  Bits per configuration count the
stored values only (L 96, S 180, D 60, G 180, J 7).  Writes every row to a CSV and prints the
Pareto front of bits against each error plus the named assignments.

  python tests/report_precision_sweep.py [--out precision_sweep.csv] [--limit N]
"""
from __future__ import annotations

import argparse
import csv
import itertools
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import cost as OC  # noqa: E402
from paper_2310_07854_amd import Context  # noqa: E402
from paper_2310_07854_amd.context import Shape  # noqa: E402
from synthetic import make_workload  # noqa: E402

FORMATS = ["f32", "f16", "bf16", "e4m3", "e5m2", "e3m2", "e2m1"]
BITS = {"f32": 32, "f16": 16, "bf16": 16, "e4m3": 8, "e5m2": 8, "e3m2": 6, "e2m1": 4}
MAX_FINITE = {"f16": 65504.0, "bf16": 3.3895313892515355e38, "e4m3": 448.0, "e5m2": 57344.0, "e3m2": 28.0,
              "e2m1": 6.0}
TENSORS = ["link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad"]
VALUES = {"link_poses": 96, "sphere_pos": 180, "sphere_dist": 60, "sphere_grad": 180, "joint_grad": 7}
NAMED = {
    "fp32": ("f32", "f32", "f32", "f32", "f32"),
    "all_fp16": ("f16",) * 5,
    "all_bf16": ("bf16",) * 5,
    "all_fp8": ("e4m3", "e4m3", "e4m3", "e5m2", "e5m2"),
    "mixed_fp4_fp8": ("e4m3", "e4m3", "e2m1", "e2m1", "e4m3"),
    "paper_like": ("f16", "f16", "e4m3", "e4m3", "e4m3"),
    "all_fp6": ("e3m2",) * 5,
}


def scale_exp(amax: float, fmt: str) -> int:
    if fmt == "f32" or amax <= 0.0:
        return 0
    return int(min(16, max(-16, math.ceil(math.log2(amax / MAX_FINITE[fmt])))))


def pareto(rows, key):
    """Rows not dominated in (bits, key): sorted by bits, keeping strict improvements of key."""
    front, best = [], float("inf")
    for r in sorted(rows, key=lambda r: (r["bits"], r[key])):
        if r[key] < best:
            front.append(r)
            best = r[key]
    return front


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="precision_sweep.csv", help="CSV path (default: the working directory)")
    ap.add_argument("--limit", type=int, default=0, help="only the first N assignments (0: all)")
    args = ap.parse_args()

    wl = make_workload("batched")
    shape = Shape(wl.worlds.pose.shape[0], wl.traj_per_world, wl.T, wl.n_ls)
    t0 = time.time()
    ref = OC.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls, prec=None)
    c64 = ref["cost_traj"]
    g64 = ref["grad_q"].reshape(-1)
    print(f"FP64 oracle on {shape.B} configurations: {time.time() - t0:.1f} s", flush=True)

    ctx = Context(0)
    ctx.set_robot(wl.robot)
    ctx.set_worlds(wl.worlds.pose, wl.worlds.half_ext)
    q = torch.tensor(wl.q, dtype=torch.float32, device="cuda:0")

    # amax of every stored tensor on the FP32 path
    ctx.set_precision({})
    _, ws = ctx.cost_fwd(q, shape)
    ctx.cost_bwd(q, ws)
    amax = {t: float(ctx.ws_export(t, ws, shape).view(torch.float32).abs().max()) for t in TENSORS}
    print("amax: " + ", ".join(f"{t} {v:.4g}" for t, v in amax.items()), flush=True)

    combos = list(itertools.product(FORMATS, repeat=5))
    if args.limit:
        combos = combos[:args.limit]
    rows = []
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    t0 = time.time()
    for i, combo in enumerate(combos):
        spec = {t: (f, scale_exp(amax[t], f)) for t, f in zip(TENSORS, combo)}
        ctx.set_precision(spec)
        cost, ws = ctx.cost_fwd(q, shape)
        grad = ctx.cost_bwd(q, ws)
        c = cost.cpu().numpy()
        g = grad.cpu().numpy().astype(np.float64).reshape(-1)
        rel = np.abs(c - c64) / np.maximum(np.abs(c64), 1e-30)
        rows.append({"L": combo[0], "S": combo[1], "D": combo[2], "G": combo[3], "J": combo[4],
                     "bits": sum(VALUES[t] * BITS[f] for t, f in zip(TENSORS, combo)),
                     "cost_max_rel": float(rel.max()), "cost_med_rel": float(np.median(rel)),
                     "grad_rel_l2": float(np.linalg.norm(g - g64) / np.linalg.norm(g64)),
                     "scales": " ".join(str(spec[t][1]) for t in TENSORS)})
        if (i + 1) % 1000 == 0:
            print(f"{i + 1}/{len(combos)} assignments, {time.time() - t0:.0f} s", flush=True)
    ctx.close()

    with open(args.out, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    print(f"wrote {len(rows)} rows to {args.out}", flush=True)

    def show(r):
        return (f"| {r['L']} | {r['S']} | {r['D']} | {r['G']} | {r['J']} | {r['bits']} | {r['cost_max_rel']:.2e} "
                f"| {r['cost_med_rel']:.2e} | {r['grad_rel_l2']:.2e} |")

    head = "| L | S | D | G | J | bits/config | cost max rel | cost median rel | grad rel L2 |\n" + "|---" * 9 + "|"
    by = {(r["L"], r["S"], r["D"], r["G"], r["J"]): r for r in rows}
    print("\nnamed assignments\n" + head)
    for name, combo in NAMED.items():
        if combo in by:
            print(show(by[combo]) + f" {name}")
    for key in ("grad_rel_l2", "cost_max_rel"):
        print(f"\nPareto front, bits vs {key}\n" + head)
        for r in pareto(rows, key):
            print(show(r))


if __name__ == "__main__":
    main()
