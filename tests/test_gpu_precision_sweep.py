"""Error of every precision assignment against the FP64 oracle on the batched workload (60 spheres,
40 cuboids, 4 worlds x 32 seeds x 32 timesteps x 4 line-search candidates = 16,384 configurations):
the cost and gradient path once per assignment of a format in {F32, F16, BF16, E4M3, E5M2, E3M2, E2M1}
to each of the five stored tensors (7^5 = 16,807 assignments, stored poses), against the unquantised
FP64 oracle:

  cost_max_rel   max over trajectory candidates of |c - c64| / |c64|
  cost_med_rel   median of the same
  grad_rel_l2    |g - g64|_2 / |g64|_2 over the whole batch of joint gradients

Scales as the benchmark calibrates them (link poses and sphere positions from the arm's reach, the
others from their FP32 magnitude, a binade of headroom where overflow gives Inf).  Asserts: every
cost and gradient finite (the overflow guard), the FP32 assignment at FP32 accuracy, the named
assignments within the error stated for them; prints the named rows and the bits/error Pareto fronts,
and writes every row to $VAPR_SWEEP_CSV when set.
"""
import csv
import itertools
import os
import time

import numpy as np
import pytest

from oracle import cost as OC
from synthetic import make_workload
from tests.gpu_helpers import dev, make_context, need_gpu, shape_of, torch

pytestmark = pytest.mark.gpu

FORMATS = ["f32", "f16", "bf16", "e4m3", "e5m2", "e3m2", "e2m1"]
BITS = {"f32": 32, "f16": 16, "bf16": 16, "e4m3": 8, "e5m2": 8, "e3m2": 6, "e2m1": 4}
VALUES = {"link_poses": 96, "sphere_pos": 180, "sphere_dist": 60, "sphere_grad": 180, "joint_grad": 7}
# name: (formats L, S, D, G, J), stated bound on (cost max rel, grad rel L2)
NAMED = {
    "fp32": (("f32",) * 5, (1e-6, 1e-5)),
    "all_fp16": (("f16",) * 5, (2e-4, 5e-2)),
    "all_bf16": (("bf16",) * 5, (2e-3, 1e-1)),
    "paper_like": (("f16", "f16", "e4m3", "e4m3", "e4m3"), (2e-2, 5e-2)),
    "all_fp8": (("e4m3", "e4m3", "e4m3", "e5m2", "e5m2"), (5e-2, 4e-1)),
    "mixed_fp4_fp8": (("e4m3", "e4m3", "e2m1", "e2m1", "e4m3"), (1e-1, 4e-1)),
    "all_fp6": (("e3m2",) * 5, (1e-1, 5e-1)),
}


def pareto(rows, key):
    front, best = [], float("inf")
    for r in sorted(rows, key=lambda r: (r["bits"], r[key])):
        if r[key] < best:
            front.append(r)
            best = r[key]
    return front


def test_precision_sweep():
    need_gpu()
    from paper_2310_07854_amd.search import spec

    wl = make_workload("batched")
    shape = shape_of(wl)
    t0 = time.time()
    ref = OC.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls, prec=None)
    c64, g64 = ref["cost_traj"], ref["grad_q"].reshape(-1)
    print(f"FP64 oracle on {shape.B} configurations: {time.time() - t0:.1f} s", flush=True)
    ctx = make_context(wl)
    q = dev(wl.q, torch.float32)
    ctx.set_precision({})
    _, ws = ctx.cost_fwd(q, shape)
    ctx.cost_bwd(q, ws, want_grad=False)
    tensors = list(VALUES)
    amax = {t: float(ctx.ws_export(t, ws, shape).view(torch.float32).abs().max()) for t in tensors}
    reach = ctx.reach()
    rows = []
    t0 = time.time()
    for i, combo in enumerate(itertools.product(FORMATS, repeat=5)):
        sp = spec(dict(zip(tensors, combo)), amax, reach)
        ctx.set_precision(sp)
        cost, ws = ctx.cost_fwd(q, shape, ws=ws)
        grad = ctx.cost_bwd(q, ws)
        c = cost.cpu().numpy()
        g = grad.cpu().numpy().astype(np.float64).reshape(-1)
        assert np.all(np.isfinite(c)) and np.all(np.isfinite(g)), combo
        rel = np.abs(c - c64) / np.abs(c64)
        rows.append({"L": combo[0], "S": combo[1], "D": combo[2], "G": combo[3], "J": combo[4],
                     "bits": sum(VALUES[t] * BITS[f] for t, f in zip(tensors, combo)),
                     "cost_max_rel": float(rel.max()), "cost_med_rel": float(np.median(rel)),
                     "grad_rel_l2": float(np.linalg.norm(g - g64) / np.linalg.norm(g64)),
                     "scales": " ".join(str(sp[t][1]) for t in tensors)})
        if (i + 1) % 4000 == 0:
            print(f"{i + 1} assignments, {time.time() - t0:.0f} s", flush=True)
    ctx.close()
    out = os.environ.get("VAPR_SWEEP_CSV")
    if out:
        with open(out, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=list(rows[0]))
            w.writeheader()
            w.writerows(rows)

    def show(r):
        return (f"| {r['L']} | {r['S']} | {r['D']} | {r['G']} | {r['J']} | {r['scales']} | {r['bits']} | "
                f"{r['cost_max_rel']:.2e} | {r['cost_med_rel']:.2e} | {r['grad_rel_l2']:.2e} |")

    head = ("| L | S | D | G | J | scales | bits/config | cost max rel | cost median rel | grad rel L2 |\n"
            + "|---" * 10 + "|")
    by = {(r["L"], r["S"], r["D"], r["G"], r["J"]): r for r in rows}
    print(f"\n{len(rows)} assignments in {time.time() - t0:.1f} s\nnamed assignments\n" + head)
    for name, (combo, _) in NAMED.items():
        print(show(by[combo]) + f" {name}")
    for key in ("grad_rel_l2", "cost_max_rel"):
        front = pareto(rows, key)
        print(f"\nPareto front, bits vs {key} ({len(front)} points)\n" + head)
        for r in front:
            print(show(r))
    for name, (combo, (cb, gb)) in NAMED.items():
        r = by[combo]
        assert r["cost_max_rel"] <= cb and r["grad_rel_l2"] <= gb, (name, r)
