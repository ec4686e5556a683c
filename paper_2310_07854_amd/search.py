"""Variable-precision search (Sec. V-A; results Sec. VI-A): find, for the stored tensors, the
narrowest floating-point types that keep the task success rate of FP32.

  phase 1   per tensor, binary search along the type ladder for the narrowest type whose success
            rate (every other tensor FP32) reaches the target; types narrower than it are dropped
  phase 2   across tensors, minimise the total bit width over the reduced space subject to the
            same success constraint.  The paper drives this phase with NSGA-II in a black-box
            optimiser; here a budgeted local search stands in: repair the phase-1 assignment step
            by step until feasible, descend greedily to narrower types, then a seeded (mu + lambda)
            evolution with the remaining budget

The ladder holds the 21 types of the format space, narrowest first; a type with a storage codec
(e2m1, e3m2, e4m3, e5m2, f16, bf16, f32) is stored in it, every other type is emulated (FP32
values rounded to it at each write).  Each type gets a power-of-two scale so that its largest finite
value covers the tensor: the robot's reach for link poses and sphere positions, the FP32 magnitude
on a calibration batch (with a binade of headroom where overflow gives Inf) for the others.

The search only needs an `evaluate(assignment) -> success rate` callable; `OptimizerTask` builds
one from synthetic planning problems run through the library's optimiser.
"""
from __future__ import annotations

import math
import re
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

TENSORS = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")

# narrowest first; storage-format names where the type has a codec
LADDER: Tuple[str, ...] = (
    "e1m2", "e2m1",                        # FP4
    "e1m3", "e2m2", "e3m1", "e4m0",        # FP5
    "e2m3", "e3m2", "e4m1",                # FP6
    "e3m4", "e4m3", "e5m2",                # FP8
    "e4m5", "e5m4",                        # FP10
    "e5m7", "e6m6",                        # FP13
    "e5m9", "e6m8",                        # FP15
    "f16", "bf16",                         # FP16
    "f32",                                 # FP32
)

_STORAGE = {"f32": (8, 23), "f16": (5, 10), "bf16": (8, 7), "e4m3": (4, 3), "e5m2": (5, 2), "e3m2": (3, 2),
            "e2m1": (2, 1)}
# largest finite values of the storage formats (E4M3 and E5M2 follow their 8-bit storage encodings)
_STORAGE_MAX = {"f32": 3.4028234663852886e38, "f16": 65504.0, "bf16": 3.3895313892515355e38, "e4m3": 448.0,
                "e5m2": 57344.0, "e3m2": 28.0, "e2m1": 6.0}


def exp_man(fmt: str) -> Tuple[int, int]:
    if fmt in _STORAGE:
        return _STORAGE[fmt]
    m = re.fullmatch(r"e(\d+)m(\d+)", fmt)
    if not m:
        raise ValueError(f"unknown format {fmt!r}")
    return int(m.group(1)), int(m.group(2))


def bits(fmt: str) -> int:
    E, M = exp_man(fmt)
    return 1 + E + M


def max_finite(fmt: str) -> float:
    """Largest finite value: the storage encodings', else that of the emulated type (E5M10 and the
    8-exponent-bit types reserve the top exponent field, the others use every field)."""
    if fmt in _STORAGE_MAX:
        return _STORAGE_MAX[fmt]
    E, M = exp_man(fmt)
    bias = (1 << (E - 1)) - 1
    e_max = ((1 << E) - 2 if (E, M) == (5, 10) or E == 8 else (1 << E) - 1) - bias
    return (2.0 - 2.0 ** -M) * 2.0 ** e_max


def saturates(fmt: str) -> bool:
    """True for the types whose overflow clamps to the largest finite value; FP16, BF16, FP32 and
    the IEEE-like emulated types (E5M10, E8My) overflow to Inf instead."""
    E, M = exp_man(fmt)
    return not (fmt in ("f16", "bf16", "f32") or (E, M) == (5, 10) or E == 8)


def scale_for(fmt: str, amax: float, headroom: int = 0) -> int:
    """Power-of-two scale exponent k (|k| <= 16) with amax 2^(headroom - k) within the type's range;
    0 for f32."""
    if fmt == "f32" or amax <= 0:
        return 0
    return int(min(16, max(-16, math.ceil(math.log2(amax * 2.0 ** headroom / max_finite(fmt))))))


def spec(assignment: Dict[str, str], amax: Dict[str, float],
         reach: Optional[Tuple[float, float]] = None) -> Dict[str, Tuple[str, int]]:
    """Context.set_precision argument for an assignment of ladder types.  With the robot's reach
    (Context.reach(): bounds of every link-pose entry and sphere coordinate over all
    configurations), link poses and sphere positions take their scale from it, so that no
    configuration leaves the range; the other tensors from their FP32 magnitude `amax` on a
    calibration batch, with one binade of headroom for the types that overflow to Inf."""
    out = {}
    for t, f in assignment.items():
        if reach is not None and t in ("link_poses", "sphere_pos"):
            out[t] = (f, scale_for(f, reach[0] if t == "link_poses" else reach[1]))
        else:
            out[t] = (f, scale_for(f, amax.get(t, 0.0), 0 if saturates(f) else 1))
    return out


@dataclass
class SearchResult:
    target: float
    fp32_rate: float
    per_tensor: Dict[str, str]
    best: Dict[str, str]
    best_rate: float
    best_bits: int
    evaluations: int
    history: List[Tuple[Dict[str, str], float]] = field(default_factory=list)
    seconds: float = 0.0


class Search:
    """The two-phase search over `ladder` for `tensors`, with a memoising evaluator."""

    def __init__(self, evaluate: Callable[[Dict[str, str]], float], tensors: Sequence[str] = TENSORS,
                 ladder: Sequence[str] = LADDER, tolerance: float = 0.0):
        self._evaluate = evaluate
        self.tensors = tuple(tensors)
        self.ladder = tuple(ladder)
        self.tolerance = tolerance
        self.cache: Dict[Tuple[str, ...], float] = {}
        self.history: List[Tuple[Dict[str, str], float]] = []

    def rate(self, assignment: Dict[str, str]) -> float:
        key = tuple(assignment[t] for t in self.tensors)
        if key not in self.cache:
            r = float(self._evaluate(dict(assignment)))
            self.cache[key] = r
            self.history.append((dict(assignment), r))
        return self.cache[key]

    def _fp32(self) -> Dict[str, str]:
        return {t: "f32" for t in self.tensors}

    def per_tensor(self, target: float) -> Dict[str, str]:
        """Phase 1: for each tensor, the narrowest ladder type that reaches the target with every
        other tensor FP32 (binary search: the success rate is taken as monotone in the ladder)."""
        out = {}
        top = len(self.ladder) - 1
        for t in self.tensors:
            lo, hi = 0, top                    # the answer lies in [lo, hi]; ladder[top] reaches the target
            while lo < hi:
                mid = (lo + hi) // 2
                a = self._fp32()
                a[t] = self.ladder[mid]
                if self.rate(a) >= target:
                    hi = mid
                else:
                    lo = mid + 1
            out[t] = self.ladder[lo]
        return out

    def combine(self, floor: Dict[str, str], target: float, budget: int = 60, population: int = 6,
                seed: int = 0) -> Tuple[Dict[str, str], float]:
        """Phase 2: fewest total bits over assignments at or above each tensor's phase-1 type whose
        success rate reaches the target, within `budget` new evaluations:
          repair   from the phase-1 types (usually infeasible together), raise one tensor one ladder
                   step at a time, the step with the best success rate (then fewest bits), until
                   feasible
          descent  lower any tensor to the next narrower type while that stays feasible
          evolve   (mu + lambda) with the remaining budget: mutate one tensor one ladder step,
                   keep the feasible assignments with the fewest bits"""
        rng = np.random.default_rng(seed)
        lo = {t: self.ladder.index(floor[t]) for t in self.tensors}
        top = len(self.ladder) - 1
        evals0 = len(self.cache)

        def left():
            return budget - (len(self.cache) - evals0)

        def total(a):
            return sum(bits(a[t]) for t in self.tensors)

        def order(a):
            return (total(a), tuple(self.ladder.index(a[t]) for t in self.tensors))

        def feasible(a):
            return self.rate(a) >= target

        def moved(a, t, step):
            i = self.ladder.index(a[t])
            j = min(top, max(lo[t], i + step))
            if j == i:
                return None
            b = dict(a)
            b[t] = self.ladder[j]
            return b

        pool = [self._fp32()] if feasible(self._fp32()) else []
        a = dict(floor)
        while not feasible(a) and left() > 0:
            ups = [b for b in (moved(a, t, 1) for t in self.tensors) if b is not None]
            if not ups:
                break
            a = max(ups, key=lambda b: (self.rate(b), -total(b)))
        if feasible(a):
            pool.append(a)
            improved = True
            while improved and left() > 0:
                improved = False
                for t in sorted(self.tensors, key=lambda t: -bits(a[t])):
                    b = a
                    while True:  # the next narrower type (equal widths are skipped)
                        b = moved(b, t, -1)
                        if b is None or bits(b[t]) < bits(a[t]):
                            break
                    if b is not None and left() > 0 and feasible(b):
                        a = b
                        pool.append(a)
                        improved = True
        for _ in range(8 * budget):
            if left() <= 0 or not pool:
                break
            pool.sort(key=order)
            parents = pool[:population]
            child = moved(parents[int(rng.integers(len(parents)))], self.tensors[int(rng.integers(len(self.tensors)))],
                          -1 if rng.random() < 0.75 else 1)  # mostly try narrower types
            if child is not None and feasible(child) and child not in pool:
                pool.append(child)
        pool.sort(key=order)
        best = pool[0] if pool else self._fp32()
        return best, self.rate(best)

    def run(self, budget: int = 60, seed: int = 0) -> SearchResult:
        t0 = time.perf_counter()
        fp32_rate = self.rate(self._fp32())
        target = fp32_rate - self.tolerance
        floor = self.per_tensor(target)
        best, r = self.combine(floor, target, budget=budget, seed=seed)
        return SearchResult(target=target, fp32_rate=fp32_rate, per_tensor=floor, best=best, best_rate=r,
                            best_bits=sum(bits(best[t]) for t in self.tensors), evaluations=len(self.cache),
                            history=list(self.history), seconds=time.perf_counter() - t0)


class OptimizerTask:
    """Success rate of an assignment on synthetic planning problems: every problem's seeds go
    through `iters` optimiser iterations with the assignment's stored-tensor types, and a problem
    succeeds when one of its final trajectories is collision-free (no sphere penetrates a cuboid, no
    self pair overlaps, joint limits hold, at every timestep, checked in FP32)."""

    def __init__(self, ctx, worlds, start, goal, x0, iters: int = 40, n_ls: int = 4):
        import torch

        from .context import Shape

        self.ctx = ctx
        self.worlds = worlds
        self.W, self.S, self.T = x0.shape[0], x0.shape[1], x0.shape[2]
        self.x0 = torch.as_tensor(np.asarray(x0, dtype=np.float32), device="cuda:0")
        self.iters = iters
        self.n_ls = n_ls
        ctx.set_worlds(worlds.pose, worlds.half_ext)
        ctx.set_precision({})
        shape = Shape(self.W, self.S, self.T, 1)
        q = self.x0.reshape(-1, 7).contiguous()
        _, ws = ctx.cost_fwd(q, shape)
        ctx.cost_bwd(q, ws, want_grad=False)
        self.amax = {t: float(ctx.ws_export(t, ws, shape).view(torch.float32).abs().max()) for t in TENSORS}
        self.reach = ctx.reach()

    def __call__(self, assignment: Dict[str, str]) -> float:
        from . import seed_pipeline as SP
        from .optim import TrajectoryOptimizer

        self.ctx.set_precision(spec(assignment, self.amax, self.reach))
        opt = TrajectoryOptimizer(self.ctx, self.W, self.S, self.T, n_ls=self.n_ls)
        opt.init(self.x0)
        for _ in range(self.iters):
            opt.step()
        x = opt.x.view(self.W, self.S, self.T, 7).clone()
        self.ctx.set_precision({})
        free = SP.trajectories_free(self.ctx, x).any(dim=1)
        return float(free.float().mean().item())
