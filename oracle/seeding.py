"""FP64 reference of the learned trajectory seeder.  TEST INFRASTRUCTURE (only tests/, the smoke
check and the benchmark's CPU leg use it; the library never does).

The paper seeds trajectory optimisation with a geometric planner and notes that a network trained
for an environment could take its place (Sec. II-A, III-B) and that better seeding would cut the
number of planning attempts (Sec. VI-B).  This module defines such a seeder plainly, in FP64:

  occupancy  the cube [-0.75, 0.75]^3 m cut into 8 x 8 x 8 voxels of edge e = 0.1875 m; voxel
             (x, y, z) (index (z * 8 + y) * 8 + x) is occupied (1) when the smallest signed
             distance of its centre to the world's cuboids is <= e / 2, else 0
  features   x = [start (7), goal (7), occupancy (512)]                        526 values
  network    h_l = GELU(h_{l-1} W_l + b_l), l = 1..3, 256 units each; y = h_3 W_4 + b_4, 1792
             values read as 8 seeds x 32 timesteps x 7 joints: seed s's trajectory is the
             straight line from start to goal plus y[s] (rows t = 0 and 31 are pinned to the
             endpoints by the optimiser that consumes the seeds)
             GELU(z) = z * Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (exact form)
  loss       min-over-slot matching: e_sj = mean over (t, joint) of (y_s - y*_j)^2 for predicted
             slot s and target j; L = sum over valid (problem, target) of min_s e_sj / #valid;
             the smallest e wins, ties to the lowest slot
  optimiser  Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
             w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

The GPU multiplies BF16 operands with FP32 accumulation.  With `emulate=True` the features,
weights, hidden activations and the back-propagated gradients are rounded to BF16 (round to
nearest even) exactly where the GPU path stores them in BF16; FP32 rounding of the accumulations
is not emulated (the parity tests bound it instead).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

from . import formats as fmts
from .geometry import obb_signed_distance

GRID = 8
CUBE_LO, CUBE_HI = -0.75, 0.75
N_SEEDS, T_SEED, N_J = 8, 32, 7
N_IN = 2 * N_J + GRID ** 3          # 526
N_HID = 256
N_OUT = N_SEEDS * T_SEED * N_J       # 1792
LAYERS = ((N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT))


def bf16(x) -> np.ndarray:
    """Round to BF16 (through FP32), as an FP64 array."""
    return fmts.roundtrip(fmts.fp32(x), "bf16")[1].astype(np.float64)


def voxel_centres() -> np.ndarray:
    """[512, 3] centres in index order (z * 8 + y) * 8 + x."""
    e = (CUBE_HI - CUBE_LO) / GRID
    c = CUBE_LO + (np.arange(GRID) + 0.5) * e
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], axis=1)


def occupancy(pose: np.ndarray, half_ext: np.ndarray) -> np.ndarray:
    """pose [W, K, 3, 4], half_ext [W, K, 3] -> [W, 512] in {0, 1}."""
    pose = np.asarray(pose, dtype=np.float64)
    half_ext = np.asarray(half_ext, dtype=np.float64)
    W, K = pose.shape[:2]
    cen = voxel_centres()
    half_edge = 0.5 * (CUBE_HI - CUBE_LO) / GRID
    out = np.zeros((W, GRID ** 3))
    for w in range(W):
        sd = np.full(cen.shape[0], np.inf)
        for k in range(K):
            d, _, _ = obb_signed_distance(cen, pose[w, k, :, :3], pose[w, k, :, 3], half_ext[w, k])
            sd = np.minimum(sd, d)
        out[w] = (sd <= half_edge).astype(np.float64)
    return out


def features(start: np.ndarray, goal: np.ndarray, occ: np.ndarray) -> np.ndarray:
    return np.concatenate([np.asarray(start, np.float64), np.asarray(goal, np.float64),
                           np.asarray(occ, np.float64)], axis=1)


def gelu(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d GELU / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


_erf_vec = np.vectorize(math.erf, otypes=[np.float64])


def _erf(x: np.ndarray) -> np.ndarray:
    return _erf_vec(x)


def forward(params: Dict[str, np.ndarray], x: np.ndarray, emulate: bool = False):
    """y [N, 1792] and the cache for backward: layer inputs a_l (as the GPU stores them) and
    pre-activations z_l."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    cache = {"a0": a}
    for l in range(1, 4):
        z = a @ r(params[f"W{l}"]) + params[f"b{l}"]
        cache[f"z{l}"] = z
        a = r(gelu(z))
        cache[f"a{l}"] = a
    y = a @ r(params["W4"]) + params["b4"]
    return y, cache


def straight_line(start: np.ndarray, goal: np.ndarray) -> np.ndarray:
    """[N, 32, 7]: start + (goal - start) * t / 31."""
    tau = np.arange(T_SEED, dtype=np.float64) / (T_SEED - 1)
    return start[:, None, :] + (goal - start)[:, None, :] * tau[None, :, None]


def seeds(y: np.ndarray, start: np.ndarray, goal: np.ndarray) -> np.ndarray:
    """[N, 8, 32, 7] seed trajectories: straight line + predicted deviation, endpoints pinned."""
    dev = np.asarray(y, np.float64).reshape(-1, N_SEEDS, T_SEED, N_J).copy()
    dev[:, :, 0, :] = 0.0
    dev[:, :, -1, :] = 0.0
    return straight_line(start, goal)[:, None] + dev


def loss(y: np.ndarray, targets: np.ndarray, valid: np.ndarray) -> Tuple[float, np.ndarray, np.ndarray]:
    """Min-over-slot loss.  y [N, 1792], targets [N, 8, 32, 7] (deviations from the straight
    line), valid [N, 8] in {0, 1}.  Returns (L, dL/dy [N, 1792], assignment [N, 8])."""
    N = y.shape[0]
    yp = np.asarray(y, np.float64).reshape(N, N_SEEDS, T_SEED * N_J)
    yt = np.asarray(targets, np.float64).reshape(N, N_SEEDS, T_SEED * N_J)
    e = np.mean((yp[:, :, None, :] - yt[:, None, :, :]) ** 2, axis=3)   # [N, slot s, target j]
    assign = np.argmin(e, axis=1)                                          # first minimum
    n_valid = float(np.sum(valid))
    if n_valid == 0:
        return 0.0, np.zeros_like(np.asarray(y, np.float64)), assign
    best = np.take_along_axis(e, assign[:, None, :], axis=1)[:, 0, :]
    L = float(np.sum(best * valid) / n_valid)
    dy = np.zeros_like(yp)
    coef = 2.0 / (T_SEED * N_J * n_valid)
    for n in range(N):
        for j in range(N_SEEDS):
            if valid[n, j]:
                s = assign[n, j]
                dy[n, s] += coef * (yp[n, s] - yt[n, j])
    return L, dy.reshape(N, -1), assign


def backward(params: Dict[str, np.ndarray], cache, dy: np.ndarray, emulate: bool = False) -> Dict[str, np.ndarray]:
    """Gradients of the loss w.r.t. every weight and bias (chain rule through the layers)."""
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    g = {}
    d = np.asarray(dy, np.float64)                   # dL/dy (FP32 on the GPU)
    for l in (4, 3, 2, 1):
        dq = r(d)                                     # the GEMM operand
        g[f"W{l}"] = cache[f"a{l - 1}"].T @ dq
        g[f"b{l}"] = np.sum(d, axis=0)
        if l > 1:
            dh = dq @ r(params[f"W{l}"]).T           # dL/d a_{l-1}
            d = dh * gelu_grad(cache[f"z{l - 1}"])   # dL/d z_{l-1}
    return g


def adam(params, grads, m, v, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = {}, {}, {}
    for k in params:
        mk = b1 * m[k] + (1.0 - b1) * grads[k]
        vk = b2 * v[k] + (1.0 - b2) * grads[k] ** 2
        mh = mk / (1.0 - b1 ** step)
        vh = vk / (1.0 - b2 ** step)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v
