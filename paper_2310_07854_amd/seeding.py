"""Learned trajectory seeder: binding over libvapr's seeder kernels (argument marshalling only).

A network proposes initial trajectories for the optimiser in place of the geometric planner
(Sec. II-A, III-B; Sec. VI-B: better seeding cuts planning attempts):
x = [start (7), goal (7), 8x8x8 occupancy (512)] -> 3 x (256, GELU) -> 8 seeds x 32 timesteps x 7
joints, read as deviations from the straight line.  Weights are BF16 operands of the matrix cores
(FP32 accumulation); the master weights, gradients and Adam moments are FP32 in one flat buffer
each, so that one Adam launch updates every tensor.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import _lib as L
from .context import _dev, _stream_handle

N_J, N_SEEDS, T_SEED = 7, 8, 32
N_VOX = 512
N_IN, N_IN_PAD, N_HID = 2 * N_J + N_VOX, 544, 256
N_TRAJ = T_SEED * N_J
N_OUT = N_SEEDS * N_TRAJ
# stored shapes (W1 padded to 544 rows; the padding rows stay zero)
SHAPES = (("W1", (N_IN_PAD, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_OUT)), ("b4", (N_OUT,)))
PLAIN, GELU, GELU_GRAD = 0, 1, 2


def _call(name, *args):
    L.check(getattr(L.load(), name)(*args))


def _p(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def occupancy(pose: torch.Tensor, half_ext: torch.Tensor) -> torch.Tensor:
    """[W, 512] float32 occupancy of the 1.5 m cube for device tensors pose [W, K, 3, 4] and
    half_ext [W, K, 3]."""
    W, K = pose.shape[0], pose.shape[1]
    occ = torch.empty(W, N_VOX, dtype=torch.float32, device=pose.device)
    _call("vapr_seed_occupancy", W, K, _dev(pose, torch.float32, "pose") if K else None,
          _dev(half_ext, torch.float32, "half_ext") if K else None, occ.data_ptr(), _stream_handle())
    return occ


def features(start: torch.Tensor, goal: torch.Tensor, occ: torch.Tensor) -> torch.Tensor:
    """Network input rows [n, 544] bfloat16."""
    n = start.shape[0]
    x = torch.empty(n, N_IN_PAD, dtype=torch.bfloat16, device=start.device)
    _call("vapr_seed_features", n, _dev(start, torch.float32, "start"), _dev(goal, torch.float32, "goal"),
          _dev(occ, torch.float32, "occ"), x.data_ptr(), _stream_handle())
    return x


def gemm(A: torch.Tensor, a_ms: int, a_ks: int, B: torch.Tensor, b_ks: int, b_ns: int, M: int, N: int, K: int,
         bias: Optional[torch.Tensor] = None, epilogue: int = PLAIN, aux: Optional[torch.Tensor] = None,
         C: Optional[torch.Tensor] = None, C16: Optional[torch.Tensor] = None, ldc: Optional[int] = None) -> None:
    """Z = A B (+ bias) with A(m, k) = A[m * a_ms + k * a_ks], B(k, n) = B[k * b_ks + n * b_ns]
    (BF16 tensors), written through the chosen epilogue to C (FP32) and/or C16 (BF16)."""
    assert A.dtype == torch.bfloat16 and B.dtype == torch.bfloat16
    _call("vapr_gemm_bf16", M, N, K, A.data_ptr(), a_ms, a_ks, B.data_ptr(), b_ks, b_ns, _p(bias), epilogue,
          _p(aux), _p(C), _p(C16), N if ldc is None else ldc, _stream_handle())


def to_bf16(x: torch.Tensor) -> torch.Tensor:
    """Round-to-nearest-even BF16 copy of a float32 device tensor (the library's codec)."""
    from .context import quantize
    return quantize(x.contiguous(), "bf16").view(torch.bfloat16).reshape(x.shape)


def column_sum(X: torch.Tensor, out: torch.Tensor) -> None:
    """out[n] = sum_m X[m, n] for a float32 device matrix whose rows may be strided (unit column stride)."""
    M, N = X.shape
    if not X.is_cuda or X.dtype != torch.float32 or X.stride(1) != 1:
        raise ValueError("X must be a float32 device matrix with unit column stride")
    _call("vapr_column_sum", M, N, X.data_ptr(), X.stride(0), _dev(out, torch.float32, "out"), _stream_handle())


def deviations(traj: torch.Tensor, start: torch.Tensor, goal: torch.Tensor) -> torch.Tensor:
    """Deviations [n, m, 32, 7] of trajectories traj [n, m, 32, 7] from the straight line between
    start and goal [n, 7] (the inverse of `trajectories`)."""
    n, m = traj.shape[0], traj.shape[1]
    if traj.shape[2:] != (T_SEED, N_J):
        raise ValueError(f"trajectories must be [n, m, {T_SEED}, {N_J}]")
    out = torch.empty_like(traj)
    _call("vapr_seed_deviations", n, m, _dev(traj, torch.float32, "traj"), _dev(start, torch.float32, "start"),
          _dev(goal, torch.float32, "goal"), out.data_ptr(), _stream_handle())
    return out


def trajectories(y: torch.Tensor, start: torch.Tensor, goal: torch.Tensor) -> torch.Tensor:
    """[n, 8, 32, 7] seeds: straight line plus the predicted deviation, endpoints exact."""
    n = y.shape[0]
    out = torch.empty(n, N_SEEDS, T_SEED, N_J, dtype=torch.float32, device=y.device)
    _call("vapr_seed_trajectories", n, _dev(y, torch.float32, "y"), _dev(start, torch.float32, "start"),
          _dev(goal, torch.float32, "goal"), out.data_ptr(), _stream_handle())
    return out


class SeedNet:
    """The seeding network's parameters and training state on one device."""

    def __init__(self, params: Dict[str, np.ndarray], device: str = "cuda:0"):
        self.offsets = {}
        o = 0
        for name, shape in SHAPES:
            self.offsets[name] = (o, shape)
            o += int(np.prod(shape))
        self.n_params = o
        f32 = dict(dtype=torch.float32, device=device)
        self.w = torch.zeros(o, **f32)
        self.g = torch.zeros(o, **f32)
        self.m = torch.zeros(o, **f32)
        self.v = torch.zeros(o, **f32)
        for name, (off, shape) in self.offsets.items():
            src = torch.tensor(np.asarray(params[name], dtype=np.float32), device=device)
            if name == "W1":
                self.view(self.w, name)[:src.shape[0]].copy_(src)
            else:
                self.view(self.w, name).copy_(src.reshape(shape))
        self.w16 = to_bf16(self.w)
        self.step = 0

    def view(self, buf: torch.Tensor, name: str) -> torch.Tensor:
        off, shape = self.offsets[name]
        return buf[off:off + int(np.prod(shape))].view(shape)

    def params(self) -> Dict[str, np.ndarray]:
        """Current FP32 weights on the host (W1 without its padding rows)."""
        out = {name: self.view(self.w, name).cpu().numpy().astype(np.float64) for name, _ in SHAPES}
        out["W1"] = out["W1"][:N_IN]
        return out

    def forward(self, x: torch.Tensor, train: bool = True) -> Tuple[torch.Tensor, dict]:
        """y [n, 1792] float32 for input rows x [n, 544] bfloat16 (n a multiple of 32 for training,
        any n >= 1 for inference), and the activations backward needs (train=False keeps none and
        skips writing the pre-activations)."""
        n = x.shape[0]
        dev = x.device
        cache = {"a0": x}
        a = x
        k = N_IN_PAD
        for l in (1, 2, 3):
            z = torch.empty(n, N_HID, dtype=torch.float32, device=dev) if train else None
            a_next = torch.empty(n, N_HID, dtype=torch.bfloat16, device=dev)
            gemm(a, k, 1, self.view(self.w16, f"W{l}"), N_HID, 1, n, N_HID, k, bias=self.view(self.w, f"b{l}"),
                 epilogue=GELU, aux=z, C16=a_next)
            cache[f"z{l}"], cache[f"a{l}"] = z, a_next
            a, k = a_next, N_HID
        y = torch.empty(n, N_OUT, dtype=torch.float32, device=dev)
        gemm(a, N_HID, 1, self.view(self.w16, "W4"), N_OUT, 1, n, N_OUT, N_HID, bias=self.view(self.w, "b4"), C=y)
        return y, cache

    def backward(self, cache: dict, dy: torch.Tensor) -> None:
        """Gradients of every weight and bias into self.g (n a multiple of 32)."""
        n = dy.shape[0]
        dev = dy.device
        d = dy
        d16 = to_bf16(d)
        width = {1: N_IN_PAD, 2: N_HID, 3: N_HID, 4: N_HID}
        out_w = {1: N_HID, 2: N_HID, 3: N_HID, 4: N_OUT}
        for l in (4, 3, 2, 1):
            a_prev = cache[f"a{l - 1}"]
            # dW_l = a_{l-1}^T d16: A(m, k) = a_{l-1}[k][m]
            gemm(a_prev, 1, width[l], d16, out_w[l], 1, width[l], out_w[l], n, C=self.view(self.g, f"W{l}"))
            column_sum(d, self.view(self.g, f"b{l}"))
            if l > 1:
                # dz_{l-1} = (d16 W_l^T) * GELU'(z_{l-1}): B(k, j) = W_l[j][k]
                dz = torch.empty(n, N_HID, dtype=torch.float32, device=dev)
                dz16 = torch.empty(n, N_HID, dtype=torch.bfloat16, device=dev)
                gemm(d16, out_w[l], 1, self.view(self.w16, f"W{l}"), 1, out_w[l], n, N_HID, out_w[l],
                     epilogue=GELU_GRAD, aux=cache[f"z{l - 1}"], C=dz, C16=dz16)
                d, d16 = dz, dz16

    def loss(self, y: torch.Tensor, targets: torch.Tensor, valid: torch.Tensor, n_valid: int):
        """(loss [1] float64, dL/dy [n, 1792], assignment [n, 8]) of the min-over-slot matching."""
        n = y.shape[0]
        dev = y.device
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        dy = torch.empty_like(y)
        assign = torch.empty(n, N_SEEDS, dtype=torch.int32, device=dev)
        partial = torch.empty(n, dtype=torch.float64, device=dev)
        _call("vapr_seed_loss", n, _dev(y, torch.float32, "y"), _dev(targets, torch.float32, "targets"),
              _dev(valid, torch.float32, "valid"), int(n_valid), loss.data_ptr(), assign.data_ptr(), dy.data_ptr(),
              partial.data_ptr(), _stream_handle())
        return loss, dy, assign

    def adam(self, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
        self.step += 1
        _call("vapr_adam", self.n_params, self.w.data_ptr(), self.w16.data_ptr(), self.g.data_ptr(),
              self.m.data_ptr(), self.v.data_ptr(), ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2),
              ctypes.c_float(eps), self.step, _stream_handle())

    def train_step(self, x: torch.Tensor, targets: torch.Tensor, valid: torch.Tensor, n_valid: int,
                   lr: float = 1e-3) -> torch.Tensor:
        """One Adam step on a batch; returns the batch loss (device float64 [1])."""
        y, cache = self.forward(x)
        loss, dy, _ = self.loss(y, targets, valid, n_valid)
        self.backward(cache, dy)
        self.adam(lr)
        return loss

    def hidden(self, x: torch.Tensor) -> torch.Tensor:
        """The last hidden layer [n, 256] bfloat16 for input rows x [n, 544] (inference)."""
        n = x.shape[0]
        a, k = x, N_IN_PAD
        for l in (1, 2, 3):
            a_next = torch.empty(n, N_HID, dtype=torch.bfloat16, device=x.device)
            gemm(a, k, 1, self.view(self.w16, f"W{l}"), N_HID, 1, n, N_HID, k, bias=self.view(self.w, f"b{l}"),
                 epilogue=GELU, C16=a_next)
            a, k = a_next, N_HID
        return a

    def head(self, a3: torch.Tensor, start: torch.Tensor, goal: torch.Tensor) -> torch.Tensor:
        """Output layer fused with trajectory construction: [n, 8, 32, 7] seeds from a3 [n, 256]."""
        n = a3.shape[0]
        assert a3.dtype == torch.bfloat16 and a3.is_cuda and a3.stride(1) == 1
        out = torch.empty(n, N_SEEDS, T_SEED, N_J, dtype=torch.float32, device=a3.device)
        _call("vapr_seed_head", n, a3.data_ptr(), a3.stride(0), self.view(self.w16, "W4").data_ptr(),
              self.view(self.w, "b4").data_ptr(), _dev(start, torch.float32, "start"),
              _dev(goal, torch.float32, "goal"), out.data_ptr(), _stream_handle())
        return out

    def seeds(self, start: torch.Tensor, goal: torch.Tensor, occ: torch.Tensor) -> torch.Tensor:
        """[n, 8, 32, 7] seed trajectories for problems (start, goal [n, 7], occ [n, 512])."""
        return self.head(self.hidden(features(start, goal, occ)), start, goal)
