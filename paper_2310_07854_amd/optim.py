"""Batched trajectory optimisation driver: parallel line search over N step scales and L-BFGS
(Sec. III-B steps (1)-(7)).  Each iteration is one forward + backward pass over all candidates
followed by the optimiser kernel; the only data the host touches are launch arguments."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .context import Context, Shape, _dev


class TrajectoryOptimizer:
    def __init__(self, vctx: Context, n_worlds: int, traj_per_world: int, T: int, n_ls: int = 4, m: int = 8,
                 max_step: float = 0.2, pin_ends: bool = True):
        """pin_ends: the first and last timestep stay fixed (trajectory optimisation); False lets
        every row move (inverse kinematics: T = 1, one seed per trajectory, goals set on the
        context)."""
        self.vctx = vctx
        self.shape1 = Shape(n_worlds, traj_per_world, T, 1)
        self.shape = Shape(n_worlds, traj_per_world, T, n_ls)
        self.m = m
        dev = f"cuda:{vctx.device}"
        n_traj, n = self.shape.n_traj, T * 7
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = torch.zeros(n_traj, n, **f32)
        self.g = torch.zeros(n_traj, n, **f32)
        self.d = torch.zeros(n_traj, n, **f32)
        self.cost = torch.zeros(n_traj, dtype=torch.float64, device=dev)
        self.s_hist = torch.zeros(n_traj, m, n, **f32)
        self.y_hist = torch.zeros(n_traj, m, n, **f32)
        self.rho = torch.zeros(n_traj, m, dtype=torch.float64, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        self.hist_len = torch.zeros(n_traj, **i32)
        self.hist_head = torch.zeros(n_traj, **i32)
        self.accepted = torch.zeros(n_traj, **i32)
        self.flags = torch.zeros(n_traj, **i32)
        self.q_cand = torch.zeros(self.shape.B, 7, **f32)
        self.cost_cand = torch.zeros(self.shape.n_tc, dtype=torch.float64, device=dev)
        self.ws = vctx.new_workspace(self.shape)
        self.ws1 = vctx.new_workspace(self.shape1)
        self._st = L.LbfgsStateC(n_traj, T, n_ls, m, max_step, *[t.data_ptr() for t in (
            self.x, self.g, self.d, self.cost, self.s_hist, self.y_hist, self.rho, self.hist_len, self.hist_head,
            self.accepted, self.flags)], 0 if pin_ends else 1)

    def init(self, x0: torch.Tensor) -> None:
        """Start from x0 [n_traj, T, 7] (with pin_ends, rows t=0 and t=T-1 are the fixed start and goal)."""
        self.x.copy_(x0.reshape(self.x.shape))
        q0 = self.x.reshape(-1, 7)
        c0, _ = self.vctx.cost_fwd(q0, self.shape1, ws=self.ws1)
        self.vctx.cost_bwd(q0, self.ws1, want_grad=False)
        self.vctx._call("vapr_optimizer_init", ctypes.byref(self._st), _dev(self.ws1, torch.uint8, "ws"),
                        self.ws1.numel(), _dev(c0, torch.float64, "cost0"), _dev(self.q_cand, torch.float32, "q"))

    def capture(self) -> None:
        """Record one iteration (forward, backward and optimiser kernels on the candidates) as a HIP
        graph; `replay` then runs it with one launch.  Call after `init` (which builds the
        library's lazy tables); the graph reads and writes this optimiser's buffers in place, so
        replays continue the same optimisation.  Changing the context's robot, worlds, precision or
        cost parameters afterwards needs a new capture."""
        torch.cuda.synchronize()
        self._graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self._graph):
            self.step()
        torch.cuda.synchronize()

    def replay(self) -> None:
        """One iteration by replaying the captured graph."""
        self._graph.replay()

    def step(self) -> None:
        """One iteration: evaluate all candidates (fwd + bwd), select, update, next candidates."""
        self.evaluate()
        self.update()

    def evaluate(self) -> None:
        """The iteration's forward and backward pass over every candidate."""
        self.vctx.cost_fwd(self.q_cand, self.shape, ws=self.ws, cost_traj=self.cost_cand)
        self.vctx.cost_bwd(self.q_cand, self.ws, want_grad=False)

    def update(self) -> None:
        """The iteration's line-search selection, L-BFGS update and next candidates."""
        self.vctx._call("vapr_optimizer_step", ctypes.byref(self._st), _dev(self.ws, torch.uint8, "ws"),
                        self.ws.numel(), _dev(self.cost_cand, torch.float64, "cost"),
                        _dev(self.q_cand, torch.float32, "q"))
