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


def split_worlds(n_worlds: int, parts: int):
    """Contiguous world ranges [(w0, w1), ...] for `parts` partitions (sizes differ by at most one;
    never more partitions than worlds)."""
    if n_worlds < 1 or parts < 1:
        raise ValueError("need at least one world and one partition")
    parts = min(parts, n_worlds)
    return [(p * n_worlds // parts, (p + 1) * n_worlds // parts) for p in range(parts)]


def streams_run_concurrently(streams, spin_cycles: int = 20_000_000) -> bool:
    """True when work queued on each stream runs while every other one is busy.  Streams that the
    runtime put on one hardware queue execute one after another, and partitions on them would
    lose what partitioning is for; this is checked by keeping one stream busy with a bounded spin
    kernel and seeing an event on each other stream complete before it."""
    for i, busy in enumerate(streams):
        done = torch.cuda.Event()
        with torch.cuda.stream(busy):
            torch.cuda._sleep(spin_cycles)
            done.record(busy)
        ok = True
        for j, s in enumerate(streams):
            if j == i:
                continue
            ev = torch.cuda.Event()
            ev.record(s)
            ev.synchronize()
            if done.query():  # the busy stream finished first: s waited behind it
                ok = False
        done.synchronize()
        if not ok:
            return False
    return True


def concurrent_streams(n: int, device: int = 0, attempts: int = 16):
    """n streams that run concurrently (see streams_run_concurrently), taking fresh ones from
    torch's pool until a set does; the last set drawn if none does within `attempts`."""
    streams = []
    for _ in range(attempts):
        streams = [torch.cuda.Stream(device=device) for _ in range(n)]
        if n < 2 or streams_run_concurrently(streams):
            break
    return streams


class PartitionedOptimizer:
    """The optimiser over a batch split by worlds into partitions, each with its own context and
    HIP stream.  Worlds are independent problems (every kernel works per configuration, per
    trajectory or per world), so the results are those of one TrajectoryOptimizer over the whole
    batch, bit for bit.  What changes is scheduling: with one stream, each of an iteration's five
    kernels drains before the next starts and the GPU idles in every drain; with a few streams
    running free, one partition's kernels fill the CUs that another's are leaving.  The streams
    are checked to run concurrently: two streams the runtime puts on one hardware queue run one
    after the other, which is slower than one stream.

    `step` queues each partition's iteration on its own stream and returns; `join` makes the
    caller's current stream wait for all of them (the properties below join first)."""

    def __init__(self, vctx: Context, n_worlds: int, traj_per_world: int, T: int, n_ls: int = 4, m: int = 8,
                 max_step: float = 0.2, pin_ends: bool = True, parts: int = 2):
        self.ranges = split_worlds(n_worlds, parts)
        self.traj_per_world = traj_per_world
        self.shape = Shape(n_worlds, traj_per_world, T, n_ls)
        self.parts = []
        streams = concurrent_streams(len(self.ranges), vctx.device)
        for (w0, w1), s in zip(self.ranges, streams):
            c = vctx.subset(w0, w1)
            with torch.cuda.stream(s):
                o = TrajectoryOptimizer(c, w1 - w0, traj_per_world, T, n_ls=n_ls, m=m, max_step=max_step,
                                        pin_ends=pin_ends)
            self.parts.append((c, s, o))

    def _follow_current(self) -> None:
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        for _, s, _ in self.parts:
            s.wait_event(ev)

    def init(self, x0: torch.Tensor) -> None:
        """Start from x0 [n_traj, T, 7] of the whole batch (see TrajectoryOptimizer.init)."""
        self._follow_current()
        for (w0, w1), (_, s, o) in zip(self.ranges, self.parts):
            with torch.cuda.stream(s):
                o.init(x0[w0 * self.traj_per_world:w1 * self.traj_per_world])

    def step(self) -> None:
        """One iteration of every partition, each queued on its own stream."""
        for _, s, o in self.parts:
            with torch.cuda.stream(s):
                o.step()

    def join(self) -> None:
        cur = torch.cuda.current_stream()
        for _, s, _ in self.parts:
            ev = torch.cuda.Event()
            ev.record(s)
            cur.wait_event(ev)

    def _cat(self, name: str) -> torch.Tensor:
        self.join()
        return torch.cat([getattr(o, name) for _, _, o in self.parts])

    @property
    def x(self) -> torch.Tensor:
        return self._cat("x")

    @property
    def cost(self) -> torch.Tensor:
        return self._cat("cost")

    @property
    def accepted(self) -> torch.Tensor:
        return self._cat("accepted")

    @property
    def flags(self) -> torch.Tensor:
        return self._cat("flags")

    def profile_enable(self, on: bool = True) -> None:
        for c, _, _ in self.parts:
            c.profile_enable(on)

    def profile_read(self):
        """Per-kernel (total ms, launches) summed over the partitions."""
        out = {}
        for c, _, _ in self.parts:
            for k, (ms, n) in c.profile_read().items():
                a, b = out.get(k, (0.0, 0))
                out[k] = (a + ms, b + n)
        return out

    def close(self) -> None:
        torch.cuda.synchronize()
        for c, _, _ in self.parts:
            c.close()
        self.parts = []
