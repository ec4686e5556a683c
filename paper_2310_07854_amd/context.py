"""Python face of the library: a context owning the robot/world tables, plus thin wrappers of every
C entry point.  torch supplies device memory and the current stream; every step of the cost path
runs in the HIP kernels behind the C ABI.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, Mapping, Optional, Sequence, Tuple, Union

import numpy as np
import torch

from . import _lib as L

TENSORS = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad")
FormatSpec = Union[str, Tuple[str, int]]


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype: torch.dtype, what: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def _host(a, dtype) -> np.ndarray:
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass(frozen=True)
class Shape:
    """Batch shape of a cost evaluation: B = n_worlds * traj_per_world * n_ls * T."""

    n_worlds: int
    traj_per_world: int
    T: int
    n_ls: int = 1

    @property
    def n_traj(self) -> int:
        return self.n_worlds * self.traj_per_world

    @property
    def n_tc(self) -> int:
        return self.n_traj * self.n_ls

    @property
    def B(self) -> int:
        return self.n_tc * self.T

    def args(self):
        return (self.n_worlds, self.traj_per_world, self.T, self.n_ls)


STORED = TENSORS + ("swept_grad",)
SCALARS = ("self_cost", "bound_cost", "swept_cost", "pose_cost")


def precision_struct(spec: Mapping[str, FormatSpec], recompute_poses: bool = False) -> L.PrecisionC:
    p = L.PrecisionC()
    for name in STORED:
        v = spec.get(name, "f32")
        fmt, k = (v, 0) if isinstance(v, str) else v
        fid, e_bits, m_bits = L.format_id(fmt)
        setattr(p, name, L.TensorFormat(fid, int(k), e_bits, m_bits))
    p.recompute_poses = 1 if recompute_poses else 0
    return p


class Context:
    """One library context on a device.  Work is queued on torch's current stream at call time."""

    def __init__(self, device: int = 0):
        self._lib = L.load()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            L.check(self._lib.vapr_create(ctypes.byref(h), device, _stream_handle()))
        self._h = h
        self.n_spheres = 0
        # the library's defaults (eta as the FP32 value the kernels compare with)
        self.cost_params = {"eta": float(np.float32(0.02)), "w_coll": 100.0, "w_self": 100.0, "w_bound": 10.0,
                            "w_smooth": 1.0, "swept_steps": 0, "w_swept": 100.0, "w_goal_pos": 100.0,
                            "w_goal_rot": 10.0}
        self.precision: Dict[str, Tuple[str, int]] = {t: ("f32", 0) for t in STORED}
        self.recompute_poses = False
        # what was uploaded, for subset()
        self._robot = None
        self._worlds = None
        self._goals = None
        self._culling = True

    # -- lifetime ----------------------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.vapr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name: str, *args) -> None:
        fn = getattr(self._lib, name)
        self._lib.vapr_set_stream(self._h, _stream_handle())
        L.check(fn(self._h, *args), self._h)

    # -- setup ---------------------------------------------------------------------------------
    def set_robot(self, robot) -> None:
        """robot: object with fixed_tf [8,3,4], sphere_center [n_s,3], sphere_radius [n_s],
        sphere_link [n_s], pairs [P,2], q_lo [7], q_hi [7] (numpy or CPU tensors)."""
        fixed = _host(robot.fixed_tf, np.float32)
        centers = _host(robot.sphere_center, np.float32)
        radius = _host(robot.sphere_radius, np.float32)
        link = _host(robot.sphere_link, np.int32)
        pairs = _host(robot.pairs, np.int32).reshape(-1, 2)
        lo, hi = _host(robot.q_lo, np.float32), _host(robot.q_hi, np.float32)
        self._call("vapr_set_robot", 7, _ptr(fixed), int(radius.shape[0]), _ptr(centers), _ptr(radius), _ptr(link),
                   int(pairs.shape[0]), _ptr(pairs) if pairs.size else None, _ptr(lo), _ptr(hi))
        self.n_spheres = int(radius.shape[0])
        self._robot = robot

    def reach(self) -> Tuple[float, float]:
        """(link-pose bound, sphere-centre bound): the largest |value| any configuration stores in
        L and S, from the robot's translation lengths and sphere offsets."""
        lp, sp = ctypes.c_double(), ctypes.c_double()
        self._call("vapr_robot_reach", ctypes.byref(lp), ctypes.byref(sp))
        return lp.value, sp.value

    def set_worlds(self, pose, half_ext) -> None:
        pose = _host(pose, np.float32)
        half = _host(half_ext, np.float32)
        W, K = pose.shape[0], pose.shape[1]
        self._call("vapr_set_worlds", W, K, _ptr(pose) if pose.size else None, _ptr(half) if half.size else None)
        self._worlds = (pose, half)

    def set_precision(self, spec: Optional[Mapping[str, FormatSpec]] = None, recompute_poses: bool = False) -> None:
        spec = spec or {}
        p = precision_struct(spec, recompute_poses)
        self._call("vapr_set_precision", ctypes.byref(p))
        self.precision = {t: ((spec.get(t, "f32"), 0) if isinstance(spec.get(t, "f32"), str) else tuple(spec[t]))
                          for t in STORED}
        self.recompute_poses = recompute_poses

    def set_cost_params(self, eta=0.02, w_coll=100.0, w_self=100.0, w_bound=10.0, w_smooth=1.0,
                        swept_steps: int = 0, w_swept: float = 100.0, w_goal_pos: float = 100.0,
                        w_goal_rot: float = 10.0) -> None:
        """Cost weights; swept_steps > 0 turns on the swept term with that many samples per
        segment (the workspace then also holds the swept gradient and cost); the goal weights
        apply while goal poses are set."""
        p = L.CostParamsC(eta, w_coll, w_self, w_bound, w_smooth, int(swept_steps), w_swept, w_goal_pos, w_goal_rot)
        self._call("vapr_set_cost_params", ctypes.byref(p))
        self.cost_params = {"eta": float(p.eta), "w_coll": w_coll, "w_self": w_self, "w_bound": w_bound,
                            "w_smooth": w_smooth, "swept_steps": int(swept_steps), "w_swept": w_swept,
                            "w_goal_pos": w_goal_pos, "w_goal_rot": w_goal_rot}

    def set_goals(self, goals) -> None:
        """Goal poses of inverse kinematics, one per world: [n, 3, 4] row-major [R_g | p_g] of the
        end-effector link (None or n = 0 clears them)."""
        if goals is None:
            self._call("vapr_set_goals", 0, None)
            self._goals = None
            return
        g = _host(goals, np.float32).reshape(-1, 3, 4)
        self._call("vapr_set_goals", int(g.shape[0]), _ptr(g) if g.size else None)
        self._goals = g if g.size else None

    def set_culling(self, enable: bool) -> None:
        """Exact cuboid culling in the sphere-cost stage (on by default; results are identical)."""
        self._call("vapr_set_culling", 1 if enable else 0)
        self._culling = bool(enable)

    def subset(self, w0: int, w1: int) -> "Context":
        """A new context on the same device for worlds w0 .. w1 - 1 of this one: the same robot, cost
        parameters, precision, culling and (if set) those worlds' goal poses."""
        if self._robot is None or self._worlds is None:
            raise ValueError("subset needs the robot and worlds to be set")
        pose, half = self._worlds
        if not 0 <= w0 < w1 <= pose.shape[0]:
            raise ValueError(f"world range {w0}..{w1} outside 0..{pose.shape[0]}")
        c = Context(self.device)
        c.set_robot(self._robot)
        c.set_worlds(pose[w0:w1], half[w0:w1])
        c.set_cost_params(**self.cost_params)
        if self._goals is not None:
            c.set_goals(self._goals[w0:w1])
        if not self._culling:
            c.set_culling(False)
        c.set_precision({t: v for t, v in self.precision.items()}, self.recompute_poses)
        return c

    def culling_grid(self, world: int):
        """The culling grid of one world: (info dict, uint32 mask array [n^3, mask_words]), or
        (info, None) when culling is off or there are no cuboids."""
        info = L.GridInfoC()
        self._call("vapr_get_culling_grid", world, ctypes.byref(info), None, 0)
        d = {"n": info.n, "mask_words": info.mask_words, "origin": tuple(info.origin), "inv_cell": info.inv_cell}
        if info.n == 0:
            return d, None
        words = info.n ** 3 * info.mask_words
        out = np.empty(words, dtype=np.uint32)
        self._call("vapr_get_culling_grid", world, ctypes.byref(info), _ptr(out), words)
        return d, out.reshape(info.n ** 3, info.mask_words)

    # -- cost path -----------------------------------------------------------------------------
    def workspace_size(self, shape: Shape) -> int:
        n = ctypes.c_size_t()
        L.check(self._lib.vapr_workspace_size(self._h, *shape.args(), ctypes.byref(n)), self._h)
        return int(n.value)

    def new_workspace(self, shape: Shape) -> torch.Tensor:
        """A workspace for batches of this shape, announced to the library (vapr_ws_reset): memory
        torch hands out again never passes for the forward pass it held before."""
        ws = torch.empty(self.workspace_size(shape), dtype=torch.uint8, device=f"cuda:{self.device}")
        self.ws_reset(ws)
        return ws

    def ws_reset(self, ws: torch.Tensor) -> None:
        self._call("vapr_ws_reset", _dev(ws, torch.uint8, "ws"), ws.numel())

    def ws_poison(self, ws: torch.Tensor) -> None:
        """Fill the workspace (after its header) with 0xFF bytes and forget its forward pass."""
        self._call("vapr_ws_poison", _dev(ws, torch.uint8, "ws"), ws.numel())

    def census(self, name: str, ws: torch.Tensor, shape: Shape) -> Tuple[int, int]:
        """(codes at the largest finite magnitude, Inf/NaN codes) of a stored tensor."""
        out = (ctypes.c_int64 * 2)()
        self._call("vapr_ws_census", *shape.args(), _dev(ws, torch.uint8, "ws"), ws.numel(), L.TENSOR_IDS[name], out)
        return int(out[0]), int(out[1])

    def sync(self) -> None:
        """Wait for the context's work; raises VaprError (E_STATE) if a backward or optimiser kernel
        met a workspace that no longer held its forward pass."""
        self._call("vapr_sync")

    def cost_fwd(self, q: torch.Tensor, shape: Shape, ws: Optional[torch.Tensor] = None,
                 cost_traj: Optional[torch.Tensor] = None, cost_cfg: Optional[torch.Tensor] = None,
                 first: int = 1):
        """Trajectory-candidate costs [n_tc] float64 (and the workspace that holds the stored
        tensors).  first > 1 resumes from a stored stage (2: sphere costs, 3: aggregation)."""
        if ws is None:
            ws = self.new_workspace(shape)
        if cost_traj is None:
            cost_traj = torch.empty(shape.n_tc, dtype=torch.float64, device=q.device)
        if q.shape != (shape.B, 7):
            raise ValueError(f"q must be [{shape.B}, 7]")
        cfg_ptr = _dev(cost_cfg, torch.float32, "cost_cfg") if cost_cfg is not None else None
        self._call("vapr_cost_fwd_from", first, *shape.args(), _dev(q, torch.float32, "q"),
                   _dev(ws, torch.uint8, "ws"), ws.numel(), _dev(cost_traj, torch.float64, "cost_traj"), cfg_ptr)
        return cost_traj, ws

    def cost_bwd(self, q: torch.Tensor, ws: torch.Tensor, grad_cost_traj: Optional[torch.Tensor] = None,
                 grad_q: Optional[torch.Tensor] = None, want_grad: bool = True) -> Optional[torch.Tensor]:
        if want_grad and grad_q is None:
            grad_q = torch.empty_like(q)
        up = _dev(grad_cost_traj, torch.float64, "grad_cost_traj") if grad_cost_traj is not None else None
        gp = _dev(grad_q, torch.float32, "grad_q") if grad_q is not None else None
        self._call("vapr_cost_bwd", _dev(q, torch.float32, "q"), _dev(ws, torch.uint8, "ws"), ws.numel(), up, gp)
        return grad_q

    def collision_free(self, ws: torch.Tensor, shape: Shape) -> torch.Tensor:
        """[B] bool from the forward pass in ws: every sphere clears every cuboid, every self pair is
        apart and the joints are within their limits."""
        out = torch.empty(shape.B, dtype=torch.int32, device=ws.device)
        self._call("vapr_collision_free", *shape.args(), _dev(ws, torch.uint8, "ws"), ws.numel(), out.data_ptr())
        return out.bool()

    def cost_fwd_bwd_noalloc(self, q: torch.Tensor, shape: Shape, cost_traj: torch.Tensor, grad_q: torch.Tensor,
                             grad_cost_traj: Optional[torch.Tensor] = None,
                             cost_cfg: Optional[torch.Tensor] = None) -> None:
        """Forward + backward pass into caller-provided outputs, with the stored tensors in the
        library's static per-device workspace (no allocation; batches up to 64 MiB of workspace)."""
        if q.shape != (shape.B, 7) or grad_q.shape != (shape.B, 7):
            raise ValueError(f"q and grad_q must be [{shape.B}, 7]")
        up = _dev(grad_cost_traj, torch.float64, "grad_cost_traj") if grad_cost_traj is not None else None
        cfg = _dev(cost_cfg, torch.float32, "cost_cfg") if cost_cfg is not None else None
        self._call("vapr_cost_fwd_bwd_noalloc", *shape.args(), _dev(q, torch.float32, "q"), up,
                   _dev(cost_traj, torch.float64, "cost_traj"), cfg, _dev(grad_q, torch.float32, "grad_q"))

    # -- stored tensors --------------------------------------------------------------------------
    def tensor_count(self, name: str) -> int:
        return {"link_poses": 96, "sphere_pos": 3 * self.n_spheres, "sphere_dist": self.n_spheres,
                "sphere_grad": 3 * self.n_spheres, "joint_grad": 7, "self_cost": 1, "bound_cost": 1,
                "swept_grad": 3 * self.n_spheres, "swept_cost": 1, "pose_cost": 1}[name]

    def tensor_nbytes(self, name: str, shape: Shape) -> int:
        n = shape.B * self.tensor_count(name)
        if name in SCALARS:
            return 4 * n
        return packed_bytes(self.precision[name][0], n)

    def ws_export(self, name: str, ws: torch.Tensor, shape: Shape) -> torch.Tensor:
        """Packed codes (uint8) of a stored tensor in canonical order, or float32 for the scalars."""
        nb = self.tensor_nbytes(name, shape)
        out = torch.empty((nb + 3) // 4 * 4, dtype=torch.uint8, device=ws.device)
        self._call("vapr_ws_export", *shape.args(), _dev(ws, torch.uint8, "ws"), ws.numel(), L.TENSOR_IDS[name],
                   out.data_ptr(), out.numel())
        out = out[:nb]
        return out.view(torch.float32) if name in SCALARS else out

    def ws_import(self, name: str, ws: torch.Tensor, shape: Shape, data: torch.Tensor) -> None:
        data = data.contiguous()
        nb = data.numel() * data.element_size()
        buf = torch.zeros((nb + 3) // 4 * 4, dtype=torch.uint8, device=ws.device)
        buf[:nb] = data.view(torch.uint8).reshape(-1)
        self._call("vapr_ws_import", *shape.args(), _dev(ws, torch.uint8, "ws"), ws.numel(), L.TENSOR_IDS[name],
                   buf.data_ptr(), buf.numel())

    # -- per-kernel timing -----------------------------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        self._call("vapr_profile_enable", 1 if on else 0)

    def profile_read(self) -> Dict[str, Tuple[float, int]]:
        n = len(L.KERNEL_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._call("vapr_profile_read", ms, cnt, n)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.KERNEL_NAMES)}


def packed_bytes(fmt: str, n: int) -> int:
    """Bytes of n packed codes of a storage format or an emulated "eXmY" type."""
    lib = L.load()
    f, e_bits, m_bits = L.format_id(fmt)
    if f == L.EXMY:
        return int(lib.vapr_exmy_packed_bytes(e_bits, m_bits, n))
    return int(lib.vapr_packed_bytes(f, n))


def quantize_exmy(x: torch.Tensor, exp_bits: int, man_bits: int, scale_exp: int = 0) -> torch.Tensor:
    """Packed codes (uint8 tensor, floor(32 / b) codes to a 32-bit word) of float32 device tensor x
    in the emulated type E<exp_bits>M<man_bits>."""
    lib = L.load()
    n = x.numel()
    nb = int(lib.vapr_exmy_packed_bytes(exp_bits, man_bits, n))
    out = torch.empty(nb, dtype=torch.uint8, device=x.device)
    L.check(lib.vapr_quantize_exmy(exp_bits, man_bits, scale_exp, _dev(x, torch.float32, "x"), out.data_ptr(), n,
                                   _stream_handle()))
    return out


def dequantize_exmy(words: torch.Tensor, exp_bits: int, man_bits: int, n: int, scale_exp: int = 0) -> torch.Tensor:
    """float32 values of n packed codes of an emulated type (uint8 device tensor)."""
    lib = L.load()
    nb = int(lib.vapr_exmy_packed_bytes(exp_bits, man_bits, n))
    buf = words
    if words.numel() % 4 or words.data_ptr() % 4:
        buf = torch.zeros((nb + 3) // 4 * 4, dtype=torch.uint8, device=words.device)
        buf[:nb] = words[:nb]
    out = torch.empty(n, dtype=torch.float32, device=words.device)
    L.check(lib.vapr_dequantize_exmy(exp_bits, man_bits, scale_exp, _dev(buf, torch.uint8, "words"), out.data_ptr(),
                                     n, _stream_handle()))
    return out


def quantize(x: torch.Tensor, fmt: str, scale_exp: int = 0) -> torch.Tensor:
    """Packed codes (uint8 tensor) of float32 device tensor x in a storage format, or in an emulated
    "eXmY" type named by one that is not a storage format's name."""
    lib = L.load()
    f, e_bits, m_bits = L.format_id(fmt)
    if f == L.EXMY:
        return quantize_exmy(x, e_bits, m_bits, scale_exp)
    n = x.numel()
    nb = packed_bytes(fmt, n)
    out = torch.empty((nb + 3) // 4 * 4, dtype=torch.uint8, device=x.device)
    L.check(lib.vapr_quantize(f, scale_exp, _dev(x, torch.float32, "x"), out.data_ptr(), n, _stream_handle()))
    return out[:nb]


def round_exmy(x: torch.Tensor, exp_bits: int, man_bits: int, scale_exp: int = 0) -> torch.Tensor:
    """float32 device tensor x rounded to the emulated ExMy type (a new tensor)."""
    lib = L.load()
    out = torch.empty_like(x)
    L.check(lib.vapr_round_exmy(exp_bits, man_bits, scale_exp, _dev(x, torch.float32, "x"), out.data_ptr(), x.numel(),
                                _stream_handle()))
    return out


def dequantize(codes: torch.Tensor, fmt: str, n: int, scale_exp: int = 0) -> torch.Tensor:
    """float32 values of n packed codes (uint8 device tensor)."""
    lib = L.load()
    f, e_bits, m_bits = L.format_id(fmt)
    if f == L.EXMY:
        return dequantize_exmy(codes, e_bits, m_bits, n, scale_exp)
    nb = packed_bytes(fmt, n)
    buf = codes
    if codes.numel() % 4 or codes.data_ptr() % 4:
        buf = torch.zeros((nb + 3) // 4 * 4, dtype=torch.uint8, device=codes.device)
        buf[:nb] = codes[:nb]
    out = torch.empty(n, dtype=torch.float32, device=codes.device)
    L.check(lib.vapr_dequantize(f, scale_exp, _dev(buf, torch.uint8, "codes"), out.data_ptr(), n, _stream_handle()))
    return out
