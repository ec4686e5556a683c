"""ctypes declarations of the C ABI in include/vapr.h.  Argument marshalling only.

Loading fails loudly when libvapr.so has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import re
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvapr.so")

# status codes and enums mirror include/vapr.h
OK, E_INVALID, E_OOM, E_HIP, E_UNSUPPORTED, E_STATE = range(6)
F32, F16, BF16, E4M3, E5M2, E3M2, E2M1 = range(7)
FORMAT_IDS = {"f32": F32, "f16": F16, "bf16": BF16, "e4m3": E4M3, "e5m2": E5M2, "e3m2": E3M2, "e2m1": E2M1}
EXMY = 7  # an emulated ExMy type: any other "eXmY" format name


def format_id(fmt: str):
    """(format id, exponent bits, mantissa bits) of a format name: a storage format, or an emulated
    "eXmY" type (1 <= X <= 8, 0 <= Y <= 23)."""
    if fmt in FORMAT_IDS:
        return FORMAT_IDS[fmt], 0, 0
    m = re.fullmatch(r"e(\d+)m(\d+)", fmt)
    if not m:
        raise ValueError(f"unknown format {fmt!r}")
    return EXMY, int(m.group(1)), int(m.group(2))
FORMAT_BITS = {F32: 32, F16: 16, BF16: 16, E4M3: 8, E5M2: 8, E3M2: 6, E2M1: 4}
T_LINK_POSES, T_SPHERE_POS, T_SPHERE_DIST, T_SPHERE_GRAD, T_JOINT_GRAD, T_SELF_COST, T_BOUND_COST = range(7)
ABI_VERSION = 4  # the structs below match include/vapr.h at this version
TENSOR_IDS = {"link_poses": 0, "sphere_pos": 1, "sphere_dist": 2, "sphere_grad": 3, "joint_grad": 4,
              "self_cost": 5, "bound_cost": 6, "swept_grad": 7, "swept_cost": 8,
              "pose_cost": 9}
KERNEL_NAMES = ("fk", "sphere_cost", "reduce", "adjoint", "optimizer", "codec", "repack", "swept")


class VaprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vapr status {status}: {msg}")
        self.status = status


class TensorFormat(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("scale_exp", ctypes.c_int32), ("exp_bits", ctypes.c_int32),
                ("man_bits", ctypes.c_int32)]


class PrecisionC(ctypes.Structure):
    _fields_ = [("link_poses", TensorFormat), ("sphere_pos", TensorFormat), ("sphere_dist", TensorFormat),
                ("sphere_grad", TensorFormat), ("joint_grad", TensorFormat), ("recompute_poses", ctypes.c_int32),
                ("swept_grad", TensorFormat)]


class CostParamsC(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_float), ("w_coll", ctypes.c_float), ("w_self", ctypes.c_float),
                ("w_bound", ctypes.c_float), ("w_smooth", ctypes.c_float), ("swept_steps", ctypes.c_int32),
                ("w_swept", ctypes.c_float), ("w_goal_pos", ctypes.c_float), ("w_goal_rot", ctypes.c_float)]


class GridInfoC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mask_words", ctypes.c_int32), ("origin", ctypes.c_float * 3),
                ("inv_cell", ctypes.c_float)]


class LbfgsStateC(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("T", ctypes.c_int32), ("n_ls", ctypes.c_int32), ("m", ctypes.c_int32),
                ("max_step", ctypes.c_float), ("x", ctypes.c_void_p), ("g", ctypes.c_void_p), ("d", ctypes.c_void_p), ("cost", ctypes.c_void_p),
                ("s_hist", ctypes.c_void_p), ("y_hist", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("hist_len", ctypes.c_void_p), ("hist_head", ctypes.c_void_p), ("accepted", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("free_ends", ctypes.c_int32)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "vapr_abi_version": (_I, []),
    "vapr_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "vapr_destroy": (_I, [_P]),
    "vapr_set_stream": (_I, [_P, _P]),
    "vapr_set_robot": (_I, [_P, _I, _P, _I, _P, _P, _P, _I, _P, _P, _P]),
    "vapr_set_worlds": (_I, [_P, _I, _I, _P, _P]),
    "vapr_robot_reach": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "vapr_set_goals": (_I, [_P, _I, _P]),
    "vapr_round_exmy": (_I, [_I, _I, _I, _P, _P, _I64, _P]),
    "vapr_set_precision": (_I, [_P, ctypes.POINTER(PrecisionC)]),
    "vapr_get_precision": (_I, [_P, ctypes.POINTER(PrecisionC)]),
    "vapr_set_cost_params": (_I, [_P, ctypes.POINTER(CostParamsC)]),
    "vapr_set_culling": (_I, [_P, _I]),
    "vapr_get_culling_grid": (_I, [_P, _I, ctypes.POINTER(GridInfoC), _P, _SZ]),
    "vapr_workspace_size": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(_SZ)]),
    "vapr_ws_reset": (_I, [_P, _P, _SZ]),
    "vapr_sync": (_I, [_P]),
    "vapr_collision_free": (_I, [_P, _I, _I, _I, _I, _P, _SZ, _P]),
    "vapr_seed_deviations": (_I, [_I, _I, _P, _P, _P, _P, _P]),
    "vapr_cost_fwd": (_I, [_P, _I, _I, _I, _I, _P, _P, _SZ, _P, _P]),
    "vapr_cost_fwd_from": (_I, [_P, _I, _I, _I, _I, _I, _P, _P, _SZ, _P, _P]),
    "vapr_cost_bwd": (_I, [_P, _P, _P, _SZ, _P, _P]),
    "vapr_cost_fwd_bwd_noalloc": (_I, [_P, _I, _I, _I, _I, _P, _P, _P, _P, _P]),
    "vapr_optimizer_init": (_I, [_P, ctypes.POINTER(LbfgsStateC), _P, _SZ, _P, _P]),
    "vapr_optimizer_step": (_I, [_P, ctypes.POINTER(LbfgsStateC), _P, _SZ, _P, _P]),
    "vapr_quantize": (_I, [_I, _I, _P, _P, _I64, _P]),
    "vapr_dequantize": (_I, [_I, _I, _P, _P, _I64, _P]),
    "vapr_packed_bytes": (_SZ, [_I, _I64]),
    "vapr_ws_poison": (_I, [_P, _P, _SZ]),
    "vapr_ws_census": (_I, [_P, _I, _I, _I, _I, _P, _SZ, _I, _P]),
    "vapr_exmy_packed_bytes": (_SZ, [_I, _I, _I64]),
    "vapr_quantize_exmy": (_I, [_I, _I, _I, _P, _P, _I64, _P]),
    "vapr_dequantize_exmy": (_I, [_I, _I, _I, _P, _P, _I64, _P]),
    "vapr_ws_export": (_I, [_P, _I, _I, _I, _I, _P, _SZ, _I, _P, _SZ]),
    "vapr_ws_import": (_I, [_P, _I, _I, _I, _I, _P, _SZ, _I, _P, _SZ]),
    "vapr_profile_enable": (_I, [_P, _I]),
    "vapr_profile_read": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), _I]),
    "vapr_seed_occupancy": (_I, [_I, _I, _P, _P, _P, _P]),
    "vapr_seed_features": (_I, [_I, _P, _P, _P, _P, _P]),
    "vapr_seed_trajectories": (_I, [_I, _P, _P, _P, _P, _P]),
    "vapr_gemm_bf16": (_I, [_I, _I, _I, _P, _I64, _I64, _P, _I64, _I64, _P, _I, _P, _P, _P, _I64, _P]),
    "vapr_seed_head": (_I, [_I, _P, _I64, _P, _P, _P, _P, _P, _P]),
    "vapr_seed_loss": (_I, [_I, _P, _P, _P, _I, _P, _P, _P, _P, _P]),
    "vapr_column_sum": (_I, [_I, _I, _P, _I64, _P, _P]),
    "vapr_adam": (_I, [_I64, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _I,
                       _P]),
    "vapr_status_string": (ctypes.c_char_p, [_I]),
    "vapr_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load(path: str = None) -> ctypes.CDLL:
    """The loaded library (VAPR_LIB names another build of it, e.g. libvapr_ubsan.so); raises if it
    has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("VAPR_LIB") or LIB_PATH
    # torch brings its own HIP runtime; loading it first makes this library bind to the same one
    # (two runtimes in one process do not share devices or streams)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2310_07854_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.vapr_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} implements ABI {lib.vapr_abi_version()}, these bindings ABI {ABI_VERSION}; "
                          "rebuild it")
    _lib = lib
    return lib


def check(status: int, ctx=None) -> None:
    if status != OK:
        lib = load()
        msg = lib.vapr_last_error(ctx).decode()
        raise VaprError(status, msg or lib.vapr_status_string(status).decode())
