"""Variable-precision trajectory-optimisation cost kernels for MI355X (gfx950).

The batched cost and gradient of trajectory optimisation -- serial-chain forward kinematics,
collision spheres against oriented cuboids and against each other, aggregation, the hand-written
adjoint, and the line-search + L-BFGS step -- run as HIP kernels behind the C ABI of
include/vapr.h, with the large intermediate tensors stored in per-tensor formats (FP32, FP16, BF16,
FP8 E4M3/E5M2, FP6 E3M2, FP4 E2M1).  This package is the Python binding.
"""
from ._lib import LIB_PATH, VaprError, load  # noqa: F401


def __getattr__(name):
    # the binding needs torch; import it lazily so `build` works without touching the GPU stack
    if name in ("Context", "Shape", "quantize", "dequantize", "precision_struct"):
        from . import context
        return getattr(context, name)
    if name in ("VaprCost", "trajectory_cost"):
        from . import cost
        return getattr(cost, name)
    if name in ("TrajectoryOptimizer", "PartitionedOptimizer"):
        from . import optim
        return getattr(optim, name)
    raise AttributeError(name)
