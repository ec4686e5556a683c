"""FP64 CPU oracle for the trajectory-optimisation cost and gradient path (TEST INFRASTRUCTURE).

This package is the slow, obviously-correct reference the GPU path is checked against.  Only the
test-suite, the entry point's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and it shares no code with the HIP kernels.

Modules
  formats    reference encoder/decoder of every storage format (Sec. IV-A, Sec. V-B)
  kinematics serial-chain forward kinematics and collision-sphere placement (Sec. II-B, Sec. III-B)
  geometry   oriented-cuboid signed distance and its gradient
  cost       world/self/bound costs, aggregation, the joint-space gradient two ways, and the
             whole fwd+bwd pass with quantisation emulated at the five stored tensors (Sec. III-C)
  optimizer  parallel line search + L-BFGS step (Sec. III-B, steps (1), (6), (7))

Parity status of each function is stated in its module header.
"""
