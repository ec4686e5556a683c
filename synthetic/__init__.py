"""Seeded synthetic workloads shared by the oracle tests, the GPU parity tests and the benchmark.

Only random inputs are drawn here: serial 7-joint arms with collision-sphere models, worlds of
oriented cuboids, joint configurations, seed trajectories, planning problems and the seeding
network's initial weights.  None of the method's arithmetic
(kinematics, distances, costs, gradients, number formats) lives in this package.
"""
from .generators import (  # noqa: F401
    MASTER_SEED,
    Robot,
    Worlds,
    Workload,
    make_robot,
    make_worlds,
    make_configs,
    make_trajectories,
    make_workload,
    WORKLOADS,
    SEEDNET_LAYERS,
    SeedProblems,
    make_seednet_params,
    make_seed_family,
    make_seed_problems,
    make_seed_inits,
)
