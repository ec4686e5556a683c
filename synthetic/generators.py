"""Seeded generators for the synthetic stand-ins of the paper's planning problems.

The paper evaluates on a public motion-planning benchmark with a 7-DOF manipulator (Sec. I,
Sec. III-A); neither the robot model nor the benchmark scenes are available, so every workload is
drawn here from a fixed master seed.  Recipe (all lengths in metres, angles in radians):

* Arm: 7 revolute joints, joint j turns about the local z axis after a fixed transform F_j; an 8th
  fixed transform F_8 carries the end link.  Each F_j has a rotation uniform on SO(3) (Shoemake's
  unit-quaternion construction) and a translation l*u with l ~ U[0.05, 0.35] and u uniform on the
  unit sphere.  Joint limits are +-2.9.
* Spheres: n_s spheres are dealt round-robin over the 9 links 0..8 and then listed in link order.
  A sphere on link l < 8 sits at lambda*t_{l+1} + N(0, 0.01^2 I) with lambda ~ U[0, 1], where t_{l+1}
  is the translation of F_{l+1} (so it lies along the segment to the next joint); a sphere on the
  end link is uniform in a 0.1 m ball.  Radii ~ U[0.03, 0.08].
* Self-collision pairs: a seeded sample of P pairs (a < b) among all sphere pairs whose links differ
  by at least two, sorted lexicographically.
* Worlds: K cuboids per world with centres ~ U[-0.75, 0.75]^3, side lengths ~ U[0.05, 0.5] (half
  extents are half of that) and rotations uniform on SO(3).
* Configurations: joint angles ~ U[-2.8, 2.8]^7, independent per configuration.
* Seed trajectories: each world holds one problem (start, goal ~ U[-2.8, 2.8]^7); seed s of that
  problem is the straight start->goal interpolation over T steps plus a bump
  sin(pi t/(T-1)) * delta_s with delta_0 = 0 and delta_s ~ U[-1, 1]^7 otherwise.

Every array is produced in float64 and, unless `exact=True`, rounded to float32 and widened back, so
the oracle (float64) and the GPU path (float32) consume bit-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Tuple

import numpy as np

MASTER_SEED = 2310_07854
N_JOINTS = 7
N_LINKS = N_JOINTS + 2  # link 0 (base) .. link 8 (end link)
JOINT_LIMIT = 2.9
Q_RANGE = 2.8

# independent random streams split off the master seed
_STREAMS = ("robot", "worlds", "configs", "trajectories", "calibration", "seednet", "seed_problems", "seed_inits",
            "seed_family")


def _rng(seed: int, stream: str) -> np.random.Generator:
    children = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return np.random.default_rng(children[_STREAMS.index(stream)])


def _as_inputs(a: np.ndarray, exact: bool) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    return a if exact else a.astype(np.float32).astype(np.float64)


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform rotations from Shoemake's unit-quaternion construction."""
    u1, u2, u3 = rng.random((3, n))
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    z, w = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@dataclass
class Robot:
    """Serial arm + sphere model.  `fixed_tf[j-1]` is F_j (3x4, rows [R | t]) for j = 1..8."""

    fixed_tf: np.ndarray      # [8, 3, 4]
    sphere_center: np.ndarray  # [n_s, 3] in the frame of the sphere's link
    sphere_radius: np.ndarray  # [n_s]
    sphere_link: np.ndarray    # [n_s] int32, non-decreasing, in 0..8
    pairs: np.ndarray          # [P, 2] int32, a < b, sorted
    q_lo: np.ndarray           # [7]
    q_hi: np.ndarray           # [7]

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_radius.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.pairs.shape[0])


@dataclass
class Worlds:
    """`pose[w, k]` is the 3x4 world<-box transform [R | c]; `half_ext[w, k]` the half side lengths."""

    pose: np.ndarray      # [W, K, 3, 4]
    half_ext: np.ndarray  # [W, K, 3]

    @property
    def n_worlds(self) -> int:
        return int(self.pose.shape[0])

    @property
    def n_cuboids(self) -> int:
        return int(self.pose.shape[1])


def sphere_counts(n_spheres: int, n_links: int = N_LINKS) -> np.ndarray:
    """Round-robin deal of n_spheres over the links: the first (n_s mod n_links) links get one more."""
    base, extra = divmod(n_spheres, n_links)
    return np.array([base + (1 if l < extra else 0) for l in range(n_links)], dtype=np.int64)


def make_robot(n_spheres: int = 60, n_pairs: int = 300, seed: int = MASTER_SEED,
               exact: bool = False) -> Robot:
    rng = _rng(seed, "robot")
    n_fixed = N_JOINTS + 1
    R = _random_rotations(rng, n_fixed)
    length = rng.uniform(0.05, 0.35, size=n_fixed)
    t = _unit_vectors(rng, n_fixed) * length[:, None]
    fixed = np.concatenate([R, t[:, :, None]], axis=2)

    counts = sphere_counts(n_spheres)
    link = np.repeat(np.arange(N_LINKS), counts).astype(np.int32)
    centers = np.empty((n_spheres, 3))
    for s, l in enumerate(link):
        if l < N_LINKS - 1:
            lam = rng.uniform(0.0, 1.0)
            centers[s] = lam * t[l] + rng.normal(0.0, 0.01, size=3)
        else:
            while True:  # rejection sample of the 0.1 m ball
                v = rng.uniform(-0.1, 0.1, size=3)
                if v @ v <= 0.01:
                    centers[s] = v
                    break
    radius = rng.uniform(0.03, 0.08, size=n_spheres)

    eligible = [(a, b) for a in range(n_spheres) for b in range(a + 1, n_spheres)
                if abs(int(link[a]) - int(link[b])) >= 2]
    if n_pairs > len(eligible):
        raise ValueError(f"only {len(eligible)} eligible pairs for {n_pairs} requested")
    pick = rng.choice(len(eligible), size=n_pairs, replace=False)
    pairs = np.array(sorted(eligible[i] for i in pick), dtype=np.int32).reshape(n_pairs, 2)

    return Robot(
        fixed_tf=_as_inputs(fixed, exact),
        sphere_center=_as_inputs(centers, exact),
        sphere_radius=_as_inputs(radius, exact),
        sphere_link=link,
        pairs=pairs,
        q_lo=np.full(N_JOINTS, -JOINT_LIMIT),
        q_hi=np.full(N_JOINTS, JOINT_LIMIT),
    )


def make_worlds(n_worlds: int, n_cuboids: int, seed: int = MASTER_SEED, exact: bool = False) -> Worlds:
    rng = _rng(seed, "worlds")
    n = n_worlds * n_cuboids
    R = _random_rotations(rng, n)
    c = rng.uniform(-0.75, 0.75, size=(n, 3))
    h = 0.5 * rng.uniform(0.05, 0.5, size=(n, 3))
    pose = np.concatenate([R, c[:, :, None]], axis=2).reshape(n_worlds, n_cuboids, 3, 4)
    return Worlds(pose=_as_inputs(pose, exact), half_ext=_as_inputs(h.reshape(n_worlds, n_cuboids, 3), exact))


def make_configs(n: int, seed: int = MASTER_SEED, lo: float = -Q_RANGE, hi: float = Q_RANGE,
                 exact: bool = False) -> np.ndarray:
    """Independent joint configurations [n, 7]."""
    rng = _rng(seed, "configs")
    return _as_inputs(rng.uniform(lo, hi, size=(n, N_JOINTS)), exact)


def make_trajectories(n_worlds: int, traj_per_world: int, T: int, seed: int = MASTER_SEED,
                      exact: bool = False) -> np.ndarray:
    """Seed trajectories [n_worlds, traj_per_world, T, 7]; row t=0 is the start, t=T-1 the goal."""
    rng = _rng(seed, "trajectories")
    start = rng.uniform(-Q_RANGE, Q_RANGE, size=(n_worlds, 1, 1, N_JOINTS))
    goal = rng.uniform(-Q_RANGE, Q_RANGE, size=(n_worlds, 1, 1, N_JOINTS))
    delta = rng.uniform(-1.0, 1.0, size=(n_worlds, traj_per_world, 1, N_JOINTS))
    delta[:, 0] = 0.0
    tau = np.linspace(0.0, 1.0, T).reshape(1, 1, T, 1)
    bump = np.sin(np.pi * tau)
    q = start + tau * (goal - start) + bump * delta
    q[:, :, 0] = start[:, :, 0]
    q[:, :, -1] = goal[:, :, 0]
    return _as_inputs(q, exact)


@dataclass
class Workload:
    """One synthetic workload: shapes follow the configuration layout
    b = ((traj * n_ls + candidate) * T + t), traj = world * traj_per_world + seed."""

    name: str
    robot: Robot
    worlds: Worlds
    traj_per_world: int
    T: int
    n_ls: int
    q: np.ndarray = field(repr=False)  # [B, 7]

    @property
    def n_worlds(self) -> int:
        return self.worlds.n_worlds

    @property
    def n_traj(self) -> int:
        return self.n_worlds * self.traj_per_world

    @property
    def B(self) -> int:
        return self.n_traj * self.n_ls * self.T


# name -> (n_spheres, n_pairs, n_worlds, n_cuboids, traj_per_world, T, n_ls, q kind)
WORKLOADS: Dict[str, Tuple[int, int, int, int, int, int, int, str]] = {
    # one arm, 52 spheres over 9 links, 10 cuboids, 1 trajectory x 8 timesteps
    "tiny": (52, 300, 1, 10, 1, 8, 1, "iid"),
    # 60 spheres, 40 cuboids, 4 worlds x 32 seeds x 32 timesteps, 4 line-search candidates
    "batched": (60, 300, 4, 40, 32, 32, 4, "traj"),
    # 64 worlds x 64 seeds x 48 timesteps = 196,608 configurations, 64 cuboids, 300 pairs
    "large": (60, 300, 64, 64, 64, 48, 1, "iid"),
}


def make_workload(name: str, seed: int = MASTER_SEED, exact: bool = False) -> Workload:
    n_s, n_p, W, K, S, T, n_ls, kind = WORKLOADS[name]
    robot = make_robot(n_s, n_p, seed=seed, exact=exact)
    worlds = make_worlds(W, K, seed=seed, exact=exact)
    B = W * S * n_ls * T
    if kind == "iid":
        q = make_configs(B, seed=seed, exact=exact)
    else:
        traj = make_trajectories(W, S, T, seed=seed, exact=exact)  # [W, S, T, 7]
        q = np.repeat(traj.reshape(W * S, 1, T, N_JOINTS), n_ls, axis=1).reshape(B, N_JOINTS)
    return Workload(name=name, robot=robot, worlds=worlds, traj_per_world=S, T=T, n_ls=n_ls, q=q)


# ---- learned seeder inputs --------------------------------------------------------------------

# layer sizes of the seeding network: features (start 7, goal 7, occupancy 512) -> 3 x 256 -> 8 seeds
# x 32 timesteps x 7 joints
SEEDNET_LAYERS = ((526, 256), (256, 256), (256, 256), (256, 1792))


def make_seednet_params(seed: int = MASTER_SEED) -> Dict[str, np.ndarray]:
    """Initial weights W_l [fan_in, fan_out] and biases b_l [fan_out], l = 1..4, each drawn
    U(-1/sqrt(fan_in), 1/sqrt(fan_in)) and rounded to FP32."""
    rng = _rng(seed, "seednet")
    out = {}
    for l, (fi, fo) in enumerate(SEEDNET_LAYERS, 1):
        b = 1.0 / np.sqrt(fi)
        out[f"W{l}"] = _as_inputs(rng.uniform(-b, b, size=(fi, fo)), False)
        out[f"b{l}"] = _as_inputs(rng.uniform(-b, b, size=fo), False)
    return out


@dataclass
class SeedProblems:
    """Planning problems: one world of cuboids, a start and a goal configuration each."""

    worlds: Worlds
    start: np.ndarray  # [n, 7]
    goal: np.ndarray   # [n, 7]


def _split_rng(seed: int, stream: str, split: int) -> np.random.Generator:
    child = np.random.SeedSequence(seed).spawn(len(_STREAMS))[_STREAMS.index(stream)]
    return np.random.default_rng(child.spawn(split + 1)[split])


def make_seed_problems(n: int, n_cuboids: int, split: int = 0, seed: int = MASTER_SEED) -> SeedProblems:
    """n problems drawn like the benchmark worlds (cuboid centres U[-0.75, 0.75]^3 m, sides
    U[0.05, 0.5] m, uniform rotations) with start and goal U[-2.8, 2.8]^7; `split` picks an
    independent set (0: training, 1: evaluation, ...)."""
    rng = _split_rng(seed, "seed_problems", split)
    m = n * n_cuboids
    R = _random_rotations(rng, m)
    c = rng.uniform(-0.75, 0.75, size=(m, 3))
    h = 0.5 * rng.uniform(0.05, 0.5, size=(m, 3))
    pose = np.concatenate([R, c[:, :, None]], axis=2).reshape(n, n_cuboids, 3, 4)
    start = rng.uniform(-Q_RANGE, Q_RANGE, size=(n, N_JOINTS))
    goal = rng.uniform(-Q_RANGE, Q_RANGE, size=(n, N_JOINTS))
    return SeedProblems(worlds=Worlds(pose=_as_inputs(pose, False), half_ext=_as_inputs(h.reshape(n, n_cuboids, 3), False)),
                        start=_as_inputs(start, False), goal=_as_inputs(goal, False))


def make_seed_family(n: int, n_cuboids: int, family: int, split: int = 0, jitter: float = 0.05,
                     seed: int = MASTER_SEED) -> SeedProblems:
    """n problems in one environment: a base world of n_cuboids drawn once per `family` like the
    benchmark worlds, each problem moving every cuboid centre by U[-jitter, jitter]^3 m, with start
    and goal U[-2.8, 2.8]^7; `split` picks an independent set of problems in that environment."""
    base = _split_rng(seed, "seed_family", 2 * family)
    R = _random_rotations(base, n_cuboids)
    c = base.uniform(-0.75, 0.75, size=(n_cuboids, 3))
    h = 0.5 * base.uniform(0.05, 0.5, size=(n_cuboids, 3))
    rng = _split_rng(seed, "seed_family", 2 * family + 1 + 2 * 1000 * (split + 1))
    cj = c[None] + rng.uniform(-jitter, jitter, size=(n, n_cuboids, 3))
    pose = np.concatenate([np.broadcast_to(R, (n, n_cuboids, 3, 3)), cj[..., None]], axis=3)
    half = np.broadcast_to(h, (n, n_cuboids, 3))
    start = rng.uniform(-Q_RANGE, Q_RANGE, size=(n, N_JOINTS))
    goal = rng.uniform(-Q_RANGE, Q_RANGE, size=(n, N_JOINTS))
    return SeedProblems(worlds=Worlds(pose=_as_inputs(pose, False), half_ext=_as_inputs(np.array(half), False)),
                        start=_as_inputs(start, False), goal=_as_inputs(goal, False))


def make_seed_inits(start: np.ndarray, goal: np.ndarray, n_seeds: int, T: int, kind: str, split: int = 0,
                    seed: int = MASTER_SEED) -> np.ndarray:
    """Initial trajectories [n, n_seeds, T, 7] from start to goal (rows 0 and T-1 are the endpoints).
    kind "linear": the straight line for seed 0, the straight line plus sin(pi tau) delta_s with
    delta_s ~ U[-1, 1]^7 for the others; kind "random": two straight segments through a via point
    drawn U[-2.8, 2.8]^7 at tau = 1/2."""
    rng = _split_rng(seed, "seed_inits", split * 2 + (0 if kind == "linear" else 1))
    n = start.shape[0]
    tau = np.linspace(0.0, 1.0, T).reshape(1, 1, T, 1)
    s0, g0 = start[:, None, None, :], goal[:, None, None, :]
    if kind == "linear":
        delta = rng.uniform(-1.0, 1.0, size=(n, n_seeds, 1, N_JOINTS))
        delta[:, 0] = 0.0
        traj = s0 + (g0 - s0) * tau + np.sin(np.pi * tau) * delta
    elif kind == "random":
        via = rng.uniform(-Q_RANGE, Q_RANGE, size=(n, n_seeds, 1, N_JOINTS))
        first = s0 + (via - s0) * np.minimum(2.0 * tau, 1.0)
        traj = np.where(tau <= 0.5, first, via + (g0 - via) * (2.0 * tau - 1.0))
    else:
        raise ValueError(kind)
    traj[:, :, 0, :] = start[:, None, :]
    traj[:, :, -1, :] = goal[:, None, :]
    return _as_inputs(traj, False)
