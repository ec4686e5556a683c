"""The search's evaluator on the GPU: the success rate of an assignment is deterministic, FP32 is
reachable, and a short search returns an assignment that keeps the FP32 rate."""
import dataclasses
from types import SimpleNamespace

import numpy as np
import pytest

from synthetic import make_robot, make_seed_inits, make_seed_problems
from tests.gpu_helpers import need_gpu, torch

pytestmark = pytest.mark.gpu


def test_search_on_a_small_problem_set():
    need_gpu()
    from paper_2310_07854_amd import Context, search as SR

    robot = make_robot(40, 100)
    robot = dataclasses.replace(robot, pairs=robot.pairs[:0])
    pr = make_seed_problems(24, 6, split=3)
    ctx = Context(0)
    ctx.set_robot(robot)
    worlds = SimpleNamespace(pose=pr.worlds.pose, half_ext=pr.worlds.half_ext)
    x0 = make_seed_inits(pr.start, pr.goal, 4, 16, "linear", split=2)
    task = SR.OptimizerTask(ctx, worlds, pr.start, pr.goal, x0, iters=8, n_ls=4)
    a = {t: "f32" for t in SR.TENSORS}
    r1, r2 = task(a), task(a)
    assert r1 == r2 and 0.0 < r1 <= 1.0
    b = dict(a, sphere_pos="e6m6", sphere_dist="e3m1", sphere_grad="e2m2", joint_grad="e4m3")
    rb = task(b)
    assert 0.0 <= rb <= 1.0 and task(b) == rb
    res = SR.Search(task).run(budget=6)
    assert res.best_rate >= res.target == r1
    assert res.best_bits <= 32 * 5 and res.evaluations >= 6
