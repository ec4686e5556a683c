"""Host logic of the variable-precision search (paper_2310_07854_amd/search.py): the ladder and
type limits against the oracle's definitions, scales, and both phases against evaluators whose
answers are known."""
import itertools

import numpy as np
import pytest

from oracle import exmy as X
from oracle import formats as F
from paper_2310_07854_amd import search as S


def test_ladder_and_limits_match_the_format_definitions():
    assert len(S.LADDER) == 21 and [S.bits(f) for f in S.LADDER] == sorted(S.bits(f) for f in S.LADDER)
    names = {X.name(E, M) for E, M in X.LADDER}
    for f in S.LADDER:
        E, M = S.exp_man(f)
        assert X.name(E, M) in names
        if f in F.FORMATS:
            assert S.max_finite(f) == F.max_finite(f)          # storage encodings
        else:
            assert S.max_finite(f) == X.limits(E, M)[2]        # emulated types


@pytest.mark.parametrize("fmt", ["e2m1", "e3m1", "e6m6", "f16", "e4m3"])
def test_scale_covers_the_magnitude(fmt):
    for amax in (1e-3, 0.7, 3.0, 250.0, 1e4):
        k = S.scale_for(fmt, amax)
        assert amax * 2.0 ** -k <= S.max_finite(fmt) or k == 16
        assert k == -16 or amax * 2.0 ** -(k - 1) > S.max_finite(fmt)
    assert S.scale_for("f32", 1e30) == 0


def test_phase_one_finds_per_tensor_thresholds():
    thr = {"link_poses": 18, "sphere_pos": 15, "sphere_dist": 1, "sphere_grad": 4, "joint_grad": 10}
    calls = []

    def evaluate(a):
        calls.append(a)
        ok = all(S.LADDER.index(a[t]) >= thr[t] for t in thr)
        return 0.9 if ok else 0.6

    s = S.Search(evaluate)
    floor = s.per_tensor(0.9)
    assert {t: S.LADDER.index(f) for t, f in floor.items()} == thr
    # binary search: at most ceil(log2(21)) = 5 evaluations per tensor
    assert len(calls) <= 5 * 5


def test_phase_two_reaches_the_optimum_of_a_small_space():
    """Interacting tensors: the sum of ladder indices above the floors must reach a budget, so the
    phase-1 floors alone are infeasible; the evolution must find a feasible assignment with the
    fewest bits, checked by brute force over the reduced space."""
    tensors = ("sphere_dist", "sphere_grad", "joint_grad")
    floors = {"sphere_dist": 1, "sphere_grad": 4, "joint_grad": 10}
    need = 4

    def idx(a, t):
        return S.LADDER.index(a[t])

    def evaluate(a):
        if any(idx(a, t) < floors[t] for t in tensors):
            return 0.0
        return 1.0 if sum(idx(a, t) - floors[t] for t in tensors) >= need else 0.5

    s = S.Search(evaluate, tensors=tensors)
    res = s.run(budget=200, seed=3)
    assert res.per_tensor == {t: S.LADDER[floors[t]] for t in tensors}
    assert res.best_rate >= res.target
    best_bits = min(
        sum(S.bits(S.LADDER[i]) for i in combo)
        for combo in itertools.product(*[range(floors[t], len(S.LADDER)) for t in tensors])
        if evaluate({t: S.LADDER[i] for t, i in zip(tensors, combo)}) >= 1.0)
    assert res.best_bits == best_bits
    # memoised: every assignment evaluated once
    keys = [tuple(a[t] for t in tensors) for a, _ in res.history]
    assert len(keys) == len(set(keys)) == res.evaluations


def test_spec_gives_formats_with_scales():
    amax = {"sphere_pos": 1.2, "joint_grad": 300.0}
    sp = S.spec({"sphere_pos": "e6m6", "joint_grad": "e2m1", "sphere_dist": "f32"}, amax)
    assert sp["sphere_dist"] == ("f32", 0)
    assert sp["joint_grad"][0] == "e2m1" and 300.0 * 2.0 ** -sp["joint_grad"][1] <= 6.0
    assert sp["sphere_pos"] == ("e6m6", S.scale_for("e6m6", 1.2))
