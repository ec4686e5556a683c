"""Workspace poisoning (vapr_ws_poison) and the stored-code census (vapr_ws_census).

Poisoning fills a workspace with 0xFF bytes; a forward and backward pass from it must give every
cost, gradient and stored tensor bit-identical to a clean workspace's (each stage reads only what an
earlier stage of the same pass wrote).  The census counts, per stored tensor, codes at the format's
largest finite magnitude and Inf/NaN codes; the expected counts come from the oracle's decoding of
codes imported into the workspace."""
import numpy as np
import pytest

from oracle import exmy as X
from oracle import formats as F
from synthetic import make_workload
from tests.gpu_helpers import dev, export_codes, import_codes, make_context, need_gpu, shape_of, torch

pytestmark = pytest.mark.gpu

ASSIGNMENTS = {
    "f32": ({}, False),
    "headline": ({"link_poses": ("f16", -15), "sphere_pos": ("f16", -15), "sphere_dist": ("e4m3", -10),
                  "sphere_grad": ("e4m3", -1), "joint_grad": ("e4m3", 0)}, False),
    "fp4_recompute": ({"link_poses": "e4m3", "sphere_pos": ("e4m3", -8), "sphere_dist": ("e2m1", -4),
                       "sphere_grad": ("e2m1", 5), "joint_grad": ("e3m2", 2)}, True),
    "emulated": ({"link_poses": "e5m9", "sphere_pos": "e6m6", "sphere_dist": ("e3m1", -4),
                  "sphere_grad": ("e2m2", 3), "joint_grad": ("e5m4", 2)}, False),
}


@pytest.mark.parametrize("name", list(ASSIGNMENTS))
def test_poisoned_workspace_gives_identical_results(name):
    need_gpu()
    from paper_2310_07854_amd import VaprError

    prec, recompute = ASSIGNMENTS[name]
    wl = make_workload("batched")
    ctx = make_context(wl, prec, recompute)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    out = []
    for poison in (False, True):
        ws = ctx.new_workspace(shape)
        if poison:
            ctx.ws_poison(ws)
            with pytest.raises(VaprError):
                ctx.cost_bwd(q, ws)          # a poisoned workspace holds no forward pass
        cost, _ = ctx.cost_fwd(q, shape, ws=ws)
        grad = ctx.cost_bwd(q, ws)
        torch.cuda.synchronize()
        names = [t for t in ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad", "self_cost",
                             "bound_cost") if not (recompute and t == "link_poses")]
        out.append((cost.cpu().numpy(), grad.cpu().numpy(),
                    {t: ctx.ws_export(t, ws, shape).cpu().numpy() for t in names}))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1].view(np.uint32), out[1][1].view(np.uint32))
    assert np.isfinite(out[1][0]).all()
    for t in out[0][2]:
        np.testing.assert_array_equal(out[0][2][t], out[1][2][t], err_msg=t)
    ctx.close()


def _vmax(fmt):
    if fmt == "f32":
        return float(np.finfo(np.float32).max)
    if fmt in F.FORMATS:
        return float(F.magnitude_table(fmt)[1][-1])
    return X.limits(*X.parse(fmt))[2]


def _code_of(x, fmt):
    if fmt in F.FORMATS:
        return int(F.encode(np.array([x]), fmt)[0])
    return int(X.encode(np.array([x]), *X.parse(fmt))[0])


def _expected(codes, fmt):
    """(largest finite magnitude, Inf/NaN) counts from the oracle's decoding of the codes."""
    if fmt in F.FORMATS:
        v = F.decode(np.asarray(codes).astype(np.uint32), fmt)
    else:
        v = X.decode(codes, *X.parse(fmt))
    fin = np.isfinite(v)
    return int((fin & (np.abs(v) == _vmax(fmt))).sum()), int((~fin).sum())


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16", "e4m3", "e5m2", "e3m2", "e2m1", "e3m1", "e5m10", "e8m7",
                                 "e4m5"])
def test_census_counts_match_oracle(fmt):
    """Random codes over the whole code space, with the largest finite magnitude, its neighbour and
    the top codes made frequent (both signs), imported into the sphere-gradient tensor of a ragged
    batch (24 configurations of 60 spheres)."""
    need_gpu()
    from synthetic import Worlds
    from synthetic.generators import Workload

    base = make_workload("batched")
    wl = Workload("small", base.robot, Worlds(pose=base.worlds.pose[:1], half_ext=base.worlds.half_ext[:1]), 1, 6,
                  4, base.q[:24])
    ctx = make_context(wl, {"sphere_grad": (fmt, 0)})
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    _, ws = ctx.cost_fwd(q, shape)
    bits = F.get(fmt).bits if fmt in F.FORMATS else X.bits(*X.parse(fmt))
    n = shape.B * 60 * 3
    rng = np.random.default_rng(4)
    codes = rng.integers(0, 1 << 62, size=n, dtype=np.int64) & ((1 << bits) - 1)
    maxc = _code_of(_vmax(fmt), fmt)
    special = [maxc, maxc - 1, (1 << (bits - 1)) - 1, (1 << (bits - 1)) - 2, 0]
    pick = rng.integers(0, 2 * len(special), size=n)
    sign = rng.integers(0, 2, size=n) << (bits - 1)
    for j, c in enumerate(special):
        codes = np.where(pick == j, c | sign, codes)
    codes = codes.astype(np.uint64)
    if fmt in F.FORMATS:
        import_codes(ctx, "sphere_grad", ws, shape, codes.astype(np.uint32))
    else:
        words = X.pack(codes, *X.parse(fmt))
        ctx.ws_import("sphere_grad", ws, shape, torch.from_numpy(words.view(np.uint8)).to("cuda:0"))
    got = ctx.census("sphere_grad", ws, shape)
    want = _expected(codes, fmt)
    assert got == want, (got, want)
    assert want[0] > n // 20
    print(f"[census] {fmt}: {got[0]} at the largest magnitude, {got[1]} Inf/NaN of {n}")
    ctx.close()


def test_census_of_a_forward_pass_and_errors():
    need_gpu()
    from paper_2310_07854_amd import VaprError

    wl = make_workload("batched")
    prec, _ = ASSIGNMENTS["headline"]
    ctx = make_context(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    ws = ctx.new_workspace(shape)
    with pytest.raises(VaprError):
        ctx.census("sphere_pos", ws, shape)          # no forward pass yet
    ctx.cost_fwd(q, shape, ws=ws)
    for t in ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "joint_grad"):
        got = ctx.census(t, ws, shape)
        if t == "joint_grad":
            continue
        codes = export_codes(ctx, t, ws, shape)
        assert got == _expected(codes, ctx.precision[t][0]), t
    with pytest.raises(VaprError):
        ctx.census("self_cost", ws, shape)
    ctx.close()
