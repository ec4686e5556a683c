"""GPU encoding of the paper's ExMy format space (vapr_round_exmy, vapr_quantize_exmy /
vapr_dequantize_exmy and VAPR_EXMY stored tensors) against the oracle (oracle/exmy.py): bit-exact
rounding for all 21 ladder types, packed codes bit-exact against the oracle's on random and dense
inputs and on every float32 bit pattern for four types (committed per-chunk digests), every code
decoded exactly, emulated types that coincide with storage formats giving bit-identical end-to-end
results, and a mixed emulated assignment against the oracle's emulation."""
import json
import os

import numpy as np
import pytest
import xxhash

from oracle import cost as OC
from oracle import exmy as X
from oracle import formats as F
from synthetic import make_workload
from tests.gpu_helpers import cost_tolerance, dev, grad_tolerance, kink_free, make_context, need_gpu, shape_of, torch

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exmy_hashes.json")


def _inputs():
    rng = np.random.default_rng(1)
    mags = 2.0 ** rng.uniform(-149, 128, size=300_000) * rng.choice([-1, 1], size=300_000)
    dense = np.linspace(-600.0, 600.0, 600_001)
    special = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 1.1754942e-38, 3.4028235e38, -3.4028235e38,
                        6.0, 6.5, 28.0, 30.0, 448.0, 480.0, 496.0, 65504.0, 65519.99, 65520.0, 1e30])
    return F.fp32(np.concatenate([mags, dense, special])).astype(np.float64)


@pytest.mark.parametrize("E,M", X.LADDER + [(8, 4), (1, 0), (7, 12)])
@pytest.mark.parametrize("k", [0, -4, 5])
def test_round_exmy_bit_exact(E, M, k):
    need_gpu()
    from paper_2310_07854_amd.context import round_exmy

    x = _inputs()
    got = round_exmy(dev(x, torch.float32), E, M, k).cpu().numpy()
    _, ref = X.roundtrip(x, E, M, k)
    ref32 = ref.astype(np.float32)
    nan = np.isnan(ref32)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan].view(np.uint32), ref32[~nan].view(np.uint32))


def _codes_dev(words: "torch.Tensor", E: int, M: int, n: int) -> "torch.Tensor":
    """Codes (int64, on the device) of n packed codes: unpacking done with torch, not the library."""
    b, q = X.bits(E, M), X.per_word(E, M)
    w = words.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    parts = [(w >> (j * b)) & ((1 << b) - 1) for j in range(q)]
    return torch.stack(parts, dim=1).reshape(-1)[:n]


@pytest.mark.parametrize("E,M", X.LADDER + [(8, 4), (1, 0), (7, 12), (3, 0), (6, 1)])
@pytest.mark.parametrize("k", [0, -4, 5])
def test_quantize_exmy_codes_and_values(E, M, k):
    """Packed codes equal the oracle's packing of its codes, word for word (ragged tail included);
    decoding them gives the oracle's values."""
    need_gpu()
    from paper_2310_07854_amd.context import dequantize_exmy, quantize_exmy

    x = _inputs()[:700_001]
    words = quantize_exmy(dev(x, torch.float32), E, M, k)
    assert words.numel() == 4 * -(-x.size // X.per_word(E, M))
    ref_codes = X.encode(x, E, M, k)
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), X.pack(ref_codes, E, M))
    got = dequantize_exmy(words, E, M, x.size, k).cpu().numpy()
    ref = X.decode(ref_codes, E, M, k).astype(np.float32)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan].view(np.uint32), ref[~nan].view(np.uint32))


@pytest.mark.parametrize("E,M", [(2, 1), (3, 1), (4, 3), (5, 2), (3, 4)])
def test_every_exmy_code_decodes_exactly(E, M):
    need_gpu()
    from paper_2310_07854_amd.context import dequantize_exmy

    n = 1 << X.bits(E, M)
    codes = np.arange(n, dtype=np.uint32)
    words = torch.from_numpy(X.pack(codes, E, M).view(np.uint8)).to("cuda:0")
    for k in (0, -3, 5):
        got = dequantize_exmy(words, E, M, n, k).cpu().numpy()
        ref = X.decode(codes, E, M, k).astype(np.float32)
        np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("fmt", ["e3m1", "e2m2", "e5m4", "e6m6"])
def test_exmy_exhaustive_bit_exact(fmt):
    """Codes of every float32 bit pattern against the committed digests of the oracle's codes."""
    need_gpu()
    from paper_2310_07854_amd.context import quantize

    gold = json.load(open(GOLDEN))
    E, M = X.parse(fmt)
    bits = gold["chunk_bits"]
    n = 1 << bits
    base = torch.arange(n, dtype=torch.int64, device="cuda:0")
    bad = []
    for c in range(1 << (32 - bits)):
        v = base + (c << bits)
        x = torch.where(v >= 2 ** 31, v - 2 ** 32, v).to(torch.int32).view(torch.float32)
        codes = _codes_dev(quantize(x, fmt), E, M, n)
        codes = torch.where(torch.isnan(x), 0, codes)
        codes = codes.to(torch.uint8) if X.bits(E, M) <= 8 else codes.to(torch.int16)
        if xxhash.xxh3_64_hexdigest(codes.cpu().numpy().tobytes()) != gold["codes"][fmt][c]:
            bad.append(c)
        if c % 64 == 63:
            print(f"[exhaustive] {fmt}: {c + 1} of {1 << (32 - bits)} chunks, {len(bad)} differ", flush=True)
    if bad:
        c = bad[0]
        x = (np.arange(n, dtype=np.uint64) + (c << bits)).astype(np.uint32).view(np.float32)
        ref = X.encode(x, E, M)
        got = _codes_dev(quantize(torch.from_numpy(x).to("cuda:0"), fmt), E, M, n).cpu().numpy()
        idx = np.nonzero((ref != got) & ~np.isnan(x))[0][:8]
        pytest.fail(f"{fmt}: {len(bad)} chunks differ; first chunk {c}: inputs {x[idx]} oracle {ref[idx]} gpu {got[idx]}")


@pytest.mark.parametrize("native,emulated", [("f16", "e5m10"), ("bf16", "e8m7")])
def test_emulated_equals_storage_format_end_to_end(native, emulated):
    """Rounding to E5M10 (E8M7) and storing the FP32 value is what FP16 (BF16) storage does: every
    cost, stored value and gradient is bit-identical."""
    need_gpu()
    wl = make_workload("batched")
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    outs = []
    for fmt in (native, emulated):
        prec = {"link_poses": fmt, "sphere_pos": fmt, "sphere_dist": (fmt, -6), "sphere_grad": (fmt, 3),
                "joint_grad": (fmt, 2)}
        ctx = make_context(wl, prec)
        cost, ws = ctx.cost_fwd(q, shape)
        grad = ctx.cost_bwd(q, ws)
        torch.cuda.synchronize()
        # the emulated type's packed codes are the storage format's codes (two per word, low first)
        S = ctx.ws_export("sphere_pos", ws, shape).cpu().numpy()
        outs.append((cost.cpu().numpy(), grad.cpu().numpy(), S))
        ctx.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1].view(np.uint32), outs[1][1].view(np.uint32))
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


def test_emulated_assignment_matches_oracle():
    """A mixed assignment of emulated types (one per tensor, with scales) against the oracle's
    emulation: stored positions equal the oracle's rounding of a value within the FP32 error of the
    exact one, costs within the usual bound; on kink-free configurations whose stored positions,
    poses and sphere gradients equal the oracle's, the stored joint gradient is the rounding of a
    value within the FP32 gradient band of the oracle's."""
    need_gpu()
    wl = make_workload("batched")
    prec = {"link_poses": "e5m9", "sphere_pos": "e6m6", "sphere_dist": ("e3m1", -4), "sphere_grad": ("e2m2", 3),
            "joint_grad": ("e5m4", 2)}
    ctx = make_context(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    cost, ws = ctx.cost_fwd(q, shape)
    grad = ctx.cost_bwd(q, ws).cpu().numpy()
    torch.cuda.synchronize()
    oprec = OC.Precision(**{t: ((v, 0) if isinstance(v, str) else tuple(v)) for t, v in prec.items()})
    ref = OC.fwd_bwd(wl.robot, wl.worlds, wl.q, wl.traj_per_world, wl.T, wl.n_ls, prec=oprec)
    def values(name):
        E, M = X.parse(prec[name] if isinstance(prec[name], str) else prec[name][0])
        k = 0 if isinstance(prec[name], str) else prec[name][1]
        words = ctx.ws_export(name, ws, shape).cpu().numpy().view(np.uint32)
        n = shape.B * ctx.tensor_count(name)
        return X.decode(X.unpack(words, E, M, n), E, M, k)

    S = values("sphere_pos")
    x = ref["S"].reshape(-1)
    tol = 4e-6 * np.abs(x) + 1e-5
    lo, hi = X.round_value(F.fp32(x - tol), 6, 6), X.round_value(F.fp32(x + tol), 6, 6)
    assert np.all((S >= np.minimum(lo, hi)) & (S <= np.maximum(lo, hi)))
    same = np.all(S.reshape(shape.B, -1) == ref["S_hat"].reshape(shape.B, -1), axis=1)
    assert same.mean() > 0.9
    ctol = cost_tolerance(ref, wl.robot.n_pairs, wl.T)
    c = cost.cpu().numpy()
    ok_tc = same.reshape(-1, wl.T).all(axis=1)
    # D and G carry coarse types: a cost term may sit on a rounding boundary of D, so the cost is
    # compared against the oracle's with the D-step bound of such a term added where needed
    dstep = 2.0 ** (np.floor(np.log2(np.maximum(ref["D"], 1e-30))) - 1) * 2.0 ** -4
    extra = (2.0 * OC.CostParams().w_coll * ref["D_hat"] * dstep).sum(axis=1).reshape(-1, wl.T).sum(axis=1)
    assert np.all(np.abs(c - ref["cost_traj"])[ok_tc] <= (ctol + extra)[ok_tc])
    assert np.abs(ref["J_hat"]).max() > 0 and np.isfinite(grad).all()
    # gradients: identical stored inputs to the adjoint leave only FP32 arithmetic before J's rounding
    def stored(name, key):
        v = values(name)
        return np.all(v.reshape(shape.B, -1) == ref[key].reshape(shape.B, -1), axis=1)
    rows = same & stored("link_poses", "L_hat") & stored("sphere_grad", "G_hat") & kink_free(ref)
    assert rows.mean() > 0.3, rows.mean()
    tol = grad_tolerance(ref)
    E, M = X.parse(prec["joint_grad"][0])
    kj = prec["joint_grad"][1]
    lo = X.roundtrip(ref["J"] - tol, E, M, kj)[1]
    hi = X.roundtrip(ref["J"] + tol, E, M, kj)[1]
    g = grad.astype(np.float64)
    ok = (g >= np.minimum(lo, hi)) & (g <= np.maximum(lo, hi))
    assert ok[rows].all(), int((~ok[rows]).sum())
    print(f"[exmy] gradients of {int(rows.sum())}/{shape.B} configurations compared, "
          f"{int((g != ref['J_hat'])[rows].sum())} stored values one step from the oracle's")


def test_packed_workspace_export_import_round_trip():
    """Exported packed codes of every emulated stored tensor re-import to the same words, and a
    backward pass from the re-imported tensors gives the original joint gradient bit for bit."""
    need_gpu()
    wl = make_workload("tiny")
    prec = {"link_poses": "e5m9", "sphere_pos": "e4m5", "sphere_dist": ("e3m1", -4), "sphere_grad": ("e2m3", 3),
            "joint_grad": ("e5m4", 2)}
    ctx = make_context(wl, prec)
    shape = shape_of(wl)
    q = dev(wl.q, torch.float32)
    _, ws = ctx.cost_fwd(q, shape)
    grad = ctx.cost_bwd(q, ws).cpu().numpy()
    names = ("link_poses", "sphere_pos", "sphere_dist", "sphere_grad", "self_cost", "bound_cost")
    saved = {t: ctx.ws_export(t, ws, shape).clone() for t in names}
    for t in ("sphere_pos", "sphere_dist", "sphere_grad"):
        E, M = X.parse(prec[t] if isinstance(prec[t], str) else prec[t][0])
        assert saved[t].numel() == 4 * -(-shape.B * ctx.tensor_count(t) // X.per_word(E, M))
    ws2 = ctx.new_workspace(shape)
    for t in names:
        ctx.ws_import(t, ws2, shape, saved[t])
    grad2 = ctx.cost_bwd(q, ws2).cpu().numpy()
    np.testing.assert_array_equal(grad.view(np.uint32), grad2.view(np.uint32))
    for t in names:
        assert torch.equal(ctx.ws_export(t, ws2, shape), saved[t]), t
    ctx.close()


def test_exmy_rejected_where_codes_are_needed():
    need_gpu()
    from paper_2310_07854_amd import VaprError, _lib as L
    from paper_2310_07854_amd.context import quantize, round_exmy

    x = torch.ones(16, device="cuda:0")
    with pytest.raises(VaprError):
        round_exmy(x, 9, 2)
    with pytest.raises(VaprError):
        round_exmy(x, 3, 24)
    lib = L.load()
    assert lib.vapr_quantize(L.EXMY, 0, x.data_ptr(), x.data_ptr(), 16, None) == L.E_INVALID
    with pytest.raises(VaprError):
        quantize(x, "e9m2")
    out = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    assert lib.vapr_quantize_exmy(3, 24, 0, x.data_ptr(), out.data_ptr(), 16, None) == L.E_INVALID
    assert lib.vapr_quantize_exmy(0, 2, 0, x.data_ptr(), out.data_ptr(), 16, None) == L.E_INVALID
    assert lib.vapr_dequantize_exmy(3, 2, 0, out.data_ptr(), None, 16, None) == L.E_INVALID
    assert lib.vapr_quantize_exmy(3, 2, 0, x.data_ptr() + 2, out.data_ptr(), 8, None) == L.E_INVALID
    assert lib.vapr_exmy_packed_bytes(3, 2, 11) == 12 and lib.vapr_exmy_packed_bytes(9, 2, 11) == 0
