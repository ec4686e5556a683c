"""GPU parity of the learned-seeder kernels against the FP64 oracle (oracle/seeding.py) or exact
FP64 products of the same BF16 operands.

Bounds: a K-term FP32 accumulation of exact BF16 products is within K * 2^-24 * sum |a||b| of the
exact sum in any order; a BF16 output must be the rounding of a value inside the FP32 band of its
reference (so codes are equal wherever the band holds no rounding boundary); integer decisions
(occupancy, loss assignment) must agree wherever the FP64 value is not within rounding of the
threshold or tie.
"""
import numpy as np
import pytest

from oracle import formats as F
from oracle import seeding as SD
from synthetic import make_seed_problems, make_seednet_params
from tests.gpu_helpers import need_gpu, torch

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def S():
    from paper_2310_07854_amd import seeding
    return seeding


def bf16_codes(x: np.ndarray) -> np.ndarray:
    return F.encode(F.fp32(x), "bf16").astype(np.uint16)


def dev_bf16(x: np.ndarray) -> torch.Tensor:
    return torch.tensor(bf16_codes(x).view(np.int16), device="cuda:0").view(torch.bfloat16)


def host_codes(t: torch.Tensor) -> np.ndarray:
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


def host_bf16(t: torch.Tensor) -> np.ndarray:
    return F.decode(host_codes(t), "bf16").astype(np.float64)


def assert_bf16_in_band(codes: np.ndarray, ref: np.ndarray, band: np.ndarray):
    """codes must be the BF16 rounding of some value within [ref - band, ref + band]."""
    lo = bf16_codes(ref - band).view(np.int16).astype(np.int64)
    hi = bf16_codes(ref + band).view(np.int16).astype(np.int64)
    # order codes by value (sign-magnitude -> monotone integers)
    def ordv(c):
        c = c.astype(np.int64) & 0xFFFF
        return np.where(c & 0x8000, -(c & 0x7FFF), c & 0x7FFF)
    got = ordv(codes.view(np.uint16))
    lo_o, hi_o = ordv(lo.astype(np.uint16)), ordv(hi.astype(np.uint16))
    ok = (got >= np.minimum(lo_o, hi_o)) & (got <= np.maximum(lo_o, hi_o))
    assert ok.all(), f"{(~ok).sum()} codes outside the band"


@pytest.mark.parametrize("a_k,b_n", [(True, True), (True, False), (False, True), (False, False)])
@pytest.mark.parametrize("M,N,K", [(100, 80, 96), (64, 64, 32), (37, 200, 544), (256, 1792, 64), (45, 37, 64)])
def test_gemm_layouts_and_tails(a_k, b_n, M, N, K):
    need_gpu()
    rng = np.random.default_rng(M * 7 + N + K)
    A = F.decode(bf16_codes(rng.normal(size=(M, K))), "bf16").astype(np.float64)
    B = F.decode(bf16_codes(rng.normal(size=(K, N))), "bf16").astype(np.float64)
    bias = F.fp32(rng.normal(size=N)).astype(np.float64)
    # device operands in the requested layouts
    Ad = dev_bf16(A if a_k else A.T.copy())
    Bd = dev_bf16(B if b_n else B.T.copy())
    a_ms, a_ks = (K, 1) if a_k else (1, M)
    b_ks, b_ns = (N, 1) if b_n else (1, K)
    C = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    C16 = torch.empty(M, N, dtype=torch.bfloat16, device="cuda:0")
    S().gemm(Ad, a_ms, a_ks, Bd, b_ks, b_ns, M, N, K, bias=torch.tensor(bias, dtype=torch.float32, device="cuda:0"),
             C=C, C16=C16)
    ref = A @ B + bias
    band = K * U32 * (np.abs(A) @ np.abs(B)) + U32 * np.abs(bias) + 1e-30
    got = C.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= band), float(np.max(np.abs(got - ref) / band))
    np.testing.assert_array_equal(host_codes(C16), bf16_codes(got))


def test_gemm_gelu_epilogues():
    need_gpu()
    rng = np.random.default_rng(11)
    M, N, K = 96, 128, 256
    A = F.decode(bf16_codes(rng.normal(size=(M, K)) * 0.1), "bf16").astype(np.float64)
    B = F.decode(bf16_codes(rng.normal(size=(K, N)) * 0.1), "bf16").astype(np.float64)
    bias = F.fp32(rng.normal(size=N) * 0.1).astype(np.float64)
    z = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    out = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    out16 = torch.empty(M, N, dtype=torch.bfloat16, device="cuda:0")
    S().gemm(dev_bf16(A), K, 1, dev_bf16(B), N, 1, M, N, K, bias=torch.tensor(bias, dtype=torch.float32, device="cuda:0"),
             epilogue=S().GELU, aux=z, C=out, C16=out16)
    ref = A @ B + bias
    band = K * U32 * (np.abs(A) @ np.abs(B)) + U32 * np.abs(bias) + 1e-30
    zg = z.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(zg - ref) <= band)
    # GELU of the GPU's own pre-activation: FP32 evaluation within a few ulp
    g = out.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(g, SD.gelu(zg), rtol=2e-6, atol=1e-7)
    assert_bf16_in_band(host_codes(out16), SD.gelu(zg), 2e-6 * np.abs(SD.gelu(zg)) + 1e-7)
    # times GELU'(aux): Z2 = A B (no bias)
    out2 = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    S().gemm(dev_bf16(A), K, 1, dev_bf16(B), N, 1, M, N, K, epilogue=S().GELU_GRAD, aux=z, C=out2)
    z2 = A @ B
    want = z2 * SD.gelu_grad(zg)
    bandg = (K * U32 * (np.abs(A) @ np.abs(B))) * np.abs(SD.gelu_grad(zg)) + 4e-6 * np.abs(want) + 1e-9
    assert np.all(np.abs(out2.cpu().numpy() - want) <= bandg)


@pytest.mark.parametrize("M,N,ldx", [(1, 1, 1), (15, 63, 70), (100, 65, 65), (257, 256, 256), (256, 1792, 1800)])
def test_column_sum_ragged(M, N, ldx):
    """Bias gradients: FP32 column sums of a row-major [M][ldx] matrix, within M * 2^-24 * sum |x|
    of the exact sum; the padding columns are never read into the result."""
    need_gpu()
    rng = np.random.default_rng(M * 7 + N)
    X = F.fp32(rng.normal(size=(M, ldx))).astype(np.float64)
    out = torch.full((N,), float("nan"), dtype=torch.float32, device="cuda:0")
    S().column_sum(torch.tensor(X, dtype=torch.float32, device="cuda:0")[:, :N], out)
    got = out.cpu().numpy().astype(np.float64)
    ref = X[:, :N].sum(axis=0)
    band = M * U32 * np.abs(X[:, :N]).sum(axis=0) + 1e-30
    assert np.all(np.abs(got - ref) <= band)


def test_occupancy_matches_oracle():
    need_gpu()
    pr = make_seed_problems(24, 20, split=5)
    occ = S().occupancy(torch.tensor(pr.worlds.pose, dtype=torch.float32, device="cuda:0"),
                        torch.tensor(pr.worlds.half_ext, dtype=torch.float32, device="cuda:0")).cpu().numpy()
    ref = SD.occupancy(pr.worlds.pose, pr.worlds.half_ext)
    # margin of the decision: smallest |sd - e/2| per voxel (FP64)
    cen = SD.voxel_centres()
    margin = np.full(ref.shape, np.inf)
    for w in range(ref.shape[0]):
        sd = np.full(512, np.inf)
        for k in range(pr.worlds.pose.shape[1]):
            d, _, _ = SD.obb_signed_distance(cen, pr.worlds.pose[w, k, :, :3], pr.worlds.pose[w, k, :, 3],
                                             pr.worlds.half_ext[w, k])
            sd = np.minimum(sd, d)
        margin[w] = np.abs(sd - 0.09375)
    sure = margin > 1e-5
    assert sure.mean() > 0.99
    np.testing.assert_array_equal(occ[sure], ref[sure])
    assert 0.05 < ref.mean() < 0.95
    empty = S().occupancy(torch.zeros(3, 0, 3, 4, device="cuda:0"), torch.zeros(3, 0, 3, device="cuda:0"))
    assert not empty.any()


@pytest.mark.parametrize("b_n", [True, False])
def test_gemm_large_tiles_match_small_tiles(b_n):
    """A product large enough for the 128 x 128 tiles, ragged in M and N: every output equals the
    same product computed in row slices small enough for the 64 x 64 tiles, bit for bit (both sum K
    in the same 32-wide MFMA steps), and the GELU pre-activation lies in the FP32 error band of the
    float64 product."""
    need_gpu()
    rng = np.random.default_rng(97 + b_n)
    M, N, K = 4133, 4100, 96
    A = F.decode(bf16_codes(rng.normal(size=(M, K))), "bf16").astype(np.float64)
    B = F.decode(bf16_codes(rng.normal(size=(K, N))), "bf16").astype(np.float64)
    bias_h = F.fp32(rng.normal(size=N)).astype(np.float64)
    bias = torch.tensor(bias_h, dtype=torch.float32, device="cuda:0")
    Ad = dev_bf16(A)
    Bd = dev_bf16(B if b_n else B.T.copy())
    b_ks, b_ns = (N, 1) if b_n else (1, K)

    def run(r0, r1, z, c, c16):
        S().gemm(Ad[r0:r1], K, 1, Bd, b_ks, b_ns, r1 - r0, N, K, bias=bias, epilogue=S().GELU, aux=z[r0:r1],
                 C=c[r0:r1], C16=c16[r0:r1])

    out = [(torch.empty(M, N, dtype=torch.float32, device="cuda:0"), torch.empty(M, N, dtype=torch.float32,
            device="cuda:0"), torch.empty(M, N, dtype=torch.bfloat16, device="cuda:0")) for _ in range(2)]
    run(0, M, *out[0])
    for r0 in range(0, M, 512):
        run(r0, min(M, r0 + 512), *out[1])
    torch.cuda.synchronize()
    for big, small in zip(out[0], out[1]):
        np.testing.assert_array_equal(big.view(torch.int16 if big.dtype == torch.bfloat16 else torch.int32).cpu().numpy(),
                                      small.view(torch.int16 if small.dtype == torch.bfloat16 else torch.int32).cpu().numpy())
    ref = A @ B + bias_h
    band = K * U32 * (np.abs(A) @ np.abs(B)) + U32 * np.abs(bias_h) + 1e-30
    got = out[0][0].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= band), float(np.max(np.abs(got - ref) / band))


@pytest.mark.parametrize("ldc_pad", [3, 4])
def test_gemm_row_stride_keeps_padding(ldc_pad):
    """Outputs with ldc > N (padded rows, odd and 16-byte multiple strides): every element equals the
    ldc = N result bit for bit, including the GELU epilogue's pre-activation, and the padding columns
    keep their contents."""
    need_gpu()
    rng = np.random.default_rng(31 + ldc_pad)
    M, N, K = 70, 72, 64
    A = dev_bf16(rng.normal(size=(M, K)))
    B = dev_bf16(rng.normal(size=(K, N)))
    bias = torch.tensor(F.fp32(rng.normal(size=N)), dtype=torch.float32, device="cuda:0")
    ldc = N + ldc_pad
    ref_z = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    ref_c = torch.empty(M, N, dtype=torch.float32, device="cuda:0")
    S().gemm(A, K, 1, B, N, 1, M, N, K, bias=bias, epilogue=S().GELU, aux=ref_z, C=ref_c)
    z = torch.full((M, ldc), 7.0, dtype=torch.float32, device="cuda:0")
    c = torch.full((M, ldc), 7.0, dtype=torch.float32, device="cuda:0")
    S().gemm(A, K, 1, B, N, 1, M, N, K, bias=bias, epilogue=S().GELU, aux=z, C=c, ldc=ldc)
    np.testing.assert_array_equal(z[:, :N].cpu().numpy(), ref_z.cpu().numpy())
    np.testing.assert_array_equal(c[:, :N].cpu().numpy(), ref_c.cpu().numpy())
    assert bool((z[:, N:] == 7.0).all()) and bool((c[:, N:] == 7.0).all())


@pytest.mark.parametrize("n,lda", [(1, 256), (100, 256), (257, 264), (9401, 256)])
def test_seed_head_equals_gemm_then_trajectories(n, lda):
    """The fused output layer equals the plain GEMM followed by the trajectory kernel bit for bit
    (ragged problem counts, a padded hidden-layer row stride; 9,401 problems take the 128 x 128
    tiles)."""
    need_gpu()
    rng = np.random.default_rng(n)
    net = S().SeedNet(make_seednet_params())
    a3 = dev_bf16(rng.normal(size=(n, lda)))
    start = torch.tensor(F.fp32(rng.uniform(-2.8, 2.8, size=(n, 7))), dtype=torch.float32, device="cuda:0")
    goal = torch.tensor(F.fp32(rng.uniform(-2.8, 2.8, size=(n, 7))), dtype=torch.float32, device="cuda:0")
    y = torch.empty(n, 1792, dtype=torch.float32, device="cuda:0")
    S().gemm(a3, lda, 1, net.view(net.w16, "W4"), 1792, 1, n, 1792, 256, bias=net.view(net.w, "b4"), C=y)
    ref = S().trajectories(y, start, goal).cpu().numpy()
    got = net.head(a3[:, :256], start, goal).cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("n", [1, 40, 1000])
def test_features_and_trajectories(n):
    need_gpu()
    rng = np.random.default_rng(12 + n)
    start, goal = F.fp32(rng.uniform(-2.8, 2.8, size=(n, 7))), F.fp32(rng.uniform(-2.8, 2.8, size=(n, 7)))
    occ = (rng.random((n, 512)) < 0.3).astype(np.float32)
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")
    x = S().features(d(start), d(goal), d(occ))
    want = np.zeros((n, 544))
    want[:, :526] = SD.features(start, goal, occ)
    np.testing.assert_array_equal(host_codes(x), bf16_codes(want))
    y = F.fp32(rng.normal(scale=0.3, size=(n, 1792)))
    traj = S().trajectories(d(y), d(start), d(goal)).cpu().numpy()
    ref = SD.seeds(y, start.astype(np.float64), goal.astype(np.float64))
    np.testing.assert_array_equal(traj[:, :, 0], np.broadcast_to(start[:, None], (n, 8, 7)))
    np.testing.assert_array_equal(traj[:, :, -1], np.broadcast_to(goal[:, None], (n, 8, 7)))
    np.testing.assert_allclose(traj, ref, rtol=0, atol=4e-6)


def test_loss_matches_oracle():
    need_gpu()
    rng = np.random.default_rng(13)
    n = 64
    y = F.fp32(rng.normal(scale=0.5, size=(n, 1792)))
    tgt = F.fp32(rng.normal(scale=0.5, size=(n, 8, 32, 7)))
    valid = (rng.random((n, 8)) < 0.8).astype(np.float32)
    n_valid = int(valid.sum())
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")
    net = S().SeedNet(make_seednet_params())
    loss, dy, assign = net.loss(d(y), d(tgt.reshape(n, -1)), d(valid), n_valid)
    L, dy_ref, as_ref = SD.loss(y, tgt, valid)
    assert abs(float(loss.item()) - L) <= 1e-6 * L
    # assignment: equal wherever the best slot beats the runner-up by more than FP32 rounding
    yp, tt = y.reshape(n, 8, 224).astype(np.float64), tgt.reshape(n, 8, 224).astype(np.float64)
    e = np.mean((yp[:, :, None] - tt[:, None]) ** 2, axis=3)
    srt = np.sort(e, axis=1)
    stable = (srt[:, 1] - srt[:, 0]) > 1e-5 * srt[:, 0]
    got = assign.cpu().numpy()
    np.testing.assert_array_equal(got[stable], as_ref[stable])
    rows = stable.all(axis=1)
    # dy = coef * sum_j (y_s - t_j): FP32 differences and a short FP32 sum, bounded by the terms
    coef = 2.0 / (224 * n_valid)
    absum = np.zeros((n, 8, 224))
    for j in range(8):
        use = (as_ref[:, j, None] == np.arange(8)[None, :]) & (valid[:, j, None] != 0)
        absum += use[:, :, None] * np.abs(yp - tt[:, j][:, None, :])
    band = (9 * U32 * coef * absum + 2 * U32 * np.abs(dy_ref.reshape(n, 8, 224)) + 1e-30).reshape(n, -1)
    err = np.abs(dy.cpu().numpy().astype(np.float64) - dy_ref)
    assert np.all(err[rows] <= band[rows]), float(np.max(err[rows] / band[rows]))


def test_adam_matches_oracle():
    need_gpu()
    rng = np.random.default_rng(14)
    net = S().SeedNet(make_seednet_params())
    n = net.n_params
    w0, g = F.fp32(rng.normal(size=n)), F.fp32(rng.normal(size=n) * 1e-3)
    m0, v0 = F.fp32(rng.normal(size=n) * 1e-3), F.fp32(rng.random(n) * 1e-6)
    for t, a in ((net.w, w0), (net.g, g), (net.m, m0), (net.v, v0)):
        t.copy_(torch.tensor(a, device="cuda:0"))
    net.step = 4
    net.adam(lr=1e-3)
    # the GPU runs with FP32 hyper-parameters; 1 - b is exact in FP32 for b in [0.5, 1)
    f = lambda c: float(np.float32(c))
    lr, b1, b2, eps = f(1e-3), f(0.9), f(0.999), f(1e-8)
    w0d, gd, m0d, v0d = (a.astype(np.float64) for a in (w0, g, m0, v0))
    p, m, v = SD.adam({"w": w0d}, {"w": gd}, {"w": m0d}, {"w": v0d}, 5, lr=lr, b1=b1, b2=b2, eps=eps)
    # m, v: an FMA of two rounded products; w: the rounded update (relative 1e-6) plus its rounding
    bm = 3 * U32 * (np.abs(b1 * m0d) + np.abs((1 - b1) * gd)) + 1e-30
    bv = 3 * U32 * (np.abs(b2 * v0d) + np.abs((1 - b2) * gd * gd)) + 1e-30
    assert np.all(np.abs(net.m.cpu().numpy() - m["w"]) <= bm)
    assert np.all(np.abs(net.v.cpu().numpy() - v["w"]) <= bv)
    upd = np.abs(p["w"] - w0d)
    assert np.all(np.abs(net.w.cpu().numpy() - p["w"]) <= 1e-6 * upd + 2 * U32 * np.abs(p["w"]) + 1e-30)
    np.testing.assert_array_equal(host_codes(net.w16), bf16_codes(net.w.cpu().numpy()))


def _batch(n=64, split=6):
    """Problems with learnable targets: target j bends the straight line by
    sin(pi tau) * a_j * (goal - start), a_j evenly spaced in [-0.5, 0.5]."""
    pr = make_seed_problems(n, 16, split=split)
    occ = SD.occupancy(pr.worlds.pose, pr.worlds.half_ext)
    tau = np.linspace(0.0, 1.0, 32)
    a = np.linspace(-0.5, 0.5, 8)
    tgt = F.fp32(np.sin(np.pi * tau)[None, None, :, None] * a[None, :, None, None]
                 * (pr.goal - pr.start)[:, None, None, :])
    valid = np.ones((n, 8), dtype=np.float32)
    valid[::5, 6:] = 0
    return pr, occ, tgt, valid


def test_forward_and_backward_layer_by_layer():
    """Each layer of the GPU network against FP64 of the GPU's own BF16 inputs to that layer."""
    need_gpu()
    pr, occ, tgt, valid = _batch()
    n = pr.start.shape[0]
    params = make_seednet_params()
    net = S().SeedNet(params)
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")
    x = S().features(d(pr.start), d(pr.goal), d(occ))
    y, cache = net.forward(x)
    W16 = {l: host_bf16(net.view(net.w16, f"W{l}")) for l in (1, 2, 3, 4)}
    b = {l: params[f"b{l}"] for l in (1, 2, 3, 4)}
    a = host_bf16(cache["a0"])
    for l in (1, 2, 3):
        ref = a @ W16[l] + b[l]
        band = a.shape[1] * U32 * (np.abs(a) @ np.abs(W16[l])) + U32 * np.abs(b[l]) + 1e-30
        z = cache[f"z{l}"].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(z - ref) <= band), l
        gz = SD.gelu(z)
        assert_bf16_in_band(host_codes(cache[f"a{l}"]), gz, 2e-6 * np.abs(gz) + 1e-7)
        a = host_bf16(cache[f"a{l}"])
    ref = a @ W16[4] + b[4]
    band = 256 * U32 * (np.abs(a) @ np.abs(W16[4])) + U32 * np.abs(b[4]) + 1e-30
    assert np.all(np.abs(y.cpu().numpy() - ref) <= band)
    # backward from the GPU's loss gradient
    loss, dy, _ = net.loss(y, d(tgt.reshape(n, -1)), d(valid), int(valid.sum()))
    net.backward(cache, dy)
    dcur = dy.cpu().numpy().astype(np.float64)
    acts = {l: host_bf16(cache[f"a{l}"]) for l in (0, 1, 2, 3)}
    for l in (4, 3, 2, 1):
        dq = F.decode(bf16_codes(dcur), "bf16").astype(np.float64)
        gW = net.view(net.g, f"W{l}").cpu().numpy().astype(np.float64)
        if l == 1:
            gW = gW[:544]
        ref = acts[l - 1].T @ dq
        band = n * U32 * (np.abs(acts[l - 1]).T @ np.abs(dq)) + 1e-30
        assert np.all(np.abs(gW - ref) <= band), l
        gb = net.view(net.g, f"b{l}").cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(gb, dcur.sum(axis=0), rtol=1e-5, atol=1e-6 * np.abs(dcur).sum(axis=0).max())
        if l > 1:
            z = cache[f"z{l - 1}"].cpu().numpy().astype(np.float64)
            dh = dq @ W16[l].T
            want = dh * SD.gelu_grad(z)
            # the GPU's dz (recomputed here from its own inputs) feeds the next layer
            k = W16[l].shape[1]
            band = k * U32 * (np.abs(dq) @ np.abs(W16[l]).T) * np.abs(SD.gelu_grad(z)) + 4e-6 * np.abs(want) + 1e-12
            dz_gpu = _recompute_dz(net, l, cache, dcur)
            assert np.all(np.abs(dz_gpu - want) <= band), l
            dcur = dz_gpu


def _recompute_dz(net, l, cache, dcur):
    """The GPU's dz_{l-1} for the given upstream gradient (one more backward GEMM)."""
    d16 = S().to_bf16(torch.tensor(dcur, dtype=torch.float32, device="cuda:0"))
    n, k = dcur.shape
    dz = torch.empty(n, 256, dtype=torch.float32, device="cuda:0")
    S().gemm(d16, k, 1, net.view(net.w16, f"W{l}"), 1, k, n, 256, k, epilogue=S().GELU_GRAD, aux=cache[f"z{l - 1}"],
             C=dz)
    return dz.cpu().numpy().astype(np.float64)


def test_training_reduces_the_loss():
    need_gpu()
    pr, occ, tgt, valid = _batch(n=128, split=7)
    d = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")
    net = S().SeedNet(make_seednet_params())
    x = S().features(d(pr.start), d(pr.goal), d(occ))
    tt, vv, nv = d(tgt.reshape(128, -1)), d(valid), int(valid.sum())
    first = float(net.train_step(x, tt, vv, nv, lr=1e-3).item())
    for _ in range(150):
        last = float(net.train_step(x, tt, vv, nv, lr=1e-3).item())
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
    # the FP64 oracle agrees on the loss of the trained weights (same assignment semantics)
    y, _ = net.forward(x)
    L, _, _ = SD.loss(y.cpu().numpy().astype(np.float64), tgt, valid)
    loss, _, _ = net.loss(y, tt, vv, nv)
    assert abs(L - float(loss.item())) <= 1e-5 * L


@pytest.mark.parametrize("diverse", [False, True])
def test_select_targets(diverse):
    """Training targets of the seeder: the lowest-cost collision-free solution first; then either the
    next-cheapest ones or, one at a time, the collision-free solution farthest from those picked
    (brute force over the same distances); problems with fewer than 8 collision-free solutions mark
    the rest invalid."""
    need_gpu()
    from paper_2310_07854_amd import seed_pipeline as SP
    from paper_2310_07854_amd.seeding import N_SEEDS

    rng = np.random.default_rng(3)
    W, S, T = 3, 12, 32
    start = rng.uniform(-1, 1, size=(W, 7)).astype(np.float32)
    goal = rng.uniform(-1, 1, size=(W, 7)).astype(np.float32)
    tau = np.linspace(0, 1, T)[None, None, :, None]
    bend = rng.uniform(-1, 1, size=(W, S, 1, 7))
    x = (start[:, None, None] + (goal - start)[:, None, None] * tau + np.sin(np.pi * tau) * bend).astype(np.float32)
    cost = rng.uniform(1, 2, size=(W, S))
    free = rng.random((W, S)) < 0.8
    free[2, :] = False
    free[2, :5] = True                    # only 5 collision-free solutions
    d = lambda a, dt=torch.float32: torch.tensor(a, dtype=dt, device="cuda:0")
    sol = {"x": d(x), "cost": d(cost, torch.float64), "free": d(free, torch.bool)}
    tgt, valid = SP.select_targets(sol, d(start), d(goal), diverse=diverse)
    tgt, valid = tgt.cpu().numpy(), valid.cpu().numpy()
    dev = x - (start[:, None, None] + (goal - start)[:, None, None] * tau)
    for w in range(W):
        ids = np.flatnonzero(free[w])
        n = min(N_SEEDS, len(ids))
        assert valid[w].tolist() == [1.0] * n + [0.0] * (N_SEEDS - n)
        first = ids[np.argmin(cost[w, ids])]
        picked = [first]
        if diverse:
            flat = dev[w].reshape(S, -1).astype(np.float64)
            near = np.linalg.norm(flat - flat[first], axis=1)
            for _ in range(1, n):
                cand = [i for i in ids if i not in picked]
                nxt = max(cand, key=lambda i: (near[i], -i))
                picked.append(nxt)
                near = np.minimum(near, np.linalg.norm(flat - flat[nxt], axis=1))
        else:
            picked = list(ids[np.argsort(cost[w, ids], kind="stable")][:n])
        for k, i in enumerate(picked):
            np.testing.assert_allclose(tgt[w, k], dev[w, i], atol=2e-6)
        assert np.all(tgt[w, n:] == 0)
