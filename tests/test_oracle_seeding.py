"""Pins of the seeder oracle (oracle/seeding.py) against values fixed outside it: standard normal
CDF values, PyTorch's float64 layers, central differences, hand-worked occupancy patterns, brute
force on tiny matching problems and the closed form of Adam's first steps."""
import numpy as np
import torch

from oracle import seeding as SD
from synthetic import make_seed_problems, make_seednet_params


def test_gelu_known_values():
    # GELU(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707,
    # Phi(2) = 0.9772498680518208
    z = np.array([0.0, 1.0, -1.0, 2.0, 10.0, -10.0])
    want = np.array([0.0, 0.8413447460685429, -0.15865525393145707, 2 * 0.9772498680518208, 10.0, 0.0])
    np.testing.assert_allclose(SD.gelu(z), want, rtol=1e-15, atol=1e-20)


def test_gelu_matches_torch_and_its_derivative():
    z = np.random.default_rng(0).normal(scale=3.0, size=2000)
    ref = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64), approximate="none").numpy()
    # both forms cancel in 1 + erf for very negative z: an absolute floor of 1e-15
    np.testing.assert_allclose(SD.gelu(z), ref, rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (SD.gelu(z + h) - SD.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(SD.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def _box_world(half, R=np.eye(3), c=np.zeros(3)):
    pose = np.concatenate([R, c[:, None]], axis=1)[None, None]
    return pose, np.array(half, dtype=np.float64)[None, None]


def test_occupancy_of_a_centred_cube():
    # voxel edge 0.1875 m, centres at +-0.09375, +-0.28125, ...; occupied when sd(centre) <= 0.09375
    pose, half = _box_world([0.15, 0.15, 0.15])
    occ = SD.occupancy(pose, half)[0].reshape(8, 8, 8)  # [z, y, x]
    want = np.zeros((8, 8, 8))
    want[3:5, 3:5, 3:5] = 1.0  # the 8 central voxels contain the centre-most points; neighbours are 0.13 m away
    np.testing.assert_array_equal(occ, want)
    # half extent 0.2: face neighbours are 0.28125 - 0.2 = 0.08125 away (occupied), edge neighbours
    # sqrt(2) * 0.08125 = 0.115 (free): 8 central + 6 faces x 4 = 32 voxels
    pose, half = _box_world([0.2, 0.2, 0.2])
    occ = SD.occupancy(pose, half)[0].reshape(8, 8, 8)
    assert occ.sum() == 32
    assert occ[3, 3, 2] == 1 and occ[3, 2, 2] == 0 and occ[2, 2, 2] == 0


def test_occupancy_rotates_with_the_world():
    pr = make_seed_problems(2, 5, split=3)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # (x, y) -> (-y, x)
    pose = pr.worlds.pose.copy()
    rot = pose.copy()
    rot[..., :3] = Rz @ pose[..., :3]
    rot[..., 3] = pose[..., 3] @ Rz.T
    a = SD.occupancy(pose, pr.worlds.half_ext).reshape(-1, 8, 8, 8)   # [w, z, y, x]
    b = SD.occupancy(rot, pr.worlds.half_ext).reshape(-1, 8, 8, 8)
    # the centre (x, y) goes to (-y, x): voxel (x, y) -> (7 - y, x)
    want = np.zeros_like(a)
    for x in range(8):
        for y in range(8):
            want[:, :, x, 7 - y] = a[:, :, y, x]
    np.testing.assert_array_equal(b, want)


def _torch_net(params):
    layers = []
    for l, (fi, fo) in enumerate(SD.LAYERS, 1):
        lin = torch.nn.Linear(fi, fo, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.tensor(params[f"W{l}"].T))
            lin.bias.copy_(torch.tensor(params[f"b{l}"]))
        layers.append(lin)
        if l < 4:
            layers.append(torch.nn.GELU(approximate="none"))
    return torch.nn.Sequential(*layers)


def test_forward_matches_torch_layers():
    params = make_seednet_params()
    x = np.random.default_rng(1).normal(size=(5, SD.N_IN))
    y, _ = SD.forward(params, x)
    ref = _torch_net(params)(torch.tensor(x)).detach().numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-13)


def test_backward_matches_torch_autograd_and_central_differences():
    params = make_seednet_params()
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, SD.N_IN))
    targets = rng.normal(scale=0.5, size=(3, 8, 32, 7))
    valid = np.ones((3, 8))
    valid[1, 5] = 0
    y, cache = SD.forward(params, x)
    L, dy, assign = SD.loss(y, targets, valid)
    g = SD.backward(params, cache, dy)
    # torch autograd of the same loss with the assignment fixed
    net = _torch_net(params)
    yt = net(torch.tensor(x)).reshape(3, 8, 224)
    tt = torch.tensor(targets.reshape(3, 8, 224))
    terms = [((yt[n, assign[n, j]] - tt[n, j]) ** 2).mean() for n in range(3) for j in range(8) if valid[n, j]]
    Lt = torch.stack(terms).sum() / valid.sum()
    Lt.backward()
    assert abs(float(Lt.detach()) - L) < 1e-12 * max(1.0, abs(L))
    for l, mod in zip((1, 2, 3, 4), (0, 2, 4, 6)):
        np.testing.assert_allclose(g[f"W{l}"], net[mod].weight.grad.numpy().T, rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(g[f"b{l}"], net[mod].bias.grad.numpy(), rtol=1e-9, atol=1e-14)
    # central differences on a few entries of every tensor (assignment is stable for small steps)
    h = 1e-6
    for name in ("W1", "b2", "W3", "W4", "b4"):
        idx = tuple(rng.integers(0, s) for s in params[name].shape)
        p_hi = {k: v.copy() for k, v in params.items()}
        p_lo = {k: v.copy() for k, v in params.items()}
        p_hi[name][idx] += h
        p_lo[name][idx] -= h
        fd = (SD.loss(SD.forward(p_hi, x)[0], targets, valid)[0] - SD.loss(SD.forward(p_lo, x)[0], targets, valid)[0]) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-6 * max(1e-3, abs(fd)), (name, fd, g[name][idx])


def test_loss_is_a_min_over_slots():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(2, SD.N_OUT))
    targets = rng.normal(size=(2, 8, 32, 7))
    valid = np.ones((2, 8))
    L, _, assign = SD.loss(y, targets, valid)
    # brute force
    yp = y.reshape(2, 8, 224)
    tt = targets.reshape(2, 8, 224)
    tot = 0.0
    for n in range(2):
        for j in range(8):
            errs = [np.mean((yp[n, s] - tt[n, j]) ** 2) for s in range(8)]
            tot += min(errs)
            assert assign[n, j] == int(np.argmin(errs))
    assert abs(L - tot / 16) < 1e-14
    # invariant under a permutation of the predicted slots; zero when every target is predicted
    perm = rng.permutation(8)
    L2, _, _ = SD.loss(yp[:, perm].reshape(2, -1), targets, valid)
    assert abs(L2 - L) < 1e-14
    L3, dy3, _ = SD.loss(tt[:, perm].reshape(2, -1), targets, valid)
    assert L3 == 0.0 and not np.any(dy3)


def test_adam_first_steps_closed_form():
    # with a constant gradient g the bias-corrected moments are g and g^2 at every step, so each
    # step moves w by lr * g / (|g| + eps)
    p = {"w": np.array([0.3, -0.2, 0.0])}
    g = {"w": np.array([0.5, -2.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    lr, eps = 1e-2, 1e-8
    w = p["w"].copy()
    for step in (1, 2, 3):
        p, m, v = SD.adam(p, g, m, v, step, lr=lr, eps=eps)
        w = w - lr * g["w"] / (np.abs(g["w"]) + eps)
        np.testing.assert_allclose(p["w"], w, rtol=1e-12, atol=1e-15)


def test_emulation_stores_bf16_operands():
    params = make_seednet_params()
    x = np.random.default_rng(4).normal(size=(4, SD.N_IN))
    y, cache = SD.forward(params, x, emulate=True)
    for l in range(4):
        a = cache[f"a{l}"]
        np.testing.assert_array_equal(SD.bf16(a), a)
    # BF16 keeps 8 significant bits: round to nearest moves a value by at most 2^-8 of it
    z = np.random.default_rng(5).normal(size=1000)
    rel = np.abs(SD.bf16(z) - z) / np.abs(z)
    assert rel.max() <= 2.0 ** -8 and rel.max() > 2.0 ** -9


def test_seeds_pin_the_endpoints():
    rng = np.random.default_rng(6)
    start, goal = rng.uniform(-2, 2, size=(3, 7)), rng.uniform(-2, 2, size=(3, 7))
    s = SD.seeds(rng.normal(size=(3, SD.N_OUT)), start, goal)
    np.testing.assert_array_equal(s[:, :, 0], np.broadcast_to(start[:, None], (3, 8, 7)))
    np.testing.assert_allclose(s[:, :, -1], np.broadcast_to(goal[:, None], (3, 8, 7)), atol=1e-15)
    line = SD.straight_line(start, goal)
    np.testing.assert_allclose(line[:, 16], start + (goal - start) * 16 / 31, atol=1e-15)
