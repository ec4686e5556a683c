"""Pins of the generic ExMy rounding (oracle/exmy.py) against the storage codecs, IEEE binary16,
the definition's closed forms and brute force."""
import numpy as np
import pytest

from oracle import exmy as X
from oracle import formats as F


def _inputs(seed=0, n=200_000):
    rng = np.random.default_rng(seed)
    mags = 2.0 ** rng.uniform(-30, 20, size=n) * rng.choice([-1, 1], size=n)
    dense = np.linspace(-70.0, 70.0, 140_001)
    special = np.array([0.0, -0.0, 1e-45, -1e-45, 448.0, 480.0, 65504.0, 65519.99, 65520.0, 3.0e38])
    return F.fp32(np.concatenate([mags, dense, special])).astype(np.float64)


@pytest.mark.parametrize("E,M,fmt", [(3, 2, "e3m2"), (2, 1, "e2m1"), (5, 10, "f16"), (8, 7, "bf16")])
@pytest.mark.parametrize("k", [0, -3, 4])
def test_matches_storage_codecs(E, M, fmt, k):
    x = _inputs(E + M + k)
    _, ref = F.roundtrip(x, fmt, k)
    _, got = X.roundtrip(x, E, M, k)
    np.testing.assert_array_equal(got.astype(np.float32).view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_fp32_is_the_identity_and_f16_is_ieee_binary16():
    x = _inputs(9)
    _, v = X.roundtrip(x, 8, 23)
    np.testing.assert_array_equal(v.astype(np.float32).view(np.uint32), x.astype(np.float32).view(np.uint32))
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    _, v16 = X.roundtrip(x, 5, 10)
    np.testing.assert_array_equal(v16, ref)


def test_largest_finite_values():
    assert X.limits(2, 1)[2] == 6.0 and X.limits(3, 2)[2] == 28.0
    assert X.limits(5, 10)[2] == 65504.0 and X.limits(4, 3)[2] == 480.0     # no NaN code in the generic E4M3
    assert X.limits(6, 6)[2] == (2 - 2 ** -6) * 2.0 ** 32
    assert X.limits(8, 23)[2] == float(np.finfo(np.float32).max)
    # saturation vs IEEE overflow
    assert X.round_value(1e30, 4, 3) == 480.0 and X.round_value(np.inf, 3, 1) == X.limits(3, 1)[2]
    assert np.isinf(X.round_value(65520.0, 5, 10)) and X.round_value(65519.0, 5, 10) == 65504.0


@pytest.mark.parametrize("E,M", [(1, 2), (2, 2), (3, 1), (4, 0), (2, 3), (4, 1), (3, 4)])
def test_brute_force_nearest(E, M):
    vals = X.representable(E, M)
    rng = np.random.default_rng(E * 10 + M)
    y = F.fp32(rng.uniform(0, vals[-1] * 1.01, size=20_000)).astype(np.float64)
    got = X.round_value(y, E, M)
    d = np.abs(y[:, None] - vals[None, :])
    best = d.min(axis=1)
    # every returned value is representable and no representable value is strictly nearer
    assert np.isin(got, vals).all()
    np.testing.assert_array_equal(np.abs(got - y), best)


@pytest.mark.parametrize("E,M", [(2, 2), (3, 1), (5, 4), (6, 6)])
def test_midpoints_go_to_even_and_rounding_is_monotone(E, M):
    vals = X.representable(E, M)[: 2000]
    mids = 0.5 * (vals[1:] + vals[:-1])
    got = X.round_value(mids, E, M)
    idx = np.searchsorted(vals, got)
    lo = np.arange(len(mids))
    # the chosen neighbour has an even index (even mantissa LSB within a binade, and the binade
    # edges 2^e are even codes)
    assert np.all((idx == lo) | (idx == lo + 1))
    def code_of(v):
        e_min, _, _ = X.limits(E, M)
        ex = np.maximum(np.frexp(v)[1] - 1, e_min)
        return np.rint(np.ldexp(v, M - ex)).astype(np.int64)
    assert np.all(code_of(got) % 2 == 0)
    y = np.sort(F.fp32(np.random.default_rng(E).uniform(-vals[-1], vals[-1], size=50_000)).astype(np.float64))
    assert np.all(np.diff(X.round_value(y, E, M)) >= 0)


def test_ladder_is_21_types_from_fp4_to_fp32():
    assert len(X.LADDER) == 21 and len(set(X.LADDER)) == 21
    widths = [X.bits(E, M) for E, M in X.LADDER]
    assert widths == sorted(widths) and widths[0] == 4 and widths[-1] == 32
    assert {(E, M) for E, M in X.LADDER if X.bits(E, M) >= 16} == {(5, 10), (8, 7), (8, 23)}
    assert X.ieee(8, 4) and X.limits(8, 4)[2] == (2 - 2 ** -4) * 2.0 ** 127 and not X.ieee(6, 6)
    named = {(2, 1), (2, 2), (3, 1), (2, 3), (3, 2), (4, 3), (5, 2), (6, 6), (5, 9), (6, 8), (5, 10), (8, 7), (8, 23)}
    assert named <= set(X.LADDER)


# ---- codes and word packing ---------------------------------------------------------------------

def test_codes_of_ieee_types_are_the_library_bit_patterns():
    torch = pytest.importorskip("torch")
    x = _inputs(seed=3)
    x = x[np.isfinite(x)]
    h = np.abs(x) < 65000.0
    assert np.array_equal(X.encode(x[h], 5, 10), x[h].astype(np.float32).astype(np.float16).view(np.uint16))
    assert np.array_equal(X.encode(x, 8, 23), x.astype(np.float32).view(np.uint32))
    bf = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(X.encode(x, 8, 7), bf)
    # Inf and the largest finite values
    assert X.encode(np.array([np.inf, -np.inf, 65504.0]), 5, 10).tolist() == [0x7C00, 0xFC00, 0x7BFF]


@pytest.mark.parametrize("E,M,fmt", [(3, 2, "e3m2"), (2, 1, "e2m1")])
def test_codes_equal_the_storage_codecs(E, M, fmt):
    for k in (0, -3, 4):
        x = _inputs(seed=4 + k)
        x = x[~np.isnan(x)]
        assert np.array_equal(X.encode(x, E, M, k), F.quantize(x, fmt, k))


@pytest.mark.parametrize("E,M", [(1, 2), (2, 2), (3, 1), (1, 3), (4, 0), (2, 3), (4, 1), (3, 4), (4, 5)])
def test_every_code_decodes_to_its_fields_and_back(E, M):
    bias = (1 << (E - 1)) - 1
    for c in range(1 << (1 + E + M)):
        ef, mant, s = (c >> M) & ((1 << E) - 1), c & ((1 << M) - 1), c >> (E + M)
        v = (mant / 2 ** M) * 2.0 ** (1 - bias) if ef == 0 else (1 + mant / 2 ** M) * 2.0 ** (ef - bias)
        v = -v if s else v
        got = X.decode(np.array([c]), E, M)[0]
        assert got == v and np.signbit(got) == bool(s), (E, M, c, got, v)
        assert X.encode(np.array([v]), E, M)[0] == c


@pytest.mark.parametrize("E,M", X.LADDER)
def test_decode_of_encode_is_the_rounding(E, M):
    for k in (0, -5, 3):
        x = _inputs(seed=11 + k)
        fin = ~np.isnan(x)
        _, want = X.roundtrip(x[fin], E, M, k)
        got = X.decode(X.encode(x[fin], E, M, k), E, M, k)
        assert np.array_equal(got, want) and np.array_equal(np.signbit(got), np.signbit(want))


def test_word_packing():
    # E3M1: b = 5, six codes a word; E4M5: b = 10, three codes a word; E2M1: eight codes a word
    codes = np.array([1, 2, 3, 4, 5, 6, 7], dtype=np.uint32)
    w = X.pack(codes, 3, 1)
    assert w.tolist() == [1 | 2 << 5 | 3 << 10 | 4 << 15 | 5 << 20 | 6 << 25, 7]
    assert X.pack(np.array([0x3FF, 1, 0x200, 5]), 4, 5).tolist() == [0x3FF | 1 << 10 | 0x200 << 20, 5]
    assert X.pack(np.arange(8), 2, 1).tolist() == [sum(i << (4 * i) for i in range(8))]
    assert X.per_word(5, 10) == 2 and X.per_word(2, 3) == 5 and X.per_word(8, 23) == 1
    rng = np.random.default_rng(2)
    for E, M in X.LADDER:
        c = rng.integers(0, 1 << X.bits(E, M), size=101).astype(np.uint32)
        assert np.array_equal(X.unpack(X.pack(c, E, M), E, M, 101), c)
