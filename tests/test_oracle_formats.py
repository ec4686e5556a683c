"""Pins of the reference encoder (oracle/formats.py) against the format definitions and against
independent library conversions (numpy float16, torch bfloat16 / float8)."""
import numpy as np
import pytest
import torch

from oracle import formats as F

# Value sets written out by hand from the ExMy definitions (sign bit aside), no code shared with
# the oracle.  e2m1: bias 1, subnormal 0.5; e3m2: bias 3, subnormal step 1/16.
E2M1_VALUES = [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
E3M2_VALUES = [0.0, 0.0625, 0.125, 0.1875,
               0.25, 0.3125, 0.375, 0.4375,
               0.5, 0.625, 0.75, 0.875,
               1.0, 1.25, 1.5, 1.75,
               2.0, 2.5, 3.0, 3.5,
               4.0, 5.0, 6.0, 7.0,
               8.0, 10.0, 12.0, 14.0,
               16.0, 20.0, 24.0, 28.0]


def _lib_decode(name, codes):
    codes = np.asarray(codes)
    if name == "f16":
        return codes.astype(np.uint16).view(np.float16).astype(np.float64)
    if name == "bf16":
        return torch.from_numpy(codes.astype(np.int16)).view(torch.bfloat16).double().numpy()
    if name == "e4m3":
        return torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e4m3fn).double().numpy()
    if name == "e5m2":
        return torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e5m2).double().numpy()
    raise KeyError(name)


@pytest.mark.parametrize("name", ["f16", "bf16", "e4m3", "e5m2"])
def test_decode_matches_library_for_every_code(name):
    f = F.get(name)
    codes = np.arange(1 << f.bits, dtype=np.uint32)
    ours = F.decode(codes, name)
    lib = _lib_decode(name, codes)
    nan = np.isnan(lib)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], lib[~nan])
    # signed zero
    assert np.signbit(ours[f.sign_bit]) and not np.signbit(ours[0])


@pytest.mark.parametrize("name,table", [("e2m1", E2M1_VALUES), ("e3m2", E3M2_VALUES)])
def test_decode_matches_hand_table(name, table):
    f = F.get(name)
    codes = np.arange(1 << f.bits, dtype=np.uint32)
    v = F.decode(codes, name)
    half = 1 << (f.bits - 1)
    assert list(v[:half]) == table
    assert list(-v[half:]) == table
    assert F.max_finite(name) == table[-1]


@pytest.mark.parametrize("name", F.REDUCED)
def test_encode_decode_roundtrip_every_code(name):
    f = F.get(name)
    codes = np.arange(1 << f.bits, dtype=np.uint32)
    v = F.decode(codes, name)
    ok = ~np.isnan(v)
    if f.saturate:
        ok &= np.isfinite(v)
    back = F.encode(v[ok].astype(np.float32), name)
    assert np.array_equal(back, codes[ok])


@pytest.mark.parametrize("name", F.REDUCED)
def test_midpoints_round_to_even(name):
    f = F.get(name)
    codes, vals = F.magnitude_table(name)
    mids = 0.5 * (vals[1:] + vals[:-1])
    assert np.array_equal(mids.astype(np.float32).astype(np.float64), mids)  # exact in f32
    enc = F.encode(mids.astype(np.float32), name)
    lo, hi = codes[:-1], codes[1:]
    expect = np.where(lo % 2 == 0, lo, hi)
    assert np.array_equal(enc, expect.astype(np.uint32))
    # one float32 step off the midpoint goes to the nearer value
    up = np.nextafter(mids.astype(np.float32), np.float32(np.inf))
    dn = np.nextafter(mids.astype(np.float32), np.float32(0))
    assert np.array_equal(F.encode(up, name), hi.astype(np.uint32))
    assert np.array_equal(F.encode(dn, name), lo.astype(np.uint32))


@pytest.mark.parametrize("name", F.REDUCED)
def test_overflow_rule(name):
    f = F.get(name)
    vmax = F.max_finite(name)
    codes, vals = F.magnitude_table(name)
    gap = vals[-1] - vals[-2]
    with np.errstate(over="ignore"):
        big = np.array([vmax + gap, 4.0 * vmax, np.inf], dtype=np.float32)
    enc = F.encode(big, name)
    dec = F.decode(enc, name)
    if f.saturate:
        assert np.all(dec == vmax)
        assert np.all(F.decode(F.encode(-big, name), name) == -vmax)
    else:
        assert np.all(np.isinf(dec))
        # IEEE: the overflow threshold is max + half of the next binade's step
        nxt = 2.0 * 2.0 ** np.floor(np.log2(vmax))
        thr = np.float32(0.5 * (vmax + nxt))
        assert np.isinf(F.decode(F.encode(np.array([thr]), name), name)[0])
        assert F.decode(F.encode(np.array([np.nextafter(thr, np.float32(0))]), name), name)[0] == vmax


def _random_f32(n, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    return x[np.isfinite(x)]


def test_f16_matches_numpy_on_random_patterns():
    x = _random_f32(1 << 20, 1)
    x = np.concatenate([x, np.float32(np.random.default_rng(2).normal(size=1 << 18) * 1e-5)])
    ours = F.encode(x, "f16")
    ref = x.astype(np.float16).view(np.uint16).astype(np.uint32)
    assert np.array_equal(ours, ref)


def test_bf16_matches_torch_on_random_patterns():
    x = _random_f32(1 << 20, 3)
    ours = F.encode(x, "bf16")
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16).astype(np.uint32)
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("name,dt", [("e4m3", torch.float8_e4m3fn), ("e5m2", torch.float8_e5m2)])
def test_fp8_matches_torch_in_range(name, dt):
    rng = np.random.default_rng(4)
    vmax = F.max_finite(name)
    x = np.concatenate([rng.uniform(-vmax, vmax, 1 << 18),
                        rng.normal(size=1 << 18) * 2.0 ** rng.integers(-20, 8, 1 << 18)]).astype(np.float32)
    x = x[np.abs(x) <= vmax]
    ours = F.encode(x, name)
    ref = torch.from_numpy(x).to(dt).view(torch.uint8).numpy().astype(np.uint32)
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("name", F.REDUCED)
def test_monotone(name):
    x = np.sort(np.random.default_rng(5).normal(size=200000).astype(np.float32) * 10)
    v = F.decode(F.encode(x, name), name)
    v = np.where(np.isinf(v), np.sign(v) * 1e300, v)
    assert np.all(np.diff(v) >= 0)


def test_scale_and_dequantize():
    c, v = F.roundtrip(np.array([3.0, -3.0, 0.3]), "e2m1", 1)
    assert list(v) == [3.0, -3.0, 0.0]
    c, v = F.roundtrip(np.array([0.3]), "e2m1", -3)  # 0.3 * 8 = 2.4 -> 2
    assert v[0] == 0.25
    with pytest.raises(ValueError):
        F.quantize(np.array([1.0]), "f32", 1)
    with pytest.raises(ValueError):
        F.quantize(np.array([1.0]), "e4m3", 17)


def test_pack_layout_examples():
    assert list(F.pack([1, 2], "e2m1")) == [0x21]
    assert list(F.pack([1, 2, 3, 4], "e3m2")) == [0x81, 0x30, 0x10]
    assert list(F.pack([0x1234], "f16")) == [0x34, 0x12]
    for name in F.FORMATS:
        f = F.get(name)
        codes = np.random.default_rng(6).integers(0, 1 << min(f.bits, 32), size=99, dtype=np.uint64)
        packed = F.pack(codes, name)
        assert packed.size == F.packed_nbytes(name, 99)
        assert np.array_equal(F.unpack(packed, name, 99), codes.astype(np.uint32))


def test_boundary_risk_flags_midpoints():
    x = np.array([1.25, 1.26, 1.0])  # e2m1: 1.25 is the midpoint of 1 and 1.5
    r = F.boundary_risk(x, "e2m1", 0, rel=1e-6)
    assert list(r) == [True, False, False]


def test_f16_round_trip_of_fp64_goes_through_fp32():
    # a float64 value whose direct float16 rounding differs from rounding its float32 rounding
    x = np.float64(1.0) + 2.0 ** -11 + 2.0 ** -40  # just above an f16 midpoint; fp32 drops the tail
    c = F.quantize(np.array([x]), "f16")
    assert F.decode(c, "f16")[0] == 1.0  # fp32(x) is the exact midpoint -> even code 1.0
