"""GPU codec (vapr_quantize / vapr_dequantize) against the reference encoder: bit-exact on every
float32 bit pattern (via the committed per-chunk digests of the oracle's codes), every code decoded
exactly, scaled conversions and ragged tails."""
import json
import os

import numpy as np
import pytest
import xxhash

from oracle import formats as F
from tests.gpu_helpers import need_gpu, torch

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "codec_hashes.json")


def _unpack_dev(packed: "torch.Tensor", fmt: str, n: int) -> np.ndarray:
    """Codes as uint8/uint16 from packed device bytes (unpacking done with torch on the device)."""
    b = F.get(fmt).bits
    if b == 16:
        return packed.view(torch.int16).cpu().numpy().view(np.uint16)
    if b == 8:
        return packed.cpu().numpy()
    if b == 4:
        lo, hi = packed & 0xF, packed >> 4
        return torch.stack([lo, hi], dim=1).reshape(-1)[:n].cpu().numpy()
    # 6 bits: 4 values in 3 bytes
    p = packed[: n * 6 // 8].reshape(-1, 3).to(torch.int32)
    w = p[:, 0] | (p[:, 1] << 8) | (p[:, 2] << 16)
    vals = torch.stack([(w >> (6 * i)) & 0x3F for i in range(4)], dim=1).reshape(-1)
    return vals[:n].to(torch.uint8).cpu().numpy()


@pytest.mark.parametrize("fmt", F.REDUCED)
def test_exhaustive_bit_exact(fmt):
    need_gpu()
    from paper_2310_07854_amd import quantize

    gold = json.load(open(GOLDEN))
    bits = gold["chunk_bits"]
    n = 1 << bits
    base = torch.arange(n, dtype=torch.int64, device="cuda:0")
    bad = []
    for c in range(1 << (32 - bits)):
        v = base + (c << bits)
        u = torch.where(v >= 2 ** 31, v - 2 ** 32, v).to(torch.int32)  # the same 32-bit pattern
        x = u.view(torch.float32)
        codes = _unpack_dev(quantize(x, fmt), fmt, n).copy()
        nan = torch.isnan(x).cpu().numpy()
        if F.get(fmt).has_nan and nan.any():
            # NaN inputs must give a NaN code of the format (which one is not part of the contract)
            assert np.all(np.isnan(F.decode(codes[nan].astype(np.uint32), fmt)))
        codes[nan] = 0
        if xxhash.xxh3_64_hexdigest(codes.tobytes()) != gold["codes"][fmt][c]:
            bad.append(c)
        if c % 64 == 63:
            print(f"[exhaustive] {fmt}: {c + 1} of {1 << (32 - bits)} chunks, {len(bad)} differ", flush=True)
    if bad:
        # show a few concrete mismatches of the first bad chunk, computed by the oracle
        c = bad[0]
        u = (np.arange(n, dtype=np.uint64) + (c << bits)).astype(np.uint32)
        x = u.view(np.float32)
        ref = F.encode(x, fmt)
        got = _unpack_dev(quantize(torch.from_numpy(x).to("cuda:0"), fmt), fmt, n).astype(np.uint32)
        idx = np.nonzero((ref != got) & ~np.isnan(x))[0][:8]
        pytest.fail(f"{fmt}: {len(bad)} chunks differ; first chunk {c}: inputs {x[idx]} oracle {ref[idx]} gpu {got[idx]}")


@pytest.mark.parametrize("fmt", F.REDUCED)
def test_every_code_decodes_exactly(fmt):
    need_gpu()
    from paper_2310_07854_amd import dequantize

    f = F.get(fmt)
    n = 1 << f.bits
    codes = np.arange(n, dtype=np.uint32)
    packed = torch.from_numpy(F.pack(codes, fmt)).to("cuda:0")
    for k in (0, -3, 5):
        got = dequantize(packed, fmt, n, k).cpu().numpy().astype(np.float64)
        ref = F.dequantize(codes, fmt, k)
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan)
        assert np.array_equal(got[~nan], ref[~nan])
        assert np.array_equal(np.signbit(got[~nan]), np.signbit(ref[~nan]))


@pytest.mark.parametrize("fmt", F.REDUCED)
@pytest.mark.parametrize("k", [-7, -1, 4, 16, -16])
def test_scaled_random(fmt, k):
    need_gpu()
    from paper_2310_07854_amd import dequantize, quantize

    rng = np.random.default_rng(abs(k) * 10 + F.get(fmt).fid)
    x = (rng.normal(size=100003) * 2.0 ** rng.integers(-30, 20, 100003)).astype(np.float32)
    got = quantize(torch.from_numpy(x).to("cuda:0"), fmt, k)
    ref = F.quantize(x, fmt, k)
    assert np.array_equal(F.unpack(got.cpu().numpy(), fmt, x.size), ref)
    back = dequantize(got, fmt, x.size, k).cpu().numpy().astype(np.float64)
    refv = F.dequantize(ref, fmt, k)
    fin = np.isfinite(refv)
    assert np.array_equal(back[fin], refv[fin])


@pytest.mark.parametrize("n", [1, 7, 15, 16, 17, 37, 1000, 4099])
def test_ragged_tails(n):
    need_gpu()
    from paper_2310_07854_amd import _lib as L

    lib = L.load()
    rng = np.random.default_rng(n)
    for fmt in F.FORMATS:
        x = torch.from_numpy(rng.normal(size=n).astype(np.float32)).to("cuda:0")
        nb = F.packed_nbytes(fmt, n)
        # sentinel bytes after the packed output must survive
        buf = torch.full((nb + 64,), 0xAB, dtype=torch.uint8, device="cuda:0")
        L.check(lib.vapr_quantize(L.FORMAT_IDS[fmt], 0, x.data_ptr(), buf.data_ptr(), n, None))
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        assert np.all(got[nb:] == 0xAB)
        assert np.array_equal(got[:nb], F.pack(F.quantize(x.cpu().numpy(), fmt, 0), fmt))
        back = torch.full((n + 16,), 7.0, device="cuda:0")
        L.check(lib.vapr_dequantize(L.FORMAT_IDS[fmt], 0, buf.data_ptr(), back.data_ptr(), n, None))
        torch.cuda.synchronize()
        b = back.cpu().numpy()
        assert np.all(b[n:] == 7.0)
        assert np.array_equal(b[:n].astype(np.float64), F.dequantize(F.quantize(x.cpu().numpy(), fmt, 0), fmt, 0))


def test_invalid_arguments_are_rejected():
    need_gpu()
    from paper_2310_07854_amd import VaprError, quantize

    x = torch.zeros(16, device="cuda:0")
    with pytest.raises(VaprError):
        quantize(x, "f32", 1)
    with pytest.raises(VaprError):
        quantize(x, "e4m3", 17)
