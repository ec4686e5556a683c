"""Reference encoder/decoder for the reduced floating-point storage formats.  TEST INFRASTRUCTURE.

The paper stores large FP32 tensors in narrower ExMy floating-point formats (E exponent bits, M
mantissa bits, one sign bit; Sec. IV-A) and converts FP32 to FP16 with round-to-nearest on write
and back to FP32 on read (Sec. V-B).  It fixes neither exponent bias, nor special values, nor the
overflow rule; the readings used here are:

  id name  E  M  bias  max finite   specials              overflow / Inf input
  0  f32   8 23  127   3.40e38      Inf, NaN              identity (no conversion)
  1  f16   5 10   15   65504        Inf, NaN              IEEE: |x| >= 65520 -> Inf
  2  bf16  8  7  127   3.39e38      Inf, NaN              IEEE: round-to-nearest, overflow -> Inf
  3  e4m3  4  3    7   448          NaN = S.1111.111      saturate to +-448 (Inf too)
  4  e5m2  5  2   15   57344        Inf, NaN codes exist  saturate to +-57344 (Inf too)
  5  e3m2  3  2    3   28           none                  saturate to +-28
  6  e2m1  2  1    1   6            none                  saturate to +-6

Every format keeps subnormals (exponent field 0: value m * 2^(1-bias-M)) and signed zero.
Rounding is to the nearest representable value, ties to the code with an even mantissa LSB.
NaN inputs give a NaN code where the format has one (which NaN code is not part of the contract)
and are outside the contract for e3m2/e2m1.

Per-tensor scale (not in the paper; restricted to powers of two so that scaling is exact):
  write  code = enc(fp32(fp32(x) * 2^-k))     read  x_hat = fp32(dec(code) * 2^k)
with -16 <= k <= 16 and k = 0 for f32.

Packed layout: element i occupies bits [b*i, b*i + b) of a little-endian bit stream (bit j of the
stream is bit j%8 of byte j//8).  For b = 8, 16, 32 this is the ordinary little-endian array.

Parity pins (tests/test_oracle_formats.py): every code decodes to the value of the format formula,
enc(dec(c)) == c for all non-NaN codes, exact midpoints go to the even code, monotonicity,
saturation thresholds; f16 against numpy.float16, bf16/e4m3/e5m2 in range against torch casts;
e3m2/e2m1 by the definition alone.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
from typing import Dict, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Format:
    fid: int
    name: str
    E: int
    M: int
    bias: int
    has_inf: bool      # exponent field all ones with zero mantissa is +-Inf
    has_nan: bool
    saturate: bool     # True: finite overflow and Inf inputs saturate to +-max finite

    @property
    def bits(self) -> int:
        return 1 + self.E + self.M

    @property
    def sign_bit(self) -> int:
        return 1 << (self.E + self.M)


FORMATS: Dict[str, Format] = {
    "f32": Format(0, "f32", 8, 23, 127, True, True, False),
    "f16": Format(1, "f16", 5, 10, 15, True, True, False),
    "bf16": Format(2, "bf16", 8, 7, 127, True, True, False),
    "e4m3": Format(3, "e4m3", 4, 3, 7, False, True, True),
    "e5m2": Format(4, "e5m2", 5, 2, 15, True, True, True),
    "e3m2": Format(5, "e3m2", 3, 2, 3, False, False, True),
    "e2m1": Format(6, "e2m1", 2, 1, 1, False, False, True),
}
BY_ID = {f.fid: f for f in FORMATS.values()}
REDUCED = ("f16", "bf16", "e4m3", "e5m2", "e3m2", "e2m1")
SCALE_MIN, SCALE_MAX = -16, 16


def get(fmt) -> Format:
    if isinstance(fmt, Format):
        return fmt
    if isinstance(fmt, (int, np.integer)):
        return BY_ID[int(fmt)]
    return FORMATS[fmt]


def _code_kind(f: Format, mag: int) -> str:
    """'finite', 'inf' or 'nan' for a magnitude code (sign bit stripped)."""
    e, m = mag >> f.M, mag & ((1 << f.M) - 1)
    emax_field = (1 << f.E) - 1
    if f.has_inf and e == emax_field:
        return "inf" if m == 0 else "nan"
    if f.name == "e4m3" and e == emax_field and m == (1 << f.M) - 1:
        return "nan"
    return "finite"


def code_value(f: Format, mag: int) -> Fraction:
    """Exact value of a finite magnitude code, straight from the ExMy formula."""
    e, m = mag >> f.M, mag & ((1 << f.M) - 1)
    if e == 0:
        return Fraction(m, 1 << f.M) * Fraction(2) ** (1 - f.bias)
    return (1 + Fraction(m, 1 << f.M)) * Fraction(2) ** (e - f.bias)


_TABLES: Dict[str, Tuple[np.ndarray, np.ndarray]] = {}


def magnitude_table(fmt) -> Tuple[np.ndarray, np.ndarray]:
    """(codes, values): every finite non-negative magnitude code and its exact value (float64 holds
    each exactly), ascending.  Not available for f32, which is the identity."""
    f = get(fmt)
    if f.name == "f32":
        raise ValueError("f32 has no table")
    if f.name not in _TABLES:
        codes, vals = [], []
        for mag in range(1 << (f.E + f.M)):
            if _code_kind(f, mag) == "finite":
                codes.append(mag)
                vals.append(float(code_value(f, mag)))
        c, v = np.array(codes, dtype=np.int64), np.array(vals, dtype=np.float64)
        assert np.all(np.diff(v) > 0), "codes must be monotone in value"
        _TABLES[f.name] = (c, v)
    return _TABLES[f.name]


def max_finite(fmt) -> float:
    f = get(fmt)
    if f.name == "f32":
        return float(np.finfo(np.float32).max)
    return float(magnitude_table(f)[1][-1])


def _special_code(f: Format, kind: str) -> int:
    emax_field = (1 << f.E) - 1
    if kind == "inf":
        return emax_field << f.M
    if kind == "nan":
        return (1 << (f.E + f.M)) - 1 if f.name == "e4m3" else (emax_field << f.M) | (1 << (f.M - 1))
    raise ValueError(kind)


def encode(x, fmt) -> np.ndarray:
    """Round float32 values (already scaled) to the format: nearest value, ties to the even code.
    Returns integer codes (uint32)."""
    f = get(fmt)
    x = np.asarray(x, dtype=np.float32)
    if f.name == "f32":
        return x.view(np.uint32).copy()
    codes_tab, vals = magnitude_table(f)
    xd = x.astype(np.float64)
    sign = np.signbit(xd)
    a = np.abs(xd)
    nan = np.isnan(a)
    inf = np.isinf(a)
    a_f = np.where(nan | inf, 0.0, a)

    n = vals.shape[0]
    hi = np.searchsorted(vals, a_f, side="left")       # vals[hi-1] < a <= vals[hi]
    hi_c = np.minimum(hi, n - 1)
    lo_c = np.maximum(hi - 1, 0)
    d_hi = vals[hi_c] - a_f
    d_lo = a_f - vals[lo_c]
    take_lo = (d_lo < d_hi) | ((d_lo == d_hi) & (codes_tab[lo_c] % 2 == 0))
    mag = np.where(take_lo, codes_tab[lo_c], codes_tab[hi_c])
    mag = np.where(hi == 0, codes_tab[0], mag)          # a == 0 (vals[0] == 0)

    vmax = vals[-1]
    above = a_f > vmax
    if f.saturate:
        mag = np.where(above | inf, codes_tab[-1], mag)
    else:
        # IEEE: the value after max would be 2^(emax+1) with an even (zero) mantissa, so the
        # midpoint between them and everything above it rounds to that value, which overflows.
        nxt = 2.0 ** ((1 << f.E) - 2 - f.bias + 1)
        mid = 0.5 * (vmax + nxt)
        inf_code = _special_code(f, "inf")
        mag = np.where(above & (a_f >= mid), inf_code, np.where(above, codes_tab[-1], mag))
        mag = np.where(inf, inf_code, mag)
    if f.has_nan:
        mag = np.where(nan, _special_code(f, "nan"), mag)
    else:
        mag = np.where(nan, codes_tab[-1], mag)
    return (mag.astype(np.uint32) | np.where(sign, f.sign_bit, 0).astype(np.uint32))


def decode(codes, fmt) -> np.ndarray:
    """Exact float64 value of each code (Inf/NaN for special codes)."""
    f = get(fmt)
    codes = np.asarray(codes).astype(np.uint32)
    if f.name == "f32":
        return codes.view(np.float32).astype(np.float64)
    mag = (codes & (f.sign_bit - 1)).astype(np.int64)
    lut = np.full(1 << (f.E + f.M), np.nan)
    for c in range(1 << (f.E + f.M)):
        kind = _code_kind(f, c)
        lut[c] = float(code_value(f, c)) if kind == "finite" else (np.inf if kind == "inf" else np.nan)
    v = lut[mag]
    return np.where((codes & f.sign_bit) != 0, -v, v)


def fp32(x) -> np.ndarray:
    """Round float64 values to float32 (round-to-nearest-even, subnormals kept)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def check_scale(fmt, k: int) -> None:
    f = get(fmt)
    if f.name == "f32" and k != 0:
        raise ValueError("f32 takes no scale")
    if not SCALE_MIN <= k <= SCALE_MAX:
        raise ValueError("scale exponent out of range")


def quantize(x, fmt, k: int = 0) -> np.ndarray:
    """Codes of the write path: enc(fp32(fp32(x) * 2^-k))."""
    check_scale(fmt, k)
    x32 = fp32(x)
    y32 = fp32(x32.astype(np.float64) * (2.0 ** -k))
    return encode(y32, fmt)


def dequantize(codes, fmt, k: int = 0) -> np.ndarray:
    """Values of the read path: the float32 value dec(code) * 2^k, returned as float64.  The product
    is exact whenever it lies in float32 range (k >= -16 keeps every subnormal code representable);
    scaled-up BF16 codes beyond float32 range read back as +-Inf."""
    check_scale(fmt, k)
    with np.errstate(over="ignore"):
        return fp32(decode(codes, fmt) * (2.0 ** k)).astype(np.float64)


def roundtrip(x, fmt, k: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """(codes, dequantized float64 values) for float64 inputs x."""
    c = quantize(x, fmt, k)
    return c, dequantize(c, fmt, k)


def boundary_risk(x, fmt, k: int = 0, rel: float = 0.0, abs_: float = 0.0) -> np.ndarray:
    """True where fp32(x) lies within rel*|x| + abs_ (unscaled units) of a rounding decision
    boundary of the format, i.e. where a float32 computation of x that is off by that much may
    legitimately land on the neighbouring code."""
    f = get(fmt)
    x = np.asarray(x, dtype=np.float64)
    if f.name == "f32":
        return np.zeros(x.shape, dtype=bool)
    y = np.abs(fp32(fp32(x).astype(np.float64) * 2.0 ** -k).astype(np.float64))
    tol = (rel * np.abs(x) + abs_) * 2.0 ** -k
    _, vals = magnitude_table(f)
    mids = 0.5 * (vals[1:] + vals[:-1])
    if not f.saturate:
        nxt = 2.0 ** ((1 << f.E) - 2 - f.bias + 1)
        mids = np.append(mids, 0.5 * (vals[-1] + nxt))
    j = np.clip(np.searchsorted(mids, y), 1, mids.shape[0] - 1)
    near = np.minimum(np.abs(y - mids[j - 1]), np.abs(y - mids[j]))
    near = np.minimum(near, np.abs(y - mids[0]))
    # a value whose sign is in doubt can land on either sign of the zero code
    return (near <= tol) | (np.abs(y) <= tol)


def pack(codes, fmt) -> np.ndarray:
    """Little-endian bit-stream packing of integer codes -> uint8 array."""
    f = get(fmt)
    b = f.bits
    codes = np.asarray(codes, dtype=np.uint64).ravel()
    if b in (8, 16, 32):
        dt = {8: "<u1", 16: "<u2", 32: "<u4"}[b]
        return codes.astype(dt).view(np.uint8).copy()
    bits = ((codes[:, None] >> np.arange(b, dtype=np.uint64)[None, :]) & 1).astype(np.uint8).ravel()
    return np.packbits(bits, bitorder="little")


def unpack(data, fmt, n: int) -> np.ndarray:
    """Inverse of `pack` for n codes."""
    f = get(fmt)
    b = f.bits
    data = np.asarray(data, dtype=np.uint8).ravel()
    if b in (8, 16, 32):
        dt = {8: "<u1", 16: "<u2", 32: "<u4"}[b]
        return data[: n * b // 8].view(dt).astype(np.uint32)
    bits = np.unpackbits(data, bitorder="little")[: n * b].reshape(n, b).astype(np.uint32)
    return (bits << np.arange(b, dtype=np.uint32)[None, :]).sum(axis=1).astype(np.uint32)


def packed_nbytes(fmt, n: int) -> int:
    return (get(fmt).bits * n + 7) // 8


def ulp_at(x, fmt, k: int = 0) -> np.ndarray:
    """Width of the interval between the two representable values that enclose |x| (unscaled
    units; at a representable value, the gap below it; for f32, numpy's spacing above fp32(|x|),
    which is never smaller).  Rounding to nearest moves an in-range x by at most half of it: the
    per-element term of the first-order error budget (oracle/budget.py)."""
    f = get(fmt)
    x = np.asarray(x, dtype=np.float64)
    if f.name == "f32":
        return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)
    _, vals = magnitude_table(f)
    y = np.abs(x) * 2.0 ** -k
    j = np.clip(np.searchsorted(vals, y), 1, vals.shape[0] - 1)
    gap = vals[j] - vals[j - 1]
    return gap * 2.0 ** k
