"""Generic ExMy rounding: the paper's full format space, emulated.  TEST INFRASTRUCTURE.

The paper searches 21 floating-point types from FP4 to FP32, each one sign bit, E exponent bits and
M mantissa bits (Sec. IV-A), and evaluates them by quantising every stored tensor to the type and
back to FP32 at each kernel invocation (Sec. IV-B).  It names 13 of the 21 in its results
(Table II): E2M1, E2M2, E3M1, E2M3, E3M2, E4M3, E5M2, E6M6, E5M9, E6M8, E5M10, E8M7, and E8M23
(FP32); it states that exactly three of them (E5M10, E8M7, E8M23) are 16 bits or wider, and lists
FP4, FP5, FP6, FP8, FP10, FP16 and FP32 as the widths of interest.  Readings used here:

  ladder     the 13 named types plus E1M2 (FP4), E1M3 and E4M0 (FP5), E4M1 (FP6), E3M4 (FP8),
             E5M4 and E4M5 (FP10) and E5M7 (FP13), 21 in all, ordered by width
  bias       2^(E-1) - 1; subnormals kept (exponent field 0)
  specials   E5M10 and every type with 8 exponent bits (E8M7, E8M23, ...) follow IEEE (top exponent
             field reserved for Inf/NaN; a value that rounds past the largest finite one becomes
             Inf): an 8-bit exponent without the reserved field would reach 2^128, beyond the FP32
             values the emulation holds.  Every other type has no Inf or NaN: all exponent fields
             hold finite values and overflow saturates to the largest finite value, Inf inputs too
             (the convention of the FP6/FP4 storage formats)
  rounding   to the nearest representable value, ties to even mantissa
  NaN        passes through as NaN in the rounding; as a code: the quiet NaN (top exponent field,
             mantissa MSB) for the IEEE-like types, outside the contract for the others (they
             store the largest magnitude)
  scale      as for the storage formats: y = fp32(fp32(x) 2^-k), value = fp32(round(y) 2^k)
  codes      sign bit, E exponent bits (the biased exponent, 0 for zero and subnormals) and M
             mantissa bits, sign at bit E + M; b = 1 + E + M bits
  packing    a 32-bit word holds floor(32 / b) codes (one FP32, two FP16, three FP10, four FP8, five
             FP6, six FP5, eight FP4 -- the register packing of Sec. IV-A): code i of a tensor goes
             to word i // q at bits (i % q) b, the top 32 - q b bits of each word stay zero

The rounding of a finite y != 0 with |y| = m 2^e (1 <= m < 2): the grid spacing is
2^(max(e, e_min) - M) with e_min = 1 - bias; |y| is divided by it (exact), rounded half-to-even to an
integer and multiplied back (exact).

Parity pins (tests/test_oracle_exmy.py): E3M2 and E2M1 equal the storage codecs' round trips, E5M10
equals IEEE binary16, E8M7 the bfloat16 round trip and E8M23 the identity, on dense and random
inputs; the largest finite values by formula (E8M4 too); brute-force nearest-value search over every
representable value of small types; exact midpoints to even; monotonicity.  Codes: E5M10, E8M7 and
E8M23 codes equal numpy float16 bits, bfloat16 bits (the top half of FP32) and FP32 bits; E3M2 and
E2M1 codes equal the storage codecs'; every code of small types decodes to the value its fields
give and back to itself; packing places hand-checked words.
"""
from __future__ import annotations

import re
from typing import List, Tuple

import numpy as np


def ieee(E: int, M: int) -> bool:
    return (E, M) == (5, 10) or E == 8


LADDER: List[Tuple[int, int]] = [
    (1, 2), (2, 1),                       # FP4
    (1, 3), (2, 2), (3, 1), (4, 0),       # FP5
    (2, 3), (3, 2), (4, 1),               # FP6
    (3, 4), (4, 3), (5, 2),               # FP8
    (4, 5), (5, 4),                       # FP10
    (5, 7), (6, 6),                       # FP13
    (5, 9), (6, 8),                       # FP15
    (5, 10), (8, 7),                      # FP16
    (8, 23),                              # FP32
]


def name(E: int, M: int) -> str:
    return f"e{E}m{M}"


def parse(fmt: str) -> Tuple[int, int]:
    """'eXmY' -> (X, Y); 'f32', 'f16', 'bf16' -> their (E, M)."""
    alias = {"f32": (8, 23), "f16": (5, 10), "bf16": (8, 7)}
    if fmt in alias:
        return alias[fmt]
    m = re.fullmatch(r"e(\d+)m(\d+)", fmt)
    if not m:
        raise ValueError(f"not an ExMy format: {fmt}")
    E, M = int(m.group(1)), int(m.group(2))
    check(E, M)
    return E, M


def check(E: int, M: int) -> None:
    if not (1 <= E <= 8 and 0 <= M <= 23):
        raise ValueError("ExMy needs 1 <= E <= 8 and 0 <= M <= 23")


def bits(E: int, M: int) -> int:
    return 1 + E + M


def limits(E: int, M: int) -> Tuple[int, int, float]:
    """(e_min, e_max, largest finite value)."""
    check(E, M)
    bias = (1 << (E - 1)) - 1
    e_min = 1 - bias
    e_max = ((1 << E) - 2 if ieee(E, M) else (1 << E) - 1) - bias
    return e_min, e_max, (2.0 - 2.0 ** -M) * 2.0 ** e_max


def round_value(y, E: int, M: int) -> np.ndarray:
    """Nearest ExMy value of float64 inputs y (float32 values in practice), as float64."""
    y = np.asarray(y, dtype=np.float64)
    e_min, _, vmax = limits(E, M)
    a = np.abs(y)
    fin = np.isfinite(a) & (a > 0)
    _, ex = np.frexp(np.where(fin, a, 1.0))          # a = m 2^ex, 0.5 <= m < 1
    q = np.maximum(ex - 1, e_min) - M                # grid spacing exponent
    r = np.ldexp(np.rint(np.ldexp(np.where(fin, a, 0.0), -q)), q)
    over = r > vmax
    r = np.where(over, np.inf if ieee(E, M) else vmax, r)
    r = np.where(np.isinf(a), np.inf if ieee(E, M) else vmax, r)
    r = np.where(a == 0, 0.0, r)
    out = np.copysign(r, y)
    return np.where(np.isnan(y), np.nan, out)


def roundtrip(x, E: int, M: int, k: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """(float32 bit patterns of the stored values, the values as float64) of the emulated write and
    read of x with scale exponent k."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        y = (x32 * 2.0 ** -k).astype(np.float32).astype(np.float64)
        v = (round_value(y, E, M) * 2.0 ** k).astype(np.float32)
    return v.view(np.uint32), v.astype(np.float64)


def representable(E: int, M: int) -> np.ndarray:
    """Every finite non-negative value of the type, ascending (small types only)."""
    e_min, e_max, _ = limits(E, M)
    vals = [m * 2.0 ** (e_min - M) for m in range(1 << M)]   # zero and subnormals
    for e in range(e_min, e_max + 1):
        vals += [(1.0 + m / (1 << M)) * 2.0 ** e for m in range(1 << M)]
    return np.array(sorted(set(vals)))


def encode(x, E: int, M: int, k: int = 0) -> np.ndarray:
    """Codes (uint32, sign at bit E + M) of the write path: the code of round_value(fp32(fp32(x)
    2^-k)).  Zero keeps its sign; NaN gives the quiet NaN of the IEEE-like types and the largest
    magnitude of the others (outside the contract)."""
    check(E, M)
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        y = (x32 * 2.0 ** -k).astype(np.float32).astype(np.float64)
    r = round_value(y, E, M)
    bias = (1 << (E - 1)) - 1
    e_min = 1 - bias
    sign = np.signbit(r).astype(np.uint64) << np.uint64(E + M)
    a = np.abs(r)
    top = (1 << E) - 1
    nan_code = (top << M) | ((1 << (M - 1)) if M > 0 else 0) if ieee(E, M) else (top << M) | ((1 << M) - 1)
    fin = np.isfinite(a) & (a > 0)
    af = np.where(fin, a, 1.0)
    m, ex = np.frexp(af)                              # af = m 2^ex, 1/2 <= m < 1
    e = ex - 1                                        # af = (2m) 2^e
    normal = e >= e_min
    with np.errstate(invalid="ignore", over="ignore"):   # each branch is exact where it is selected
        mant_n = np.rint((af / np.ldexp(1.0, e) - 1.0) * (1 << M)).astype(np.int64)
        mant_s = np.rint(np.minimum(af / np.ldexp(1.0, e_min - M), 2.0 ** 62)).astype(np.int64)
    mag = np.where(normal, ((e + bias).astype(np.int64) << M) | mant_n, mant_s)
    mag = np.where(a == 0, 0, mag)
    mag = np.where(np.isinf(a), top << M, mag)
    mag = np.where(np.isnan(a), nan_code, mag)
    return (mag.astype(np.uint64) | sign).astype(np.uint32)


def decode(codes, E: int, M: int, k: int = 0) -> np.ndarray:
    """Values (float64) of codes, times 2^k, rounded to FP32 as the read path returns them."""
    check(E, M)
    c = np.asarray(codes).astype(np.int64)
    bias = (1 << (E - 1)) - 1
    mag = c & ((1 << (E + M)) - 1)
    ef = mag >> M
    mant = mag & ((1 << M) - 1)
    v = np.where(ef == 0, mant * np.ldexp(1.0, 1 - bias - M),
                 ((1 << M) + mant) * np.ldexp(1.0, (ef - bias - M).astype(np.int64)))
    if ieee(E, M):
        top = (1 << E) - 1
        v = np.where(ef == top, np.where(mant != 0, np.nan, np.inf), v)
    v = np.where((c >> (E + M)) & 1, -v, v)
    with np.errstate(over="ignore"):
        return (v * 2.0 ** k).astype(np.float32).astype(np.float64)


def per_word(E: int, M: int) -> int:
    """Codes per 32-bit word: floor(32 / b)."""
    return 32 // bits(E, M)


def pack(codes, E: int, M: int) -> np.ndarray:
    """Words (uint32) holding the codes, per_word(E, M) to a word from the low bits up."""
    b, q = bits(E, M), per_word(E, M)
    c = np.asarray(codes, dtype=np.uint64).ravel()
    n_words = (c.shape[0] + q - 1) // q
    padded = np.zeros(n_words * q, dtype=np.uint64)
    padded[: c.shape[0]] = c
    shifts = (np.arange(q, dtype=np.uint64) * np.uint64(b))[None, :]
    return np.bitwise_or.reduce(padded.reshape(n_words, q) << shifts, axis=1).astype(np.uint32)


def unpack(words, E: int, M: int, n: int) -> np.ndarray:
    """Inverse of `pack` for n codes."""
    b, q = bits(E, M), per_word(E, M)
    w = np.asarray(words, dtype=np.uint64).ravel()
    shifts = (np.arange(q, dtype=np.uint64) * np.uint64(b))[None, :]
    mask = np.uint64((1 << b) - 1)
    return ((w[:, None] >> shifts) & mask).ravel()[:n].astype(np.uint32)
