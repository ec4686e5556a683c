"""Writes tests/golden/codec_hashes.json: for every reduced format and every one of the 256 chunks of
2^24 consecutive float32 bit patterns, the xxh3-64 digest of the reference encoder's codes at scale
exponent 0.  Codes are hashed unpacked (little-endian uint16 for 16-bit formats, uint8 otherwise)
and the positions of NaN inputs are set to 0, since which NaN code a NaN maps to is not part of the
contract.  Calls only the oracle.  Usage: python tests/golden/make_codec_hashes.py [workers]
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np
import xxhash

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import formats as F  # noqa: E402

CHUNK_BITS = 24
N_CHUNKS = 1 << (32 - CHUNK_BITS)


def chunk_inputs(c: int) -> np.ndarray:
    return (np.arange(1 << CHUNK_BITS, dtype=np.uint32) + np.uint32(c << CHUNK_BITS)).view(np.float32)


def canonical_codes(codes: np.ndarray, x: np.ndarray, fmt: str) -> np.ndarray:
    codes = np.where(np.isnan(x), 0, codes)
    return codes.astype("<u2" if F.get(fmt).bits == 16 else "u1")


def digest(fmt_chunk):
    fmt, c = fmt_chunk
    x = chunk_inputs(c)
    codes = canonical_codes(F.encode(x, fmt), x, fmt)
    return fmt, c, xxhash.xxh3_64_hexdigest(codes.tobytes())


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    jobs = [(f, c) for f in F.REDUCED for c in range(N_CHUNKS)]
    out = {f: [None] * N_CHUNKS for f in F.REDUCED}
    with Pool(workers) as pool:
        for i, (f, c, h) in enumerate(pool.imap_unordered(digest, jobs, chunksize=4)):
            out[f][c] = h
            if i % 128 == 0:
                print(f"{i}/{len(jobs)}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "codec_hashes.json")
    with open(path, "w") as fh:
        json.dump({"chunk_bits": CHUNK_BITS, "scale_exp": 0, "hash": "xxh3_64", "codes": out}, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
