"""Writes tests/golden/exmy_hashes.json: for a few emulated ExMy types (FP5 E3M1 and E2M2, FP10
E5M4, FP13 E6M6: six, six, three and two codes to a packed word) and every one of the 256 chunks of
2^24 consecutive float32 bit patterns, the xxh3-64 digest of the oracle's codes at scale exponent 0
(oracle/exmy.py encode).  Codes are hashed unpacked (uint8 up to 8 bits, little-endian uint16
above), with NaN inputs set to 0: these types have no NaN code, so a NaN's code is outside the
contract.  Calls only the oracle.  Usage: python tests/golden/make_exmy_hashes.py [workers]
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np
import xxhash

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import exmy as X  # noqa: E402

CHUNK_BITS = 24
N_CHUNKS = 1 << (32 - CHUNK_BITS)
TYPES = ["e3m1", "e2m2", "e5m4", "e6m6"]


def chunk_inputs(c: int) -> np.ndarray:
    return (np.arange(1 << CHUNK_BITS, dtype=np.uint32) + np.uint32(c << CHUNK_BITS)).view(np.float32)


def canonical_codes(codes: np.ndarray, x: np.ndarray, E: int, M: int) -> np.ndarray:
    codes = np.where(np.isnan(x), 0, codes)
    return codes.astype("u1" if X.bits(E, M) <= 8 else "<u2")


def digest(job):
    fmt, c = job
    E, M = X.parse(fmt)
    x = chunk_inputs(c)
    codes = canonical_codes(X.encode(x, E, M), x, E, M)
    return fmt, c, xxhash.xxh3_64_hexdigest(codes.tobytes())


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    jobs = [(f, c) for f in TYPES for c in range(N_CHUNKS)]
    out = {f: [None] * N_CHUNKS for f in TYPES}
    with Pool(workers) as pool:
        for i, (f, c, h) in enumerate(pool.imap_unordered(digest, jobs, chunksize=2)):
            out[f][c] = h
            if i % 64 == 0:
                print(f"{i}/{len(jobs)}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exmy_hashes.json")
    with open(path, "w") as fh:
        json.dump({"chunk_bits": CHUNK_BITS, "scale_exp": 0, "hash": "xxh3_64", "codes": out}, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
