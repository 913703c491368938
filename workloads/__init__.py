"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input generation only -- none of the scheme's or the
compression map's arithmetic -- so that the library and the CPU oracle can be
fed the same arrays without sharing any code path.

The paper's experiments use synthetic sparse vectors of a given length and
sparsity (Sec. 6.2); the workloads below follow that recipe at the ring and
modulus sizes of the benchmark configurations:

* index vector: t ones at distinct positions drawn uniformly (without
  replacement) from the N records, zeros elsewhere;
* value columns: uniform 16-bit integers, or uniform in Z_p for the small
  plain workload (so zero values occur among the matches);
* key and encryption randomness: 32-byte seeds derived from a label and
  integers with SHA-256.
"""
import hashlib
import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Ring:
    n: int
    p: int
    L: int
    q_bits: int
    K: int
    p_bits: int


RINGS = {
    # ring degree 4096, p = 65537, two 54-bit primes + one 60-bit special prime
    "ring-4096": Ring(4096, 65537, 2, 54, 1, 60),
    # ring degree 2^15, p = 65537, 14 x 55-bit + 2 x 60-bit special primes
    "ring-32768": Ring(1 << 15, 65537, 14, 55, 2, 60),
    # ring degree 2^16, p = 786433, 24 x 55-bit + 3 x 60-bit special primes
    "ring-65536": Ring(1 << 16, 786433, 24, 55, 3, 60),
    # small rings for parity tests that exercise groups, streams and bands
    "ring-2048-p12289": Ring(2048, 12289, 4, 54, 2, 60),
    "ring-1024-p12289": Ring(1024, 12289, 2, 54, 1, 60),
    # 60-bit ciphertext primes: the diagonal sums fold every 8 terms
    "ring-1024-q60": Ring(1024, 12289, 2, 60, 1, 61),
    # ten 60-bit primes: room for Power_{p-1} (x^3, then twelve squarings at p = 12289)
    "ring-1024-deep": Ring(1024, 12289, 10, 60, 2, 61),
}


@dataclass(frozen=True)
class Workload:
    name: str
    ring: str
    N: int          # records
    t: int          # matches (ones in the index vector)
    ncol: int       # value columns
    values: str     # "u16" or "zp"


WORKLOADS = {
    "plain-4096": Workload("plain-4096", "ring-4096", 4096, 16, 1, "zp"),
    "single-32768": Workload("single-32768", "ring-32768", 1 << 15, 256, 1, "u16"),
    "large-65536": Workload("large-65536", "ring-65536", 1 << 20, 1024, 4, "u16"),
    "multi-2048": Workload("multi-2048", "ring-2048-p12289", 7 * 2048, 13, 4, "zp"),
    "tiny-1024": Workload("tiny-1024", "ring-1024-p12289", 1024, 5, 1, "zp"),
    # s = 64, B = 8, 2 u-blocks: 16 diagonal terms per sum, more than one fold at 60 bits
    "fold-1024-q60": Workload("fold-1024-q60", "ring-1024-q60", 1024, 40, 1, "zp"),
    # the large workload's ring and moduli with one ciphertext of records and t = 16:
    # small enough for a whole compression on the CPU
    "reduced-65536": Workload("reduced-65536", "ring-65536", 1 << 16, 16, 4, "u16"),
}


def rng_for(*ints):
    return np.random.default_rng(np.random.SeedSequence([0x5EED, *ints]))


def seed32(label: str, *ints) -> bytes:
    h = hashlib.sha256(label.encode())
    for x in ints:
        h.update(int(x).to_bytes(8, "little", signed=False))
    return h.digest()


def index_vector(rng, N, t):
    v = np.zeros(N, dtype=np.uint32)
    if t:
        v[rng.choice(N, size=t, replace=False)] = 1
    return v


def value_columns(rng, N, ncol, kind, p):
    if kind == "u16":
        return rng.integers(0, 1 << 16, size=(ncol, N), dtype=np.uint32)
    if kind == "zp":
        return rng.integers(0, p, size=(ncol, N), dtype=np.uint32)
    raise ValueError(kind)


def query_inputs(wl: Workload, query=0, t=None, N=None):
    """(v, db) for one query of a workload; t / N override the defaults."""
    ring = RINGS[wl.ring]
    N = wl.N if N is None else N
    t = wl.t if t is None else t
    rng = rng_for(zlib_id(wl.name), query)
    v = index_vector(rng, N, t)
    db = value_columns(rng, N, wl.ncol, wl.values, ring.p)
    return v, db


def match_inputs(N, t, p, seed=0):
    """Exact-match workload: N record keys uniform in Z_p \\ {x}, t of them set to the
    query key x (distinct positions); returns (keys, x, index vector)."""
    rng = rng_for(0x3A7C, seed)
    x = int(rng.integers(1, p))
    keys = rng.integers(0, p - 1, size=N, dtype=np.int64)
    keys = np.where(keys >= x, keys + 1, keys)  # every value but x
    v = index_vector(rng, N, t)
    keys = np.where(v == 1, x, keys).astype(np.uint32)
    return keys, x, v


def zlib_id(name):
    return int.from_bytes(hashlib.sha256(name.encode()).digest()[:4], "little")


def batched_queries(count=64, seed=0, max_ct=32, n=1 << 15):
    """Per query: ciphertext count uniform in 1..max_ct, t log-uniform in [16, 1024]."""
    rng = rng_for(0xBA7C, seed)
    out = []
    for _ in range(count):
        n_ct = int(rng.integers(1, max_ct + 1))
        t = int(round(math.exp(rng.uniform(math.log(16), math.log(1024)))))
        out.append((n_ct * n, t))
    return out
