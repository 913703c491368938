"""Oracle: seeded randomness of key generation and encryption.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper leaves the scheme's randomness to its HE library (Sec. 6.1). For
ciphertexts to be reproducible bit for bit, every random value is drawn from
SHAKE-128 (FIPS 202) in a fixed framing:

    stream(seed, tag, obj, limb, block) =
        SHAKE128(seed[32] || tag[8] || le64(obj) || le64(limb) || le64(block))

One stream serves one block of 256 consecutive coefficients. `tag` is an ASCII
name padded with zero bytes to 8 bytes; `limb` is the index of the prime in the
basis q_1..q_L, p_1..p_K for per-limb samples and 2^64-1 for samples that are
the same integer on every limb.

Samplers (coefficient c of a block takes bytes [c*w, (c+1)*w) of its stream):
* uniform residue mod r (w = 16): the 16 bytes little-endian, mod r; drawn
  independently per limb, so by CRT the element is uniform over the product of
  the primes up to a 2^-64 bias;
* ternary (w = 4): x = le32(bytes); value floor(3x / 2^32) - 1 in {-1, 0, 1};
* discrete Gaussian, sigma = 3.2, |value| <= 19 (w = 8): r = le32(bytes[0:4]),
  magnitude = least k with r < T[k], sign = bit 0 of byte 4 (1 = negative).
  T is the cumulative distribution of |X| for P(X = x) proportional to
  exp(-x^2 / (2 sigma^2)) on -19..19, scaled to 2^32 and rounded to nearest,
  with T[19] = 2^32 (see cdt_table).
"""
import hashlib
from decimal import Decimal, getcontext

import numpy as np

BLOCK = 256
ALL_LIMBS = (1 << 64) - 1
GAUSS_TAIL = 19


def tag8(name: str) -> bytes:
    b = name.encode("ascii")
    if len(b) > 8:
        raise ValueError("tag longer than 8 bytes")
    return b + b"\0" * (8 - len(b))


def stream(seed: bytes, tag: str, obj: int, limb: int, block: int, nbytes: int) -> bytes:
    if len(seed) != 32:
        raise ValueError("seed must be 32 bytes")
    msg = seed + tag8(tag) + obj.to_bytes(8, "little") + limb.to_bytes(8, "little") \
        + block.to_bytes(8, "little")
    return hashlib.shake_128(msg).digest(nbytes)


def uniform_limb(seed, tag, obj, limb, modulus, n):
    """n residues uniform mod `modulus` for limb index `limb` (coefficient domain)."""
    out = np.empty(n, dtype=np.uint64)
    for blk in range(n // BLOCK):
        raw = np.frombuffer(stream(seed, tag, obj, limb, blk, 16 * BLOCK), dtype="<u8")
        lo = raw[0::2].astype(object)
        hi = raw[1::2].astype(object)
        out[blk * BLOCK:(blk + 1) * BLOCK] = ((hi * (1 << 64) + lo) % modulus).astype(np.uint64)
    return out


def ternary(seed, tag, obj, n):
    """n signed integers in {-1, 0, 1} (int64)."""
    out = np.empty(n, dtype=np.int64)
    for blk in range(n // BLOCK):
        x = np.frombuffer(stream(seed, tag, obj, ALL_LIMBS, blk, 4 * BLOCK), dtype="<u4")
        out[blk * BLOCK:(blk + 1) * BLOCK] = ((3 * x.astype(np.uint64)) >> np.uint64(32)).astype(np.int64) - 1
    return out


def cdt_table(sigma: float = 3.2):
    """Cumulative table of |X| for the discrete Gaussian, 60 decimal digits,
    scaled to 2^32 and rounded to nearest; T[19] = 2^32."""
    getcontext().prec = 60
    s = Decimal(repr(sigma))
    rho = [(-(Decimal(x * x)) / (2 * s * s)).exp() for x in range(GAUSS_TAIL + 1)]
    total = rho[0] + 2 * sum(rho[1:])
    table, acc = [], Decimal(0)
    for k in range(GAUSS_TAIL + 1):
        acc += rho[0] if k == 0 else 2 * rho[k]
        table.append(int(acc / total * (1 << 32) + Decimal("0.5")))
    table[GAUSS_TAIL] = 1 << 32
    return table


_CDT = None


def gaussian(seed, tag, obj, n, sigma=3.2):
    """n signed integers from the tail-cut discrete Gaussian (int64)."""
    global _CDT
    if _CDT is None:
        _CDT = np.array(cdt_table(sigma), dtype=np.uint64)
    out = np.empty(n, dtype=np.int64)
    for blk in range(n // BLOCK):
        raw = np.frombuffer(stream(seed, tag, obj, ALL_LIMBS, blk, 8 * BLOCK), dtype=np.uint8)
        raw = raw.reshape(BLOCK, 8)
        r = raw[:, 0:4].copy().view("<u4").reshape(BLOCK).astype(np.uint64)
        neg = (raw[:, 4] & 1).astype(bool)
        mag = np.searchsorted(_CDT, r, side="right").astype(np.int64)  # least k with r < T[k]
        out[blk * BLOCK:(blk + 1) * BLOCK] = np.where(neg, -mag, mag)
    return out
