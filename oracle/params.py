"""Oracle: scheme parameters derived from (n, p, L, q_bits, K, p_bits).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper fixes a ring degree n (a power of two), a plaintext prime p with
p = 1 mod 2n so that the plaintext ring splits into a 2 x (n/2) slot matrix
(Sec. 5.1), and a ciphertext modulus that it describes only as a product of
a few word-sized primes (Sec. 6.1). The readings below fix the rest:

* ciphertext primes q_1 > ... > q_L: the L largest primes below 2^q_bits with
  q = 1 mod 2n, in descending order; special primes p_1 > ... > p_K: the K
  largest primes below 2^p_bits with the same congruence, skipping any q_i;
* Q = prod q_i, P = prod p_k, Delta = floor(Q / p) (BFV scaling factor);
* zeta = the least x >= 2 with x^n = -1 (mod p): a primitive 2n-th root of
  unity mod p that fixes the slot map;
* key-switching digits: alpha = K consecutive ciphertext primes per digit,
  dnum = L / alpha digits.
"""
from dataclasses import dataclass, field
from typing import List

# Miller-Rabin with these bases is deterministic for every integer < 3.3e24.
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(x: int) -> bool:
    if x < 2:
        return False
    for b in _MR_BASES:
        if x % b == 0:
            return x == b
    d, r = x - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        y = pow(a, d, x)
        if y in (1, x - 1):
            continue
        for _ in range(r - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def largest_ntt_primes(bits: int, count: int, two_n: int, exclude=()) -> List[int]:
    """The `count` largest primes below 2^bits congruent to 1 mod two_n, descending."""
    out = []
    x = ((1 << bits) - 1) // two_n * two_n + 1
    if x >= (1 << bits):
        x -= two_n
    while len(out) < count:
        if x < 2:
            raise ValueError("not enough primes")
        if x not in exclude and is_prime(x):
            out.append(x)
        x -= two_n
    return out


def primitive_2n_root(n: int, q: int) -> int:
    """Least x >= 2 with x^n = -1 mod q (then x has order exactly 2n)."""
    x = 2
    while pow(x, n, q) != q - 1:
        x += 1
    return x


@dataclass
class Params:
    n: int
    p: int
    L: int
    q_bits: int
    K: int
    p_bits: int
    sigma: float = 3.2
    q: List[int] = field(default_factory=list)      # ciphertext primes
    sp: List[int] = field(default_factory=list)     # special primes
    Q: int = 0
    P: int = 0
    delta: int = 0
    zeta: int = 0
    alpha: int = 0
    dnum: int = 0

    @property
    def nh(self) -> int:            # slots per row
        return self.n // 2

    @property
    def qp(self) -> List[int]:      # full key-switching basis, Q limbs then P limbs
        return self.q + self.sp

    def digit_limbs(self, j: int) -> List[int]:
        return list(range(j * self.alpha, (j + 1) * self.alpha))


def make_params(n, p, L, q_bits, K, p_bits, sigma=3.2) -> Params:
    if n & (n - 1) or n < 2:
        raise ValueError("n must be a power of two")
    if (p - 1) % (2 * n) or not is_prime(p):
        raise ValueError("p must be a prime = 1 mod 2n")
    if K < 1 or L % K:
        raise ValueError("L must be a multiple of K (digits of K primes)")
    pr = Params(n=n, p=p, L=L, q_bits=q_bits, K=K, p_bits=p_bits, sigma=sigma)
    pr.q = largest_ntt_primes(q_bits, L, 2 * n)
    pr.sp = largest_ntt_primes(p_bits, K, 2 * n, exclude=set(pr.q))
    pr.Q = 1
    for x in pr.q:
        pr.Q *= x
    pr.P = 1
    for x in pr.sp:
        pr.P *= x
    pr.delta = pr.Q // p
    pr.zeta = primitive_2n_root(n, p)
    pr.alpha = K
    pr.dnum = L // K
    return pr


# The ring/modulus settings of the workloads (ring degree n, plaintext prime p,
# L ciphertext primes of q_bits, K special primes of p_bits).
WORKLOADS = {
    "plain-4096": dict(n=4096, p=65537, L=2, q_bits=54, K=1, p_bits=60),
    "single-32768": dict(n=1 << 15, p=65537, L=14, q_bits=55, K=2, p_bits=60),
    "large-65536": dict(n=1 << 16, p=786433, L=24, q_bits=55, K=3, p_bits=60),
}
