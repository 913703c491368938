"""Oracle: the SIMD slot structure of the plaintext ring (Sec. 5.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With p = 1 mod 2n, X^n + 1 splits into n linear factors mod p and
Z_p[X]/(X^n+1) is isomorphic to Z_p^(2 x n/2) (Sec. 5.1). The paper does not
fix which evaluation point sits in which slot; the reading used here is:

    slot (r, c), r in {0, 1}, 0 <= c < n/2  <->  m(zeta^e(r,c)),
    e(r, c) = (-1)^r * 3^c mod 2n,

zeta = least x >= 2 with x^n = -1 mod p. 3 has order n/2 modulo 2n and -1 is
not a power of 3, so the e(r, c) run over all odd residues exactly once.
With this map the automorphism X -> X^(3^r) moves every row left by r and
X -> X^(2n-1) swaps the two rows, which are the rotations the paper uses.

A record rho (0-based) of a vector of length N = n_ct * n lives in ciphertext
rho div n, row (rho mod n) div (n/2), column rho mod (n/2).
"""
import numpy as np

from .ring import lib, _ptr


def exponent(n, r, c):
    e = pow(3, c, 2 * n)
    return e if r == 0 else (2 * n - e) % (2 * n)


def slot_exponents(n):
    """e[r][c] as an int64 array of shape (2, n/2)."""
    nh = n // 2
    out = np.empty((2, nh), dtype=np.int64)
    e = 1
    for c in range(nh):
        out[0, c] = e
        out[1, c] = (2 * n - e) % (2 * n)
        e = e * 3 % (2 * n)
    return out


def _evaluations_to_slots(ev, n):
    # ev[i] = m(zeta^(2i+1))
    ex = slot_exponents(n)
    return ev[(ex - 1) // 2]


def decode(coeffs, pr):
    """Plaintext polynomial (coefficients mod p, length n) -> slot matrix (2, n/2)."""
    a = np.array([int(x) % pr.p for x in coeffs], dtype=np.uint64)
    lib().o_ntt(_ptr(a), pr.n, pr.p, pr.zeta)
    return _evaluations_to_slots(a, pr.n)


def encode(slots, pr):
    """Slot matrix (2, n/2) of values mod p -> coefficients m_0..m_{n-1} in [0, p).

    m is the unique polynomial of degree < n with m(zeta^e(r,c)) = slots[r][c]."""
    slots = np.asarray(slots)
    ex = slot_exponents(pr.n)
    ev = np.empty(pr.n, dtype=np.uint64)
    ev[(ex - 1) // 2] = np.asarray(slots, dtype=np.uint64) % np.uint64(pr.p)
    lib().o_intt(_ptr(ev), pr.n, pr.p, pr.zeta)
    return ev


def encode_closed_form(slots, n, p, zeta):
    """m_i = n^-1 * sum over odd e of slot(e) * zeta^(-e i)  (O(n^2); small n only)."""
    ex = slot_exponents(n)
    ninv = pow(n, -1, p)
    zinv = pow(zeta, -1, p)
    out = []
    for i in range(n):
        acc = 0
        for r in range(2):
            for c in range(n // 2):
                acc += int(slots[r][c]) * pow(zinv, int(ex[r, c]) * i, p)
        out.append(acc * ninv % p)
    return out


def centered(x, p):
    """Representative of x mod p in (-p/2, p/2]."""
    x %= p
    return x - p if x > p // 2 else x


def record_position(rho, n):
    """(ciphertext, row, column) of 0-based record rho."""
    nh = n // 2
    return rho // n, (rho % n) // nh, rho % nh


def vector_to_slot_matrices(vec, n, n_ct):
    """Lay a length-N vector (N <= n_ct * n) out as n_ct slot matrices (zero padded)."""
    full = np.zeros(n_ct * n, dtype=np.uint64)
    full[:len(vec)] = np.asarray(vec, dtype=np.uint64)
    return full.reshape(n_ct, 2, n // 2)
