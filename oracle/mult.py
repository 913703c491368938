"""Oracle: ciphertext x ciphertext multiplication, Power and Match (Sec. 3, Alg. 5,
the exact-match predicate of Sec. 4, Alg. 7 step 1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper evaluates Power_{p-1} (v_i^(p-1) is 1 for v_i != 0 and 0 otherwise, by
Fermat's little theorem) to derive the index vector from a sparse vector when no
index vector is at hand (Alg. 5, Comp), and the exact-match predicate
P(x, (k_i, v_i)) = [k_i = x] for Match (the remark on exact-match queries). Both are
homomorphic polynomial evaluations, so they need products of ciphertexts; the
paper's scheme is HElib's BGV, which it does not spell out. Readings here, for BFV:

* product of (a0, a1) and (b0, b1) at the full modulus Q: take the centred lifts
  (representatives in (-Q/2, Q/2)) of all four polynomials, form the three exact
  negacyclic products over the integers, e0 = a0 b0, e1 = a0 b1 + a1 b0,
  e2 = a1 b1, and round each coefficient: z = round(p e / Q) = floor((2 p e + Q) /
  (2 Q)) (no ties: Q is odd and prime to p), reduced mod Q. (z0, z1, z2) decrypts
  under (1, s, s^2) to the slot-wise product;
* relinearisation key: the Galois key's construction with sigma_k(s) replaced by
  s^2 (digit j: b_j = [-a_j s + e_j + P (Q/D_j) [(Q/D_j)^-1]_{D_j} s^2]_{PQ}, tags
  "rk_a" / "rk_e", object = digit); relinearisation key-switches z2 with it as a
  rotation key-switches c1 (ModUp of each digit, inner product over PQ, ModDown),
  adding the results to z0 and z1;
* Power_e: left-to-right binary exponentiation (after the leading bit, square, then
  multiply by the input for every set bit);
* Match of ciphertext i (records i n .. i n + n - 1, keys k_r in its slots): the
  query x in every slot minus the keys' plaintext (c0 - Delta m_k), Power_{p-1},
  and 1 minus the result ((Delta - c0, -c1) with Delta on the constant coefficient:
  the all-ones slot vector is the constant polynomial 1);
* generic Comp (Alg. 5) on ciphertexts of d: v = Power_{p-1}(d) at the full
  modulus, then the compression of the pair (v, d) with d given instead of masked.
"""
import numpy as np

from . import bfv, rng
from .params import largest_ntt_primes
from .ring import Poly, negacyclic_mul_limb
from .slots import encode


def centered_ints(poly):
    """Centred integer coefficients (representatives in (-M/2, M/2]) of a Poly over M."""
    from .bfv import crt
    M = 1
    for m in poly.mods:
        M *= m
    out = []
    for i in range(poly.n):
        x = crt(poly.c[:, i], poly.mods)
        out.append(x - M if x > M // 2 else x)
    return out


def exact_negacyclic(a, b):
    """The exact negacyclic product of integer coefficient lists a, b (length n):
    (a b)_j = sum_{i+k=j} a_i b_k - sum_{i+k=j+n} a_i b_k, computed modulo enough
    word-sized primes and put together by CRT (signed result)."""
    n = len(a)
    bound = max(1, max(abs(x) for x in a)) * max(1, max(abs(x) for x in b)) * n
    need = (2 * bound + 1).bit_length() + 2
    primes = largest_ntt_primes(61, -(-need // 60), 2 * n)
    res = []
    for q in primes:
        la = np.array([x % q for x in a], dtype=np.uint64)
        lb = np.array([x % q for x in b], dtype=np.uint64)
        res.append(negacyclic_mul_limb(la, lb, q))
    M = 1
    for q in primes:
        M *= q
    out = []
    for j in range(n):
        x = bfv.crt([r[j] for r in res], primes)
        out.append(x - M if x > M // 2 else x)
    return out


def tensor(pr, ct_a, ct_b):
    """(z0, z1, z2) = round(p/Q (a0 b0, a0 b1 + a1 b0, a1 b1)) mod Q (see the module text)."""
    a0, a1 = centered_ints(ct_a.c0), centered_ints(ct_a.c1)
    b0, b1 = centered_ints(ct_b.c0), centered_ints(ct_b.c1)
    e0 = exact_negacyclic(a0, b0)
    e1 = [x + y for x, y in zip(exact_negacyclic(a0, b1), exact_negacyclic(a1, b0))]
    e2 = exact_negacyclic(a1, b1)
    Q, p = pr.Q, pr.p
    out = []
    for e in (e0, e1, e2):
        out.append(Poly.from_ints(pr.q, [(2 * p * x + Q) // (2 * Q) for x in e]))
    return out


def relin_keygen(pr, sk, seed):
    """Relinearisation key: the key-switching key from s^2 to s (digits as Galois keys)."""
    mods = pr.qp
    s_qp = sk.on(mods)
    s2 = s_qp * s_qp
    digits = []
    for j in range(pr.dnum):
        a = Poly(mods, np.stack([rng.uniform_limb(seed, "rk_a", j, i, m, pr.n) for i, m in enumerate(mods)]))
        e = Poly.from_ints(mods, rng.gaussian(seed, "rk_e", j, pr.n, pr.sigma))
        g = s2.scale([bfv.gadget_constant(pr, j, m) for m in mods])
        digits.append((e - a * s_qp + g, a))
    return bfv.GaloisKey(1, digits)


def relinearize(pr, z, rk):
    z0, z1, z2 = z
    xs = [bfv.modup(pr, z2, j) for j in range(pr.dnum)]
    T0, T1 = bfv._inner(pr, xs, rk)
    return bfv.Ciphertext(z0 + bfv.moddown(pr, T0), z1 + bfv.moddown(pr, T1))


def mul(pr, ct_a, ct_b, rk):
    """Ciphertext product, relinearised: decrypts to the slot-wise product."""
    return relinearize(pr, tensor(pr, ct_a, ct_b), rk)


def power(pr, ct, e, rk):
    """ct^e slot-wise by left-to-right binary exponentiation (e >= 1)."""
    if e < 1:
        raise ValueError("exponent must be positive")
    acc = ct
    for bit in bin(e)[3:]:
        acc = mul(pr, acc, acc, rk)
        if bit == "1":
            acc = mul(pr, acc, ct, rk)
    return acc


def sub_plain(pr, ct, slots):
    """ct - plaintext: c0 - Delta m, m the encoding of `slots` (canonical in [0, p))."""
    m = encode(slots, pr)
    dm = Poly.from_ints(pr.q, [int(x) * pr.delta for x in m])
    return bfv.Ciphertext(ct.c0 - dm, ct.c1)


def one_minus(pr, ct):
    """1 - ct: (Delta - c0, -c1), Delta on the constant coefficient."""
    one = Poly.from_ints(pr.q, [pr.delta] + [0] * (pr.n - 1))
    return bfv.Ciphertext(one - ct.c0, -ct.c1)


def match(pr, ct_x, keys, rk):
    """Match (Alg. 7 step 1) for the exact-match predicate: ciphertexts of
    v_r = [k_r = x] for the keys `keys` (length N), ciphertext by ciphertext, from a
    ciphertext of x in every slot."""
    from .slots import vector_to_slot_matrices
    N = len(keys)
    n_ct = -(-N // pr.n)
    km = vector_to_slot_matrices(np.asarray(keys, dtype=np.uint64) % pr.p, pr.n, n_ct)
    out = []
    for i in range(n_ct):
        d = sub_plain(pr, ct_x, km[i])
        v = one_minus(pr, power(pr, d, pr.p - 1, rk))
        if (i + 1) * pr.n > N:
            # slots past the last record hold no record: v is multiplied by the 0/1 mask
            # of the records present, so they never count as matches
            valid = vector_to_slot_matrices(np.ones(N - i * pr.n, dtype=np.uint64), pr.n, 1)[0]
            v = bfv.mul_plain(pr, v, bfv.plain_poly(pr, valid))
        out.append(v)
    return out


def compress_generic(pr, sched, cts_d, gks, rk, level=None, out_level=None):
    """Comp of Alg. 5 on ciphertexts of a sparse vector d alone: v = Power_{p-1}(d)
    ciphertext by ciphertext at the full modulus, then the compression of the pair
    (v, d) (one value column, d given rather than masked); sched: make_schedule for
    N records and ncol = 1."""
    from . import compress as C
    if sched.ncol != 1 or len(cts_d) != sched.n_ct:
        raise C.ScheduleError("generic Comp takes one vector d")
    cts_v = [power(pr, ct, pr.p - 1, rk) for ct in cts_d]
    return C.compress(pr, sched, cts_v, None, gks, level=level, out_level=out_level, given=[list(cts_d)])
