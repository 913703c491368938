"""Oracle: RNS BFV with hybrid key switching, written out step by step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper runs its compression on BGV (Sec. 5.1) and needs from the scheme
only slot-wise additions, plaintext multiplications and the rotations Rot_row
and Rot_col. The same slot algebra holds for BFV, which is the scheme here:

* secret s ternary; public key (b, a) = ([-a s + e]_Q, a), a uniform;
* Enc_pk(m) = ([b u + e0 + Delta m]_Q, [a u + e1]_Q), u ternary, e0, e1
  Gaussian, m the plaintext polynomial with coefficients in [0, p);
* Dec(c0, c1) = round(p [c0 + c1 s]_Q / Q) mod p;
* plaintext product (Sec. 2.2 "boxtimes" with a plaintext) multiplies both
  components by the centred lift of the plaintext, coefficients in (-p/2, p/2];
* Galois key for sigma_k, digit j (limbs I_j, D_j = prod_{i in I_j} q_i):
  b_j = [-a_j s + e_j + P (Q/D_j) [(Q/D_j)^-1]_{D_j} sigma_k(s)]_{PQ}, a_j uniform
  over PQ;
* key switching of d in R_Q: X_j = ModUp_j(d) (fast basis conversion of the
  canonical residues on I_j to every other prime of PQ), T = sum_j X_j (b_j, a_j)
  over PQ, then ModDown(T) = (T - Conv_{P->Q}([T]_P)) P^-1 mod Q;
* rotation by sigma_k, plain: (sigma_k(c0), sigma_k(c1)) followed by key
  switching of the second component, added to the first;
* rotation by sigma_k, hoisted: X_j = ModUp_j(c1) once, then for each k
  T = sum_j sigma_k(X_j) (b_j, a_j) and ModDown as above. The two forms decrypt
  alike but differ in bits, since sigma and the basis conversion commute only
  modulo D_j; which rotations are hoisted is fixed by the compression schedule.
"""
import numpy as np

from . import rng
from .ring import Poly, automorphism
from .slots import encode, decode, centered


# ---------------------------------------------------------------------------
# keys and ciphertexts

class SecretKey:
    def __init__(self, s):
        self.s = np.asarray(s, dtype=np.int64)  # coefficients in {-1, 0, 1}

    def on(self, mods):
        return Poly.from_ints(mods, self.s)


class PublicKey:
    def __init__(self, b, a):
        self.b, self.a = b, a


class GaloisKey:
    def __init__(self, k, digits):
        self.k = k
        self.digits = digits  # list of (b_j, a_j), Poly over PQ


class Ciphertext:
    def __init__(self, c0, c1):
        self.c0, self.c1 = c0, c1

    def __eq__(self, o):
        return self.c0 == o.c0 and self.c1 == o.c1

    def __add__(self, o):
        return Ciphertext(self.c0 + o.c0, self.c1 + o.c1)

    def stack(self):
        """[2][L][n] uint64, the layout the library exchanges."""
        return np.stack([self.c0.c, self.c1.c])

    @staticmethod
    def from_stack(arr, mods):
        arr = np.asarray(arr, dtype=np.uint64)
        return Ciphertext(Poly(mods, arr[0].copy()), Poly(mods, arr[1].copy()))


def keygen(pr, seed):
    s = rng.ternary(seed, "sk", 0, pr.n)
    sk = SecretKey(s)
    a = Poly(pr.q, np.stack([rng.uniform_limb(seed, "pk_a", 0, i, qi, pr.n)
                             for i, qi in enumerate(pr.q)]))
    e = Poly.from_ints(pr.q, rng.gaussian(seed, "pk_e", 0, pr.n, pr.sigma))
    b = e - a * sk.on(pr.q)
    return sk, PublicKey(b, a)


def gadget_constant(pr, j, mod):
    """P * (Q/D_j) * [(Q/D_j)^-1 mod D_j], reduced mod `mod`."""
    D = 1
    for i in pr.digit_limbs(j):
        D *= pr.q[i]
    Qh = pr.Q // D
    return pr.P * Qh * pow(Qh % D, -1, D) % mod


def galois_obj(k, j):
    return (k << 16) | j


def galois_keygen(pr, sk, k, seed):
    mods = pr.qp
    s_qp = sk.on(mods)
    sk_rot = automorphism(s_qp, k)
    digits = []
    for j in range(pr.dnum):
        obj = galois_obj(k, j)
        a = Poly(mods, np.stack([rng.uniform_limb(seed, "gk_a", obj, i, m, pr.n)
                                 for i, m in enumerate(mods)]))
        e = Poly.from_ints(mods, rng.gaussian(seed, "gk_e", obj, pr.n, pr.sigma))
        g = sk_rot.scale([gadget_constant(pr, j, m) for m in mods])
        b = e - a * s_qp + g
        digits.append((b, a))
    return GaloisKey(k, digits)


def encrypt_poly(pr, pk, m_coeffs, seed):
    """Encrypt a plaintext polynomial with coefficients in [0, p)."""
    u = Poly.from_ints(pr.q, rng.ternary(seed, "enc_u", 0, pr.n))
    e0 = Poly.from_ints(pr.q, rng.gaussian(seed, "enc_e0", 0, pr.n, pr.sigma))
    e1 = Poly.from_ints(pr.q, rng.gaussian(seed, "enc_e1", 0, pr.n, pr.sigma))
    dm = Poly.from_ints(pr.q, [int(x) * pr.delta for x in m_coeffs])
    c0 = pk.b * u + e0 + dm
    c1 = pk.a * u + e1
    return Ciphertext(c0, c1)


def encrypt(pr, pk, slots, seed):
    """Encrypt a slot matrix (2, n/2) of values in [0, p)."""
    return encrypt_poly(pr, pk, encode(slots, pr), seed)


def crt(residues, mods):
    """Integer in [0, prod mods) with the given residues."""
    M = 1
    for m in mods:
        M *= m
    x = 0
    for r, m in zip(residues, mods):
        Mi = M // m
        x += int(r) * Mi * pow(Mi % m, -1, m)
    return x % M


def phase(pr, sk, ct):
    """[c0 + c1 s]_Q as a list of n integers in [0, Q)."""
    v = ct.c0 + ct.c1 * sk.on(pr.q)
    return [crt(v.c[:, i], pr.q) for i in range(pr.n)]


def decrypt_poly(pr, sk, ct):
    x = phase(pr, sk, ct)
    # round(p x / Q) = floor((2 p x + Q) / (2 Q)); no ties since Q is odd and p < Q
    return [((2 * pr.p * xi + pr.Q) // (2 * pr.Q)) % pr.p for xi in x]


def decrypt(pr, sk, ct):
    return decode(decrypt_poly(pr, sk, ct), pr)


def noise_bits(pr, sk, ct):
    """log2 of max |[c0 + c1 s]_Q - Delta m| (centred), m the decryption."""
    x = phase(pr, sk, ct)
    worst = 0
    for xi in x:
        m = ((2 * pr.p * xi + pr.Q) // (2 * pr.Q)) % pr.p
        v = (xi - pr.delta * m) % pr.Q
        if v > pr.Q // 2:
            v -= pr.Q
        worst = max(worst, abs(v))
    return worst.bit_length()


def noise_budget_bits(pr):
    """log2(Q / (2p)): decryption is correct while the noise stays below this."""
    return (pr.Q // (2 * pr.p)).bit_length() - 1


# ---------------------------------------------------------------------------
# homomorphic operations

def plain_poly(pr, slots):
    """Centred lift of the encoding of `slots` (the plaintext multiplier)."""
    return [centered(int(x), pr.p) for x in encode(slots, pr)]


def mul_plain(pr, ct, m_centered):
    """ct boxtimes plaintext: both components times the centred plaintext."""
    m = Poly.from_ints(ct.c0.mods, m_centered)
    return Ciphertext(ct.c0 * m, ct.c1 * m)


def modup(pr, d, j):
    """Fast basis conversion of digit j of d (residues on I_j) to all of PQ.

    On a prime r outside I_j the result is sum_{i in I_j} y_i (D_j / q_i) mod r
    with y_i = [d_i (D_j/q_i)^-1]_{q_i} fully reduced; on I_j it is d itself."""
    mods = pr.qp
    I = pr.digit_limbs(j)
    D = 1
    for i in I:
        D *= pr.q[i]
    ys = []
    for i in I:
        qi = pr.q[i]
        inv = pow((D // qi) % qi, -1, qi)
        ys.append((d.c[i].astype(object) * inv) % qi)
    out = np.empty((len(mods), pr.n), dtype=np.uint64)
    for r_idx, r in enumerate(mods):
        if r_idx in I:
            out[r_idx] = d.c[r_idx]
            continue
        acc = np.zeros(pr.n, dtype=object)
        for y, i in zip(ys, I):
            acc = acc + y * ((D // pr.q[i]) % r)
        out[r_idx] = (acc % r).astype(np.uint64)
    return Poly(mods, out)


def moddown(pr, T):
    """(T - Conv_{P->Q}([T]_P)) * P^-1 mod each q_i, for T over PQ."""
    L, K = pr.L, pr.K
    ys = []
    for k in range(K):
        pk = pr.sp[k]
        inv = pow((pr.P // pk) % pk, -1, pk)
        ys.append((T.c[L + k].astype(object) * inv) % pk)
    out = np.empty((L, pr.n), dtype=np.uint64)
    for i, qi in enumerate(pr.q):
        conv = np.zeros(pr.n, dtype=object)
        for k in range(K):
            conv = conv + ys[k] * ((pr.P // pr.sp[k]) % qi)
        conv = conv % qi
        diff = (T.c[i].astype(object) - conv) % qi
        out[i] = (diff * pow(pr.P % qi, -1, qi) % qi).astype(np.uint64)
    return Poly(pr.q, out)


def _inner(pr, xs, gk, k_perm=None):
    T0 = Poly.zero(pr.qp, pr.n)
    T1 = Poly.zero(pr.qp, pr.n)
    for j, (b, a) in enumerate(gk.digits):
        x = xs[j] if k_perm is None else automorphism(xs[j], k_perm)
        T0 = T0 + x * b
        T1 = T1 + x * a
    return T0, T1


def rotate(pr, ct, gk):
    """Non-hoisted rotation by sigma_k (k = gk.k) with key switching."""
    c0 = automorphism(ct.c0, gk.k)
    c1 = automorphism(ct.c1, gk.k)
    xs = [modup(pr, c1, j) for j in range(pr.dnum)]
    T0, T1 = _inner(pr, xs, gk)
    return Ciphertext(c0 + moddown(pr, T0), moddown(pr, T1))


def rotate_sum(pr, cts, gks):
    """Sum of the non-hoisted rotations sigma_{k_g}(ct_g), g = 0.., with the key
    products summed over PQ and brought down once: sum_g sigma(c0_g) +
    ModDown(sum_g T0_g), ModDown(sum_g T1_g). Up to ModDown's rounding this is
    sum_g rotate(ct_g); every modular sum is exact, so only the one ModDown rounds."""
    C0 = T0s = T1s = None
    for ct, gk in zip(cts, gks):
        c1 = automorphism(ct.c1, gk.k)
        xs = [modup(pr, c1, j) for j in range(pr.dnum)]
        T0, T1 = _inner(pr, xs, gk)
        c0 = automorphism(ct.c0, gk.k)
        C0 = c0 if C0 is None else C0 + c0
        T0s = T0 if T0s is None else T0s + T0
        T1s = T1 if T1s is None else T1s + T1
    return Ciphertext(C0 + moddown(pr, T0s), moddown(pr, T1s))


def rotate_hoisted(pr, ct, gks):
    """Rotations of one ciphertext by several sigma_k sharing one ModUp."""
    xs = [modup(pr, ct.c1, j) for j in range(pr.dnum)]
    out = []
    for gk in gks:
        T0, T1 = _inner(pr, xs, gk, k_perm=gk.k)
        out.append(Ciphertext(automorphism(ct.c0, gk.k) + moddown(pr, T0), moddown(pr, T1)))
    return out


# ---------------------------------------------------------------------------
# modulus switching (the BFV form of switching to smaller parameters, Sec. 5.3)

def at_level(pr, level, keyswitch=True):
    """Parameters of the ring restricted to the first `level` ciphertext primes:
    Q' = q_1 ... q_level, same special primes. Key switching needs whole digits,
    so `level` must be a multiple of the digit size unless keyswitch is False (a
    ciphertext that is only decrypted, such as a mod-switched output)."""
    import copy
    if not 0 < level <= pr.L or (keyswitch and level % pr.alpha):
        raise ValueError("level must be in [1, L] (a multiple of the digit size for key switching)")
    lo = copy.copy(pr)
    lo.L = level
    lo.q = pr.q[:level]
    lo.Q = 1
    for x in lo.q:
        lo.Q *= x
    lo.delta = lo.Q // pr.p
    lo.dnum = level // pr.alpha
    return lo


def key_at_level(pr, gk, level):
    """A Galois key restricted to the first `level` ciphertext primes, the special
    primes and the digits inside them. On those primes the gadget
    P (Q/D_j) [(Q/D_j)^-1]_{D_j} agrees with P (Q'/D_j) [(Q'/D_j)^-1]_{D_j}
    (both are P on the digit's primes and 0 on the other primes of Q'), so the
    restriction is a key for the smaller modulus."""
    rows = list(range(level)) + list(range(pr.L, pr.L + pr.K))
    digits = [(b.limbs(rows), a.limbs(rows)) for b, a in gk.digits[:level // pr.alpha]]
    return GaloisKey(gk.k, digits)


def mod_switch(pr, ct, level):
    """Drop the ciphertext primes beyond `level`: with D the product of the dropped
    primes, each component c becomes (c - Conv_{D->Q'}([c]_D)) D^-1 mod Q', the
    fast basis conversion of the dropped residues written out as in moddown
    (y_j = [c_j (D/q_j)^-1]_{q_j}, Conv = sum_j y_j (D/q_j)); this divides the
    ciphertext by D, so it decrypts under Q' to the same plaintext."""
    kept, dropped = pr.q[:level], pr.q[level:]
    D = 1
    for x in dropped:
        D *= x
    out = []
    for comp in (ct.c0, ct.c1):
        ys = []
        for j, qj in enumerate(dropped):
            inv = pow((D // qj) % qj, -1, qj)
            ys.append((comp.c[level + j].astype(object) * inv) % qj)
        rows = np.empty((level, pr.n), dtype=np.uint64)
        for i, qi in enumerate(kept):
            conv = np.zeros(pr.n, dtype=object)
            for y, qj in zip(ys, dropped):
                conv = conv + y * ((D // qj) % qi)
            conv = conv % qi
            diff = (comp.c[i].astype(object) - conv) % qi
            rows[i] = (diff * pow(D % qi, -1, qi) % qi).astype(np.uint64)
        out.append(Poly(kept, rows))
    return Ciphertext(out[0], out[1])


# ---------------------------------------------------------------------------
# Galois elements of the rotations (Sec. 5.1)

def rot_row_element(pr, r):
    """sigma_k with k = 3^(r mod n/2) mod 2n moves both rows left by r."""
    return pow(3, r % pr.nh, 2 * pr.n)


def rot_col_element(pr):
    """sigma_(2n-1) swaps the two rows."""
    return 2 * pr.n - 1
