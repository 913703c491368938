"""Pins of the CPU oracle against definitions that do not go through it.

Each test fixes one building block by something other than the oracle's own
code: brute-force convolution, direct polynomial evaluation, exact CRT,
closed forms, brute force over tiny inputs, the paper's printed sizes.
"""
import hashlib
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import bfv, compress as C, decompress as D, rng, slots
from oracle.params import make_params, is_prime
from oracle.ring import Poly, automorphism, negacyclic_mul_limb, ntt_limb, intt_limb, psi_for

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- ring

def brute_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += int(a[i]) * int(b[j])
            else:
                out[k - n] -= int(a[i]) * int(b[j])
    return [x % q for x in out]


@pytest.mark.parametrize("n,q", [(8, 17), (16, 97), (64, 18014398509309953), (32, 1152921504606830593)])
def test_ring_product_matches_brute_force(n, q):
    r = np.random.default_rng(n)
    for _ in range(3):
        a = np.array([int(x) for x in r.integers(0, 2**62, n)], dtype=object) % q
        b = np.array([int(x) for x in r.integers(0, 2**62, n)], dtype=object) % q
        got = negacyclic_mul_limb(a.astype(np.uint64), b.astype(np.uint64), q)
        assert [int(x) for x in got] == brute_negacyclic(a, b, q)


def test_ntt_is_evaluation_at_odd_powers():
    n, q = 16, 97
    psi = psi_for(n, q)
    assert pow(psi, n, q) == q - 1
    a = np.arange(3, 3 + n, dtype=np.uint64)
    ev = ntt_limb(a, q)
    for i in range(n):
        x = pow(psi, 2 * i + 1, q)
        assert int(ev[i]) == sum(int(a[j]) * pow(x, j, q) for j in range(n)) % q
    assert np.array_equal(intt_limb(ev, q), a)


# --------------------------------------------------------------------------- params

def fermat_probable_prime(x):
    return all(pow(b, x - 1, x) == 1 for b in (2, 3, 5, 7))


@pytest.mark.parametrize("n,p,L,qb,K,pb", [
    (4096, 65537, 2, 54, 1, 60), (1 << 15, 65537, 14, 55, 2, 60), (1 << 16, 786433, 24, 55, 3, 60)])
def test_primes_rule(n, p, L, qb, K, pb):
    pr = make_params(n, p, L, qb, K, pb)
    assert len(set(pr.q + pr.sp)) == L + K
    assert pr.q == sorted(pr.q, reverse=True)
    for bits, ps in ((qb, pr.q), (pb, pr.sp)):
        for x in ps:
            assert x < 2 ** bits and x % (2 * n) == 1 and fermat_probable_prime(x)
        # no skipped candidate between consecutive chosen primes (largest-first rule)
        for y in range(ps[0] + 2 * n, 2 ** bits, 2 * n):
            assert not fermat_probable_prime(y)
        for a, b in zip(ps, ps[1:]):
            for y in range(b + 2 * n, a, 2 * n):
                assert not fermat_probable_prime(y) or y in pr.q
    assert pr.delta == pr.Q // p
    assert pow(pr.zeta, n, p) == p - 1
    assert all(pow(x, n, p) != p - 1 for x in range(2, pr.zeta))


def test_is_prime_small_table():
    sieve = [True] * 2000
    sieve[0] = sieve[1] = False
    for i in range(2, 2000):
        if sieve[i]:
            for j in range(i * i, 2000, i):
                sieve[j] = False
    assert [i for i in range(2000) if is_prime(i)] == [i for i in range(2000) if sieve[i]]


# --------------------------------------------------------------------------- slots

def small_params():
    # n = 16, p = 97 (97 = 1 mod 32); tiny moduli keep brute force cheap
    return make_params(16, 97, 2, 30, 1, 31)


def test_encode_matches_closed_form_and_evaluation():
    pr = small_params()
    r = np.random.default_rng(0)
    sl = r.integers(0, pr.p, size=(2, pr.nh))
    m = slots.encode(sl, pr)
    assert [int(x) for x in m] == slots.encode_closed_form(sl, pr.n, pr.p, pr.zeta)
    for row in range(2):
        for c in range(pr.nh):
            x = pow(pr.zeta, slots.exponent(pr.n, row, c), pr.p)
            assert sum(int(m[i]) * pow(x, i, pr.p) for i in range(pr.n)) % pr.p == sl[row][c]
    assert np.array_equal(slots.decode(m, pr), sl)


def test_exponents_cover_odd_residues():
    for n in (16, 1024):
        ex = slots.slot_exponents(n)
        assert sorted(ex.ravel().tolist()) == list(range(1, 2 * n, 2))


def plain_automorphism(coeffs, k, p):
    n = len(coeffs)
    out = [0] * n
    for i, c in enumerate(coeffs):
        j = i * k % (2 * n)
        if j < n:
            out[j] = (out[j] + int(c)) % p
        else:
            out[j - n] = (out[j - n] - int(c)) % p
    return out


def test_rotations_are_slot_permutations():
    """Rot_row(.; r) <-> X -> X^(3^r), Rot_col <-> X -> X^(2n-1) (Sec. 5.1)."""
    pr = small_params()
    sl = np.random.default_rng(1).integers(0, pr.p, size=(2, pr.nh))
    m = slots.encode(sl, pr)
    for r in range(pr.nh):
        got = slots.decode(plain_automorphism(m, pow(3, r, 2 * pr.n), pr.p), pr)
        assert np.array_equal(got, np.roll(sl, -r, axis=1))   # left rotation
    got = slots.decode(plain_automorphism(m, 2 * pr.n - 1, pr.p), pr)
    assert np.array_equal(got, sl[::-1])
    # the RNS automorphism of the oracle agrees with the plain one
    poly = Poly([pr.p], np.array([m], dtype=np.uint64))
    assert [int(x) for x in automorphism(poly, 3, ).c[0]] == plain_automorphism(m, 3, pr.p)


# --------------------------------------------------------------------------- randomness

def test_shake128_known_answer():
    # FIPS 202 / NIST example: SHAKE128 of the empty message
    assert hashlib.shake_128(b"").hexdigest(16) == "7f9c2ba4e88f827d616045507605853e"


def test_stream_framing_layout():
    seed = bytes(range(32))
    msg = seed + b"pk_a\0\0\0\0" + (5).to_bytes(8, "little") + (2).to_bytes(8, "little") \
        + (7).to_bytes(8, "little")
    assert rng.stream(seed, "pk_a", 5, 2, 7, 40) == hashlib.shake_128(msg).digest(40)


def test_cdt_table_margin_and_double_precision_agreement():
    T = rng.cdt_table(3.2)
    rho = [math.exp(-x * x / (2 * 3.2 * 3.2)) for x in range(20)]
    S = rho[0] + 2 * sum(rho[1:])
    acc = 0.0
    for k in range(20):
        acc += rho[0] if k == 0 else 2 * rho[k]
        scaled = acc / S * 2 ** 32
        if k < 19:
            assert T[k] == math.floor(scaled + 0.5)
            assert abs((scaled - math.floor(scaled)) - 0.5) > 2 ** -12  # far from a tie
    assert T[19] == 2 ** 32 and T == sorted(T)


def test_samplers_distribution():
    seed = bytes(32)
    g = rng.gaussian(seed, "pk_e", 0, 1 << 14)
    assert abs(g.std() - 3.2) < 0.15 and abs(g.mean()) < 0.15 and np.abs(g).max() <= 19
    t = rng.ternary(seed, "sk", 0, 1 << 14)
    counts = np.bincount(t + 1)
    assert set(np.unique(t)) <= {-1, 0, 1} and counts.min() > 5000
    q = 18014398509309953
    u = rng.uniform_limb(seed, "pk_a", 0, 0, q, 4096)
    assert u.max() < q and abs(u.astype(float).mean() / q - 0.5) < 0.03


# --------------------------------------------------------------------------- BFV

@pytest.fixture(scope="module")
def p4096():
    pr = make_params(4096, 65537, 2, 54, 1, 60)
    sk, pk = bfv.keygen(pr, bytes(32))
    return pr, sk, pk


def test_encrypt_decrypt_and_noise(p4096):
    pr, sk, pk = p4096
    sl = np.random.default_rng(2).integers(0, pr.p, size=(2, pr.nh))
    ct = bfv.encrypt(pr, pk, sl, bytes([1] * 32))
    assert np.array_equal(bfv.decrypt(pr, sk, ct), sl)
    assert bfv.noise_bits(pr, sk, ct) < 20 < bfv.noise_budget_bits(pr)


def test_plain_product_is_slotwise(p4096):
    pr, sk, pk = p4096
    r = np.random.default_rng(3)
    a = r.integers(0, pr.p, size=(2, pr.nh))
    m = r.integers(0, pr.p, size=(2, pr.nh))
    ct = bfv.mul_plain(pr, bfv.encrypt(pr, pk, a, bytes([4] * 32)), bfv.plain_poly(pr, m))
    assert np.array_equal(bfv.decrypt(pr, sk, ct), a * m % pr.p)


def exact_crt(res, mods):
    M = math.prod(mods)
    return sum(int(r) * (M // m) * pow(M // m, -1, m) for r, m in zip(res, mods)) % M


def test_modup_is_exact_crt_plus_small_multiple(p4096):
    pr = make_params(4096, 65537, 4, 54, 2, 60)  # two primes per digit
    r = np.random.default_rng(5)
    d = Poly(pr.q, np.stack([r.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q]))
    for j in range(pr.dnum):
        X = bfv.modup(pr, d, j)
        I = pr.digit_limbs(j)
        Dj = math.prod(pr.q[i] for i in I)
        for coef in range(0, pr.n, 97):
            x = exact_crt([d.c[i, coef] for i in I], [pr.q[i] for i in I])
            ok = [all(int(X.c[l, coef]) == (x + u * Dj) % m for l, m in enumerate(pr.qp))
                  for u in range(len(I))]
            assert any(ok)


def test_moddown_is_division_by_P(p4096):
    pr = make_params(4096, 65537, 2, 54, 2, 60)
    r = np.random.default_rng(6)
    x = [int(v) for v in r.integers(-2**40, 2**40, pr.n)]
    e = [int(v) for v in r.integers(-2**20, 2**20, pr.n)]
    T = Poly.from_ints(pr.qp, [pr.P * a + b for a, b in zip(x, e)])
    out = bfv.moddown(pr, T)
    for coef in range(0, pr.n, 61):
        val = exact_crt(out.c[:, coef], pr.q)
        val = val - pr.Q if val > pr.Q // 2 else val
        # floor((P x + e) / P) minus a BConv overflow u in [0, K]
        base = (pr.P * x[coef] + e[coef]) // pr.P
        assert base - pr.K <= val <= base


def test_galois_key_encrypts_gadget_times_rotated_secret(p4096):
    pr, sk, pk = p4096
    k = pow(3, 7, 2 * pr.n)
    gk = bfv.galois_keygen(pr, sk, k, bytes([9] * 32))
    s = sk.on(pr.qp)
    srot = automorphism(s, k)
    for j, (b, a) in enumerate(gk.digits):
        lhs = b + a * s - srot.scale([bfv.gadget_constant(pr, j, m) for m in pr.qp])
        for coef in range(0, pr.n, 101):
            v = exact_crt(lhs.c[:, coef], pr.qp)
            M = math.prod(pr.qp)
            v = v - M if v > M // 2 else v
            assert abs(v) <= 19


@pytest.mark.parametrize("r_step", [1, 5, 2047])
def test_rotation_forms_decrypt_alike(p4096, r_step):
    pr, sk, pk = p4096
    sl = np.random.default_rng(r_step).integers(0, pr.p, size=(2, pr.nh))
    ct = bfv.encrypt(pr, pk, sl, bytes([r_step % 256] * 32))
    k = bfv.rot_row_element(pr, r_step)
    gk = bfv.galois_keygen(pr, sk, k, bytes([7] * 32))
    plain = bfv.rotate(pr, ct, gk)
    hoisted = bfv.rotate_hoisted(pr, ct, [gk])[0]
    want = np.roll(sl, -r_step, axis=1)
    assert np.array_equal(bfv.decrypt(pr, sk, plain), want)
    assert np.array_equal(bfv.decrypt(pr, sk, hoisted), want)
    assert not (plain == hoisted)  # hoisting changes bits, not values


def test_rotate_sum_is_rotations_up_to_one_rounding(p4096):
    """A sum of rotations brought down once differs from the sum of separately
    key-switched rotations only by ModDown's rounding: per coefficient, as an
    integer mod Q, by a value in [-(K-1), G K - 1] (G rotations; each fast
    ModDown returns floor(T/P) - u with 0 <= u < K), and decrypts to the sum of
    the rotated slots."""
    pr, sk, pk = p4096
    steps = [1, 5, 2047]
    cts, gks, want = [], [], np.zeros((2, pr.nh), dtype=np.int64)
    for i, r in enumerate(steps):
        sl = np.random.default_rng(40 + i).integers(0, pr.p, size=(2, pr.nh))
        cts.append(bfv.encrypt(pr, pk, sl, bytes([50 + i] * 32)))
        gks.append(bfv.galois_keygen(pr, sk, bfv.rot_row_element(pr, r), bytes([60 + i] * 32)))
        want = (want + np.roll(sl, -r, axis=1)) % pr.p
    lazy = bfv.rotate_sum(pr, cts, gks)
    eager = None
    for ct, gk in zip(cts, gks):
        r = bfv.rotate(pr, ct, gk)
        eager = r if eager is None else eager + r
    assert np.array_equal(bfv.decrypt(pr, sk, lazy), want)
    Q = math.prod(pr.q)
    G, K = len(steps), pr.K
    for a, b in ((lazy.c0, eager.c0), (lazy.c1, eager.c1)):
        for x in range(0, pr.n, 97):
            # CRT of the difference's residues, written out here
            v = 0
            for i, q in enumerate(pr.q):
                d = (int(a.c[i][x]) - int(b.c[i][x])) % q
                Mi = Q // q
                v += d * Mi * pow(Mi % q, -1, q)
            v %= Q
            v = v - Q if v > Q // 2 else v
            assert -(K - 1) <= v <= G * K - 1, (x, v)
    assert not (lazy == eager)  # the rounding does show in the bits


# --------------------------------------------------------------------------- decompression

def test_newton_matches_direct_expansion():
    p = 65537
    r = np.random.default_rng(7)
    for _ in range(20):
        s = int(r.integers(1, 9))
        J = [int(x) for x in r.integers(0, 50, s)]
        w = [sum(pow(x, j, p) for x in J) % p for j in range(1, s + 1)]
        poly = [1]
        for x in J:  # multiply by (X - x), highest degree first
            poly = [(a - x * b) % p for a, b in zip(poly + [0], [0] + poly)]
        assert D.f_coefficients(w, p) == poly


def test_reconstruction_all_subsets_brute_force():
    p, N, s = 17, 8, 4
    for t in range(0, s + 1):
        for I in itertools.combinations(range(1, N + 1), t):
            vals = [(3 * i + 1) % p for i in I]
            d = [0] * N
            for i, x in zip(I, vals):
                d[i - 1] = x
            v = [1 if x else 0 for x in [int(i + 1 in I) for i in range(N)]]
            w = [sum(pow(i, j, p) * v[i - 1] for i in range(1, N + 1)) % p for j in range(1, s + 1)]
            e = [sum(pow(i, j, p) * d[i - 1] for i in range(1, N + 1)) % p for j in range(1, s + 1)]
            idx, got = D.decompress_group(p, N, w, [e])
            assert idx == list(I) and got == [vals]


def test_too_many_matches_is_reported():
    p, N, s = 65537, 4096, 8
    r = np.random.default_rng(11)
    failures = 0
    for _ in range(10):
        I = sorted(int(x) + 1 for x in r.choice(N, size=s + 3, replace=False))
        w = [sum(pow(i, j, p) for i in I) % p for j in range(1, s + 1)]
        try:
            idx = D.reconst_idx(w, p, N)
            assert idx != I
        except D.DecodeError:
            failures += 1
    assert failures >= 8


def test_vandermonde_product_definition():
    p, s = 97, 5
    x = [3, 0, 7, 1, 0, 96]
    want = [sum((i + 1) ** j * x[i] for i in range(len(x))) % p for j in range(1, s + 1)]
    assert C.vandermonde_product(p, s, x) == want
    assert C.vandermonde_product_sparse(p, s, x) == want
    # a long sparse vector: the sparse form equals the dense definition
    r = np.random.default_rng(12)
    v = np.zeros(5000, dtype=np.int64)
    v[r.choice(5000, 40, replace=False)] = r.integers(1, 786433, 40)
    assert C.vandermonde_product_sparse(786433, 64, v) == C.vandermonde_product(786433, 64, v)


# --------------------------------------------------------------------------- schedule

def test_baby_step_rule():
    # k (B-1) + (s/B - 1) minimised over powers of two, ties to the larger B
    for s, k in [(16, 2), (256, 2), (1024, 16), (16, 8), (1, 3), (1024, 1)]:
        costs = {B: k * (B - 1) + (s // B - 1) for B in [2 ** i for i in range(11)] if B <= s}
        best = min(costs.values())
        assert C.choose_B(s, k) == max(B for B, c in costs.items() if c == best)


def test_group_split_keeps_indices_below_p():
    for n, p, N in [(4096, 65537, 4096), (1 << 16, 786433, 1 << 20), (1 << 15, 65537, 32 << 15),
                    (2048, 12289, 7 * 2048), (1 << 15, 65537, 3 << 15)]:
        sc = C.make_schedule(n, p, N, 1, 16)
        assert sum(g.n_rec for g in sc.groups) == N
        assert all(g.n_rec <= p - 1 for g in sc.groups)
        counts = [g.ct_count for g in sc.groups]
        assert max(counts) - min(counts) <= 1


def test_band_overflow_rejected():
    with pytest.raises(C.ScheduleError):
        C.make_schedule(1024, 12289, 1024, 4, 200)   # 3 bands x 256 > 512 slots


# --------------------------------------------------------------------------- the paper's sizes

def test_paper_communication_sizes():
    """Sec. 6.2: one output ciphertext of 110.6 KB, rotation keys of 442.4 KB
    at n = 2^13 with two 54-bit primes (closed forms of the sizes)."""
    with open(os.path.join(GOLDEN, "paper_sizes.json")) as f:
        g = json.load(f)
    n, bits = g["n"], g["prime_bits"]
    ct_bytes = 2 * n * bits / 8                 # two ring elements mod one 54-bit prime
    key_bytes = 4 * n * (2 * bits) / 8          # 2 digits x 2 ring elements mod q (108 bits)
    assert round(ct_bytes / 1000, 1) == g["ciphertext_kB"]
    assert round(key_bytes / 1000, 1) == g["rotation_key_kB"]


# --------------------------------------------------------------------------- end to end

def run_pipeline(wl_name):
    import workloads as W
    from oracle.params import make_params as mp
    wl = W.WORKLOADS[wl_name]
    ring = W.RINGS[wl.ring]
    pr = mp(ring.n, ring.p, ring.L, ring.q_bits, ring.K, ring.p_bits)
    v, db = W.query_inputs(wl)
    sc = C.make_schedule(pr.n, pr.p, wl.N, wl.ncol, wl.t)
    sk, pk = bfv.keygen(pr, W.seed32("sk", 0))
    gks = {k: bfv.galois_keygen(pr, sk, k, W.seed32("gk", k)) for k in sc.keys}
    vm = slots.vector_to_slot_matrices(v, pr.n, sc.n_ct)
    cts = [bfv.encrypt(pr, pk, vm[i], W.seed32("enc", i)) for i in range(sc.n_ct)]
    out = C.compress(pr, sc, cts, db, gks)
    return pr, sc, sk, v, db, out


@pytest.mark.parametrize("wl_name", ["tiny-1024", "plain-4096", "multi-2048"])
def test_compress_decrypts_to_vandermonde_and_decompresses(wl_name):
    pr, sc, sk, v, db, out = run_pipeline(wl_name)
    pr = bfv.at_level(pr, len(out.c0.mods))
    assert bfv.noise_bits(pr, sk, out) < bfv.noise_budget_bits(pr) - 8
    dec = bfv.decrypt(pr, sk, out)
    exp = C.expected_bands(sc, v, db)
    S = len(sc.streams)
    for b in range(sc.bands):
        assert C.band_slots(sc, dec, b) == exp[b]
    for gi, grp in enumerate(sc.groups):
        rows = []
        for st in range(S):
            rows += list(C.band_slots(sc, dec, gi * S + st))
        idx, vals = D.decompress_group(pr.p, grp.n_rec, rows[0], rows[1:1 + sc.ncol])
        seg = v[grp.rec_start:grp.rec_start + grp.n_rec]
        want = [int(i) + 1 for i in np.nonzero(seg)[0]]
        assert idx == want
        for c in range(sc.ncol):
            assert vals[c] == [int(db[c][grp.rec_start + i - 1]) % pr.p for i in want]


def test_missing_key_is_reported():
    import workloads as W
    pr = make_params(1024, 12289, 2, 54, 1, 60)
    sc = C.make_schedule(pr.n, pr.p, 1024, 1, 5)
    sk, pk = bfv.keygen(pr, bytes(32))
    gks = {k: bfv.galois_keygen(pr, sk, k, bytes(32)) for k in sc.keys[1:]}
    ct = bfv.encrypt(pr, pk, np.zeros((2, pr.nh), dtype=np.uint64), bytes(32))
    with pytest.raises(KeyError):
        C.compress(pr, sc, [ct], np.zeros((1, 1024), dtype=np.uint32), gks)


def test_mod_switch_divides_by_dropped_primes(p4096):
    """Dropping primes q_{l+1..L} (product D): the result is floor(c / D) minus a
    basis-conversion overflow in [0, L-l), and decrypts to the same slots."""
    pr = make_params(4096, 65537, 4, 54, 2, 60)
    sk, pk = bfv.keygen(pr, bytes(32))
    sl = np.random.default_rng(8).integers(0, pr.p, size=(2, pr.nh))
    ct = bfv.encrypt(pr, pk, sl, bytes([5] * 32))
    lo = bfv.mod_switch(pr, ct, 2)
    plo = bfv.at_level(pr, 2)
    assert np.array_equal(bfv.decrypt(plo, sk, lo), sl)
    D = pr.q[2] * pr.q[3]
    for comp, comp_lo in ((ct.c0, lo.c0), (ct.c1, lo.c1)):
        for coef in range(0, pr.n, 257):
            c = exact_crt(comp.c[:, coef], pr.q)
            got = exact_crt(comp_lo.c[:, coef], plo.q)
            want = c // D
            assert any(got == (want - u) % plo.Q for u in range(2))


def test_answer_switch_to_one_prime(p4096):
    """The answer's switch to one prime (Sec. 6.2 counts the answer as one ciphertext
    modulo one prime): from a Comp-level ciphertext at 2 primes down to 1, the result
    is floor(c / q_2) up to a conversion overflow in [0, 1), i.e. exactly the floor,
    and decrypts under q_1 alone to the same slots; a whole compression switched this
    way decrypts to the Vandermonde products."""
    pr = make_params(4096, 65537, 4, 54, 2, 60)
    sk, pk = bfv.keygen(pr, bytes(32))
    sl = np.random.default_rng(10).integers(0, pr.p, size=(2, pr.nh))
    ct = bfv.mod_switch(pr, bfv.encrypt(pr, pk, sl, bytes([5] * 32)), 2)
    p2 = bfv.at_level(pr, 2)
    one = bfv.mod_switch(p2, ct, 1)
    p1 = bfv.at_level(pr, 1, keyswitch=False)
    assert np.array_equal(bfv.decrypt(p1, sk, one), sl)
    for comp, comp1 in ((ct.c0, one.c0), (ct.c1, one.c1)):
        for coef in range(0, pr.n, 131):
            c = exact_crt(comp.c[:, coef], p2.q)
            assert int(comp1.c[0, coef]) == (c // pr.q[1]) % pr.q[0]
    # end to end with out_level = 1
    import workloads as W
    wl = W.WORKLOADS["multi-2048"]
    ring = W.RINGS[wl.ring]
    pr = make_params(ring.n, ring.p, ring.L, ring.q_bits, ring.K, ring.p_bits)
    v, db = W.query_inputs(wl)
    sc = C.make_schedule(pr.n, pr.p, wl.N, wl.ncol, wl.t)
    sk, pk = bfv.keygen(pr, W.seed32("sk", 0))
    gks = {k: bfv.galois_keygen(pr, sk, k, W.seed32("gk", k)) for k in sc.keys}
    vm = slots.vector_to_slot_matrices(v, pr.n, sc.n_ct)
    cts = [bfv.encrypt(pr, pk, vm[i], W.seed32("enc", i)) for i in range(sc.n_ct)]
    out = C.compress(pr, sc, cts, db, gks, out_level=1)
    assert len(out.c0.mods) == 1
    p1 = bfv.at_level(pr, 1, keyswitch=False)
    assert bfv.noise_bits(p1, sk, out) < bfv.noise_budget_bits(p1) - 8
    dec = bfv.decrypt(p1, sk, out)
    exp = C.expected_bands(sc, v, db)
    for b in range(sc.bands):
        assert C.band_slots(sc, dec, b) == exp[b]


def test_restricted_key_switches_at_lower_level():
    pr = make_params(4096, 65537, 4, 54, 2, 60)
    sk, pk = bfv.keygen(pr, bytes(32))
    sl = np.random.default_rng(9).integers(0, pr.p, size=(2, pr.nh))
    plo = bfv.at_level(pr, 2)
    ct = bfv.mod_switch(pr, bfv.encrypt(pr, pk, sl, bytes([6] * 32)), 2)
    k = bfv.rot_row_element(pr, 3)
    gk = bfv.key_at_level(pr, bfv.galois_keygen(pr, sk, k, bytes([7] * 32)), 2)
    assert np.array_equal(bfv.decrypt(plo, sk, bfv.rotate(plo, ct, gk)), np.roll(sl, -3, axis=1))


# --------------------------------------------------------------------------- unencrypted database

@pytest.mark.parametrize("wl_name,out_level", [("tiny-1024", None), ("multi-2048", None), ("multi-2048", 1)])
def test_plain_db_form_decrypts_to_vandermonde(wl_name, out_level):
    """Sec. 5.2's remark on an unencrypted database: [C; C diag(DB)] v computed on the
    index vector alone decrypts to the same products as Mask + Comp (Eq. (1)) in every
    band, and decompresses (Alg. 6) to the matched records and values."""
    import workloads as W
    wl = W.WORKLOADS[wl_name]
    ring = W.RINGS[wl.ring]
    pr = make_params(ring.n, ring.p, ring.L, ring.q_bits, ring.K, ring.p_bits)
    v, db = W.query_inputs(wl)
    sc = C.make_schedule(pr.n, pr.p, wl.N, wl.ncol, wl.t)
    sc2 = C.plain_db_schedule(sc)
    sk, pk = bfv.keygen(pr, W.seed32("sk", 0))
    gks = {k: bfv.galois_keygen(pr, sk, k, W.seed32("gk", k)) for k in sc2.keys}
    vm = slots.vector_to_slot_matrices(v, pr.n, sc.n_ct)
    cts = [bfv.encrypt(pr, pk, vm[i], W.seed32("enc", i)) for i in range(sc.n_ct)]
    out = C.compress_plain_db(pr, sc, cts, db, gks, out_level=out_level)
    p_out = bfv.at_level(pr, len(out.c0.mods), keyswitch=False)
    assert bfv.noise_bits(p_out, sk, out) < bfv.noise_budget_bits(p_out) - 8
    dec = bfv.decrypt(p_out, sk, out)
    exp = C.expected_bands(sc, v, db)
    for b in range(sc.bands):
        assert C.band_slots(sc, dec, b) == exp[b], b
    S = len(sc.streams)
    for gi, grp in enumerate(sc.groups):
        rows = []
        for st in range(S):
            rows += list(C.band_slots(sc, dec, gi * S + st))
        idx, vals = D.decompress_group(pr.p, grp.n_rec, rows[0], rows[1:1 + sc.ncol])
        seg = v[grp.rec_start:grp.rec_start + grp.n_rec]
        assert idx == [int(i) + 1 for i in np.nonzero(seg)[0]]


def test_plain_db_diagonal_rows():
    """The diagonal of the unencrypted-database form, entry by entry from its definition:
    row r holds alpha^e times the value of the record the slot multiplies (C: times 1)."""
    p, nh, s, B = 12289, 16, 8, 2
    db = [np.arange(100, 140) % p, np.arange(7, 47) * 3 % p]
    rec0 = 5
    d = C.diagonal_slots_db(p, nh, s, B, (1, 0), 2, 1, (0, 2), db, rec0)
    for m in range(nh):
        c = (m + 1) % nh
        e = (m - 2 * B) % s + 1
        assert d[0, m] == pow(1 * nh + c + 1, e, p)                      # C, block 1
        rec = rec0 + 0 * nh + c
        assert d[1, m] == pow(c + 1, e, p) * int(db[1][rec]) % p         # C diag(DB_2), block 0
    z = C.diagonal_slots_db(p, nh, s, B, (0, 1), 0, 0, (1, None), db, 30)
    assert not z[1].any()                                                # a missing second vector
    assert z[0, 15] == 0                                                 # record 30 + 15 is past the end


# --------------------------------------------------------------------------- ciphertext products

def int_negacyclic(a, b):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - n] -= a[i] * b[j]
    return out


def test_exact_negacyclic_is_the_integer_product():
    from oracle import mult
    r = np.random.default_rng(20)
    for n, bits in ((8, 70), (16, 300), (32, 1000)):
        a = [int(x) - (1 << (bits - 1)) for x in r.integers(0, 1 << 62, n)]
        a = [x * (1 << (bits - 62)) + int(y) for x, y in zip(a, r.integers(0, 1 << 30, n))]
        b = [int(x) * (1 << (bits - 62)) - int(y) for x, y in zip(r.integers(-(1 << 61), 1 << 61, n),
                                                                   r.integers(0, 1 << 40, n))]
        assert mult.exact_negacyclic(a, b) == int_negacyclic(a, b)


@pytest.fixture(scope="module")
def deep():
    import workloads as W
    r = W.RINGS["ring-1024-deep"]
    pr = make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)
    from oracle import mult
    sk, pk = bfv.keygen(pr, bytes([1] * 32))
    rk = mult.relin_keygen(pr, sk, bytes([2] * 32))
    return pr, sk, pk, rk


def phase_three(pr, sk, z):
    """[z0 + z1 s + z2 s^2]_Q, decoded (the tensor's decryption)."""
    s = sk.on(pr.q)
    v = z[0] + z[1] * s + z[2] * (s * s)
    x = [bfv.crt(v.c[:, i], pr.q) for i in range(pr.n)]
    return slots.decode([((2 * pr.p * xi + pr.Q) // (2 * pr.Q)) % pr.p for xi in x], pr)


def test_tensor_and_product_decrypt_to_slotwise_product(deep):
    from oracle import mult
    pr, sk, pk, rk = deep
    r = np.random.default_rng(21)
    a = r.integers(0, pr.p, size=(2, pr.nh))
    b = r.integers(0, pr.p, size=(2, pr.nh))
    ca = bfv.encrypt(pr, pk, a, bytes([3] * 32))
    cb = bfv.encrypt(pr, pk, b, bytes([4] * 32))
    want = a * b % pr.p
    assert np.array_equal(phase_three(pr, sk, mult.tensor(pr, ca, cb)), want)
    prod = mult.mul(pr, ca, cb, rk)
    assert np.array_equal(bfv.decrypt(pr, sk, prod), want)
    assert bfv.noise_bits(pr, sk, prod) < bfv.noise_budget_bits(pr) - 200


def test_relin_key_encrypts_gadget_times_s_squared(deep):
    """b_j + a_j s = e_j + P (Q/D_j) [(Q/D_j)^-1]_{D_j} s^2 over PQ with e_j small."""
    pr, sk, pk, rk = deep
    s = sk.on(pr.qp)
    s2 = s * s
    for j, (b, a) in enumerate(rk.digits):
        e = b + a * s - s2.scale([bfv.gadget_constant(pr, j, m) for m in pr.qp])
        for i, m in enumerate(pr.qp):
            cen = np.where(e.c[i] > m // 2, e.c[i].astype(object) - m, e.c[i].astype(object))
            assert max(abs(int(x)) for x in cen) <= 19


def test_power_and_fermat_index_vector(deep):
    """Power_e slot-wise for small e, and Power_{p-1} = the index vector (Fermat)."""
    from oracle import mult
    pr, sk, pk, rk = deep
    r = np.random.default_rng(22)
    x = r.integers(0, pr.p, size=(2, pr.nh))
    x[0, :40] = 0
    cx = bfv.encrypt(pr, pk, x, bytes([5] * 32))
    for e in (2, 3, 5):
        assert np.array_equal(bfv.decrypt(pr, sk, mult.power(pr, cx, e, rk)),
                              np.array([[pow(int(v), e, pr.p) for v in row] for row in x]))
    v = mult.power(pr, cx, pr.p - 1, rk)
    assert np.array_equal(bfv.decrypt(pr, sk, v), (x != 0).astype(np.int64))
    assert bfv.noise_bits(pr, sk, v) < bfv.noise_budget_bits(pr) - 8


def test_match_is_the_exact_match_predicate(deep):
    """Match (Alg. 7 step 1) for keys with N not a multiple of n: 1 exactly where the
    record's key equals the query, 0 elsewhere and past the last record."""
    import workloads as W
    from oracle import mult
    pr, sk, pk, rk = deep
    N = pr.n + 300
    keys, x, v = W.match_inputs(N, 9, pr.p)
    cx = bfv.encrypt(pr, pk, np.full((2, pr.nh), x), bytes([6] * 32))
    out = mult.match(pr, cx, keys, rk)
    got = np.concatenate([bfv.decrypt(pr, sk, c).reshape(-1) for c in out])
    want = np.zeros(2 * pr.n, dtype=np.int64)
    want[:N] = v
    assert np.array_equal(got, want)


def test_generic_comp_recovers_sparse_vector(deep):
    """Alg. 5 on ciphertexts of d alone: v = Power_{p-1}(d), Comp of (v, d); the answer
    decrypts to (C v, C d) (Eq. (1)) and decompresses to d's support and values."""
    from oracle import mult
    pr, sk, pk, rk = deep
    N, t = pr.n, 6
    r = np.random.default_rng(23)
    d = np.zeros(N, dtype=np.int64)
    pos = r.choice(N, t, replace=False)
    d[pos] = r.integers(1, pr.p, t)
    sc = C.make_schedule(pr.n, pr.p, N, 1, t)
    gks = {k: bfv.galois_keygen(pr, sk, k, bytes([7] * 32)) for k in sc.keys}
    cd = [bfv.encrypt(pr, pk, slots.vector_to_slot_matrices(d, pr.n, 1)[0], bytes([8] * 32))]
    out = mult.compress_generic(pr, sc, cd, gks, rk, out_level=1)
    p1 = bfv.at_level(pr, 1, keyswitch=False)
    dec = bfv.decrypt(p1, sk, out)
    v = (d != 0).astype(np.int64)
    exp = C.expected_bands(sc, v, [d])
    assert C.band_slots(sc, dec, 0) == exp[0]
    idx, vals = D.decompress_group(pr.p, N, *[list(x) for x in C.band_slots(sc, dec, 0)][:1],
                                   [C.band_slots(sc, dec, 0)[1]])
    assert idx == sorted(int(i) + 1 for i in pos)
    assert vals[0] == [int(d[i - 1]) for i in idx]
