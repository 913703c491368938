"""GPU parity of the ring-level kernels against the CPU oracle, through the C ABI.

Every comparison is element by element and exact (integer arithmetic): the
NTT through the ring product it implements, the SHAKE-128 samplers, key
generation, encryption, the plaintext product, basis conversion up and down,
both rotation forms, and the diagonal encoding.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, oracle_params, to_dev, to_host, say

pytestmark = pytest.mark.gpu

RINGS_ALL = ["ring-1024-p12289", "ring-4096", "ring-32768", "ring-65536"]


@pytest.mark.parametrize("ring", RINGS_ALL)
def test_ntt_roundtrip_and_ring_product(ring):
    from oracle.ring import negacyclic_mul_limb
    ctx = context(ring)
    say("ntt", ring)
    r = np.random.default_rng(1)
    n, nq = ctx.n, ctx.nq
    a = np.stack([r.integers(0, q, n, dtype=np.uint64) for q in ctx.primes])
    b = np.stack([r.integers(0, q, n, dtype=np.uint64) for q in ctx.primes])
    da, db = to_dev(a), to_dev(b)
    ctx.ntt(da, 0, nq)
    ctx.ntt(db, 0, nq)
    fa, fb = to_host(da), to_host(db)
    assert all((fa[i] < q).all() for i, q in enumerate(ctx.primes))
    # pointwise product on the host, back through the inverse transform on the GPU
    prod = np.stack([((fa[i].astype(object) * fb[i].astype(object)) % q).astype(np.uint64)
                     for i, q in enumerate(ctx.primes)])
    dp = to_dev(prod)
    ctx.ntt(dp, 0, nq, inverse=True)
    got = to_host(dp)
    rows = range(nq) if n <= 4096 else [0, nq - 1]
    for i in rows:
        assert np.array_equal(got[i], negacyclic_mul_limb(a[i], b[i], ctx.primes[i])), i
    ctx.ntt(da, 0, nq, inverse=True)
    assert np.array_equal(to_host(da), a)


@pytest.mark.parametrize("log_n,q_bits", [(10, 60), (13, 60), (14, 60), (16, 56), (13, 56)])
def test_ntt_top_of_range_and_short_high_pass(log_n, q_bits):
    """The lazy butterflies' bounds at their limits: a 61-bit special prime (the
    largest the 64-bit transform takes), primes just below 2^56 (the forward transform
    without conditional subtractions, whose values reach 72q), every input q - 1 or
    near it, and the two-pass rings whose high-bit pass has fewer than 8 stages."""
    from paper_2408_17063_amd import hc
    from oracle.ring import negacyclic_mul_limb
    say("ntt extremes", log_n, q_bits)
    ctx = hc.Context(log_n=log_n, p=786433, L=2, q_bits=q_bits, K=1, p_bits=61)
    n, nq = ctx.n, ctx.nq
    assert max(ctx.primes) >> 60 == 1 and min(ctx.primes) >> (q_bits - 1) == 1
    r = np.random.default_rng(log_n)
    a = np.stack([np.full(n, q - 1, dtype=np.uint64) for q in ctx.primes])
    b = np.stack([r.integers(q - 4096, q, n, dtype=np.uint64) for q in ctx.primes])
    da, db = to_dev(a), to_dev(b)
    ctx.ntt(da, 0, nq)
    ctx.ntt(db, 0, nq)
    fa, fb = to_host(da), to_host(db)
    assert all((fa[i] < q).all() and (fb[i] < q).all() for i, q in enumerate(ctx.primes))
    prod = np.stack([((fa[i].astype(object) * fb[i].astype(object)) % q).astype(np.uint64)
                     for i, q in enumerate(ctx.primes)])
    dp = to_dev(prod)
    ctx.ntt(dp, 0, nq, inverse=True)
    got = to_host(dp)
    for i in range(nq):
        assert np.array_equal(got[i], negacyclic_mul_limb(a[i], b[i], ctx.primes[i])), i
    ctx.ntt(db, 0, nq, inverse=True)
    assert np.array_equal(to_host(db), b)


@pytest.mark.parametrize("ring", ["ring-4096", "ring-65536"])
def test_samplers_match_oracle(ring):
    import torch
    from oracle import rng
    ctx = context(ring)
    say("samplers", ring)
    seed = W.seed32("sampler", 7)
    out = torch.empty(ctx.n, dtype=torch.int64, device="cuda")
    for limb in (0, ctx.nq - 1):
        ctx.sample(0, seed, "gk_a", 12345, limb, out)
        want = rng.uniform_limb(seed, "gk_a", 12345, limb, ctx.primes[limb], ctx.n)
        assert np.array_equal(to_host(out), want)
    ctx.sample(1, seed, "sk", 0, 0, out)
    assert np.array_equal(out.cpu().numpy(), rng.ternary(seed, "sk", 0, ctx.n))
    ctx.sample(2, seed, "enc_e0", 3, 0, out)
    assert np.array_equal(out.cpu().numpy(), rng.gaussian(seed, "enc_e0", 3, ctx.n))


def oracle_keys(pr, sk_seed, gk_seed, elements):
    from oracle import bfv
    sk, pk = bfv.keygen(pr, sk_seed)
    gks = {k: bfv.galois_keygen(pr, sk, k, gk_seed) for k in elements}
    return sk, pk, gks


@pytest.mark.parametrize("ring", ["ring-1024-p12289", "ring-4096"])
def test_keygen_and_encrypt_match_oracle(ring):
    from oracle import bfv
    ctx = context(ring)
    pr = oracle_params(ring)
    say("keys", ring)
    sk_seed, gk_seed = W.seed32("sk", 1), W.seed32("gk", 1)
    elements = [pow(3, 5, 2 * pr.n), 2 * pr.n - 1]
    osk, opk, ogk = oracle_keys(pr, sk_seed, gk_seed, elements)
    sk, pk = ctx.keygen(sk_seed)
    gk = ctx.galois_keygen(sk, elements, gk_seed)
    assert np.array_equal(ctx.export_sk(sk), osk.s)
    epk = ctx.export_pk(pk)
    assert np.array_equal(epk[0], opk.b.c) and np.array_equal(epk[1], opk.a.c)
    for k in elements:
        eg = ctx.export_gk(gk, k)
        for j, (b, a) in enumerate(ogk[k].digits):
            assert np.array_equal(eg[j, 0], b.c), (k, j)
            assert np.array_equal(eg[j, 1], a.c), (k, j)
    slots = np.random.default_rng(3).integers(0, pr.p, size=(2, pr.nh))
    eseed = W.seed32("enc", 9)
    ct = ctx.encrypt(pk, slots, eseed)
    want = bfv.encrypt(pr, opk, slots, eseed)
    assert np.array_equal(to_host(ct), want.stack())
    assert np.array_equal(ctx.decrypt(sk, to_host(ct)), slots)


@pytest.mark.parametrize("ring", ["ring-1024-p12289", "ring-4096", "ring-2048-p12289"])
def test_ops_match_oracle(ring):
    from oracle import bfv
    from oracle.ring import Poly
    ctx = context(ring)
    pr = oracle_params(ring)
    say("ops", ring)
    r = np.random.default_rng(5)
    sk_seed, gk_seed = W.seed32("sk", 2), W.seed32("gk", 2)
    elements = [pow(3, 1, 2 * pr.n), pow(3, 7, 2 * pr.n), pow(3, pr.nh - 4, 2 * pr.n), 2 * pr.n - 1]
    osk, opk, ogk = oracle_keys(pr, sk_seed, gk_seed, elements)
    sk, pk = ctx.keygen(sk_seed)
    gk = ctx.galois_keygen(sk, elements, gk_seed)
    slots = r.integers(0, pr.p, size=(2, pr.nh))
    eseed = W.seed32("enc", 10)
    ct = ctx.encrypt(pk, slots, eseed)
    oct_ = bfv.encrypt(pr, opk, slots, eseed)
    # plaintext product
    m = r.integers(0, pr.p, size=(2, pr.nh))
    got = to_host(ctx.mul_plain(ct, m))
    assert np.array_equal(got, bfv.mul_plain(pr, oct_, bfv.plain_poly(pr, m)).stack())
    # plain rotations
    for k in elements:
        got = to_host(ctx.rotate(gk, k, ct))
        assert np.array_equal(got, bfv.rotate(pr, oct_, ogk[k]).stack()), k
    # hoisted rotations
    got = to_host(ctx.rotate_hoisted(gk, elements, ct))
    want = bfv.rotate_hoisted(pr, oct_, [ogk[k] for k in elements])
    for i, w in enumerate(want):
        assert np.array_equal(got[i], w.stack()), elements[i]
    # ModUp of a random element, every digit; ModDown of a random element over PQ
    import torch
    x = np.stack([r.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q])
    X = torch.empty((pr.L + pr.K, pr.n), dtype=torch.int64, device="cuda")
    for j in range(pr.dnum):
        ctx.modup(to_dev(x), j, X)
        assert np.array_equal(to_host(X), bfv.modup(pr, Poly(pr.q, x), j).c), j
    T = np.stack([r.integers(0, q, pr.n, dtype=np.uint64) for q in pr.qp])
    out = torch.empty((pr.L, pr.n), dtype=torch.int64, device="cuda")
    ctx.moddown(to_dev(T), out)
    assert np.array_equal(to_host(out), bfv.moddown(pr, Poly(pr.qp, T)).c)


@pytest.mark.parametrize("ring", ["ring-65536"])
def test_basis_conversion_full_size(ring):
    import torch
    from oracle import bfv
    from oracle.ring import Poly
    ctx = context(ring)
    pr = oracle_params(ring)
    say("bconv full", ring)
    r = np.random.default_rng(6)
    x = np.stack([r.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q])
    X = torch.empty((pr.L + pr.K, pr.n), dtype=torch.int64, device="cuda")
    ctx.modup(to_dev(x), pr.dnum - 1, X)
    assert np.array_equal(to_host(X), bfv.modup(pr, Poly(pr.q, x), pr.dnum - 1).c)
    T = np.stack([r.integers(0, q, pr.n, dtype=np.uint64) for q in pr.qp])
    out = torch.empty((pr.L, pr.n), dtype=torch.int64, device="cuda")
    ctx.moddown(to_dev(T), out)
    assert np.array_equal(to_host(out), bfv.moddown(pr, Poly(pr.qp, T)).c)


@pytest.mark.parametrize("ring,s,B,beta,gi,b", [
    ("ring-4096", 16, 4, 1, 2, 3), ("ring-2048-p12289", 16, 2, 7, 5, 1), ("ring-65536", 1024, 8, 15, 127, 7)])
def test_diagonal_encoding_matches_oracle(ring, s, B, beta, gi, b):
    import torch
    from oracle import bfv, compress as C
    ctx = context(ring)
    pr = oracle_params(ring)
    say("diag", ring, s, B, beta, gi, b)
    out = torch.empty((pr.L, pr.n), dtype=torch.int64, device="cuda")
    ctx.encode_diagonal(s, B, beta, gi, b, out)
    m = bfv.plain_poly(pr, C.diagonal_slots(pr.p, pr.nh, s, B, beta, gi, b))
    from oracle.ring import Poly
    assert np.array_equal(to_host(out), Poly.from_ints(pr.q, m).c)


@pytest.mark.parametrize("ring", ["ring-2048-p12289", "ring-4096"])
def test_mod_switch_and_rotate_level_match_oracle(ring):
    """hc_mod_switch for every level pair (each kept-prime count, several ciphertexts
    in one call) and hc_rotate_level at every digit-aligned level below the top, element
    by element against the oracle; each switched ciphertext still decrypts to the slots."""
    from oracle import bfv
    ctx = context(ring)
    pr = oracle_params(ring)
    say("switch and level rotation", ring)
    r = np.random.default_rng(11)
    sk_seed, gk_seed = W.seed32("sk", 3), W.seed32("gk", 3)
    k = pow(3, 5, 2 * pr.n)
    osk, opk, ogk = oracle_keys(pr, sk_seed, gk_seed, [k])
    sk, pk = ctx.keygen(sk_seed)
    gk = ctx.galois_keygen(sk, [k], gk_seed)
    slots = [r.integers(0, pr.p, size=(2, pr.nh)) for _ in range(2)]
    cts = ctx.ct_tensor(2)
    octs = []
    for i in range(2):
        ctx.encrypt(pk, slots[i], W.seed32("enc", 30, i), out=cts[i])
        octs.append(bfv.encrypt(pr, opk, slots[i], W.seed32("enc", 30, i)))
    for lin in range(2, pr.L + 1):
        src = cts[:, :, :lin, :].contiguous() if lin < pr.L else cts
        pin = bfv.at_level(pr, lin, keyswitch=False)
        osrc = [o if lin == pr.L else bfv.mod_switch(pr, o, lin) for o in octs]
        if lin < pr.L:
            # the oracle's own switch to lin is the input: feed the library the same words
            import torch
            src = torch.from_numpy(np.stack([o.stack() for o in osrc]).view(np.int64)).cuda()
        for lo in range(1, lin):
            got = to_host(ctx.mod_switch(src, lin, lo, count=2)).reshape(2, 2, lo, pr.n)
            for i in range(2):
                want = bfv.mod_switch(pin, osrc[i], lo)
                assert np.array_equal(got[i], want.stack()), (lin, lo, i)
                assert np.array_equal(ctx.decrypt(sk, got[i]), slots[i]), (lin, lo, i)
    for lvl in range(pr.alpha, pr.L, pr.alpha):
        lo_ct = bfv.mod_switch(pr, octs[0], lvl)
        plo = bfv.at_level(pr, lvl)
        want = bfv.rotate(plo, lo_ct, bfv.key_at_level(pr, ogk[k], lvl))
        got = to_host(ctx.rotate_level(gk, k, lvl, to_dev(lo_ct.stack())))
        assert np.array_equal(got.reshape(2, lvl, pr.n), want.stack()), lvl
        assert np.array_equal(ctx.decrypt(sk, got), np.roll(slots[0], -5, axis=1)), lvl


def test_mod_switch_rejects_bad_levels():
    from paper_2408_17063_amd import hc
    ctx = context("ring-2048-p12289")
    say("switch errors")
    ct = ctx.ct_tensor(1)
    for lin, lo in ((4, 4), (4, 0), (5, 2), (2, 3)):
        with pytest.raises(hc.HcError) as e:
            ctx.mod_switch(ct, lin, lo, out=ctx.ct_tensor(1))
        assert e.value.status == hc.HC_EINVAL, (lin, lo)
