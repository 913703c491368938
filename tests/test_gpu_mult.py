"""Ciphertext products (hc_mul), Power (hc_power), Match (hc_match) and the generic Comp
of Alg. 5 (hc_compress_generic): bit-identical to the oracle (oracle/mult.py) on a
ring with room for Power_{p-1} (n = 1024, p = 12289, ten 60-bit primes), and at the
large workload's parameters (n = 2^16, p = 786433, 24 primes) a whole Match ->
Answer -> Recover round trip decrypts and decompresses to the matching records."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, oracle_params, to_dev, to_host, say

pytestmark = pytest.mark.gpu

RING = "ring-1024-deep"
SK, RK, GK = W.seed32("sk", 70), W.seed32("rk", 70), W.seed32("gk", 70)


@pytest.fixture(scope="module")
def keys():
    from oracle import bfv, mult
    ctx = context(RING)
    pr = oracle_params(RING)
    sk, pk = ctx.keygen(SK)
    rk = ctx.relin_keygen(sk, RK)
    osk, opk = bfv.keygen(pr, SK)
    ork = mult.relin_keygen(pr, osk, RK)
    return ctx, pr, sk, pk, rk, osk, opk, ork


def test_relin_key_matches_oracle(keys):
    ctx, pr, sk, pk, rk, osk, opk, ork = keys
    say("relin key")
    got = ctx.export_gk(rk, 1)
    for j, (b, a) in enumerate(ork.digits):
        assert np.array_equal(got[j, 0], b.c) and np.array_equal(got[j, 1], a.c), j


def test_product_and_powers_bit_identical(keys):
    from oracle import bfv, mult
    ctx, pr, sk, pk, rk, osk, opk, ork = keys
    say("products and powers")
    r = np.random.default_rng(71)
    a = r.integers(0, pr.p, size=(2, pr.nh))
    b = r.integers(0, pr.p, size=(2, pr.nh))
    a[1, :50] = 0
    ca, cb = ctx.encrypt(pk, a, W.seed32("enc", 71, 0)), ctx.encrypt(pk, b, W.seed32("enc", 71, 1))
    oa = bfv.encrypt(pr, opk, a, W.seed32("enc", 71, 0))
    ob = bfv.encrypt(pr, opk, b, W.seed32("enc", 71, 1))
    got = to_host(ctx.mul(rk, ca, cb))
    assert np.array_equal(got, mult.mul(pr, oa, ob, ork).stack())
    assert np.array_equal(ctx.decrypt(sk, got), a * b % pr.p)
    # the output may alias either input
    for alias in (0, 1):
        x, y = ca.clone(), cb.clone()
        assert np.array_equal(to_host(ctx.mul(rk, x, y, out=(x, y)[alias])), got), alias
    for e in (2, 3, 6, pr.p - 1):
        got = to_host(ctx.power(rk, ca, e))
        assert np.array_equal(got, mult.power(pr, oa, e, ork).stack()), e
        want = (a != 0).astype(np.int64) if e == pr.p - 1 else np.array(
            [[pow(int(v), e, pr.p) for v in row] for row in a])
        assert np.array_equal(ctx.decrypt(sk, got), want), e


def test_match_bit_identical(keys):
    from oracle import bfv, mult
    ctx, pr, sk, pk, rk, osk, opk, ork = keys
    say("match")
    N = pr.n + 300
    kv, x, v = W.match_inputs(N, 9, pr.p, seed=1)
    kdb = ctx.db_upload(kv.reshape(1, -1))
    xs = np.full((2, pr.nh), x)
    cx = ctx.encrypt(pk, xs, W.seed32("enc", 72))
    ox = bfv.encrypt(pr, opk, xs, W.seed32("enc", 72))
    got = to_host(ctx.match(rk, kdb, cx, N))
    want = mult.match(pr, ox, kv, ork)
    for i, w in enumerate(want):
        assert np.array_equal(got[i], w.stack()), i
    dec = np.concatenate([ctx.decrypt(sk, got[i]).reshape(-1) for i in range(len(want))])
    assert np.array_equal(dec[:N], v) and not dec[N:].any()


def test_match_over_more_ciphertexts_than_one_batch(keys):
    """Match over 17 ciphertexts (the powers run as a batch of 16, then 1): every slot
    decrypts to the predicate, and a ciphertext's words do not depend on its batch (the
    first ciphertext equals a one-ciphertext Match of the same keys)."""
    ctx, pr, sk, pk, rk, osk, opk, ork = keys
    say("match over 17 ciphertexts")
    N = 16 * pr.n + 300
    kv, x, v = W.match_inputs(N, 40, pr.p, seed=3)
    kdb = ctx.db_upload(kv.reshape(1, -1))
    cx = ctx.encrypt(pk, np.full((2, pr.nh), x), W.seed32("enc", 75))
    got = to_host(ctx.match(rk, kdb, cx, N))
    assert got.shape[0] == 17
    dec = np.concatenate([ctx.decrypt(sk, got[i]).reshape(-1) for i in range(got.shape[0])])
    assert np.array_equal(dec[:N], v) and not dec[N:].any()
    kdb1 = ctx.db_upload(kv[:pr.n].reshape(1, -1))
    one = to_host(ctx.match(rk, kdb1, cx, pr.n))
    assert np.array_equal(one[0], got[0])


def test_generic_comp_bit_identical(keys):
    """Alg. 5 on ciphertexts of d alone, answer switched to one prime."""
    from oracle import bfv, compress as C, mult, slots
    ctx, pr, sk, pk, rk, osk, opk, ork = keys
    say("generic comp")
    N, t = pr.n, 6
    r = np.random.default_rng(73)
    d = np.zeros(N, dtype=np.int64)
    d[r.choice(N, t, replace=False)] = r.integers(1, pr.p, t)
    sc = C.make_schedule(pr.n, pr.p, N, 1, t)
    gk = ctx.galois_keygen(sk, sc.keys, GK)
    ogks = {k: bfv.galois_keygen(pr, osk, k, GK) for k in sc.keys}
    dm = slots.vector_to_slot_matrices(d, pr.n, 1)[0]
    cd = ctx.ct_tensor(1)
    ctx.encrypt(pk, dm, W.seed32("enc", 73), out=cd[0])
    out, info = ctx.compress_generic(gk, rk, cd, N, t, out_level=1)
    got = to_host(ctx.output(out, info))
    want = mult.compress_generic(pr, sc, [bfv.encrypt(pr, opk, dm, W.seed32("enc", 73))], ogks, ork, out_level=1)
    assert np.array_equal(got, want.stack())
    dec = ctx.decrypt(sk, got)
    from paper_2408_17063_amd import hc
    w, e = C.band_slots(sc, dec, 0)
    idx, vals = hc.decompress(ctx.p, N, sc.s, w, [e])
    assert idx == [int(i) + 1 for i in np.nonzero(d)[0]] and vals[0] == [int(d[i - 1]) for i in idx]


def test_match_answer_recover_large_parameters():
    """Query (x in every slot) -> Match at ring 2^16 with 24 primes (Power_{p-1} with
    p = 786433: 20 products) -> Mask + Comp -> Recover: the matched records and values."""
    from oracle import compress as C
    from paper_2408_17063_amd import hc
    say("match round trip, large parameters")
    ring = "ring-65536"
    ctx = context(ring)
    N, t = (1 << 16) + 1000, 10
    kv, x, v = W.match_inputs(N, t, ctx.p, seed=2)
    vals = W.value_columns(W.rng_for(74, 0), N, 1, "u16", ctx.p)
    sk, pk = ctx.keygen(W.seed32("sk", 74))
    rk = ctx.relin_keygen(sk, W.seed32("rk", 74))
    keys, _ = ctx.plan(N, 1, t, out_level=1)
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 74))
    kdb, vdb = ctx.db_upload(kv.reshape(1, -1)), ctx.db_upload(vals)
    cx = ctx.encrypt(pk, np.full((2, ctx.nh), x), W.seed32("enc", 74))
    ctv = ctx.match(rk, kdb, cx, N)
    dec = np.concatenate([ctx.decrypt(sk, to_host(ctv[i])).reshape(-1) for i in range(ctv.shape[0])])
    assert np.array_equal(dec[:N], v)
    out, info = ctx.compress(gk, vdb, ctv, N, t, out_level=1)
    ans = ctx.decrypt(sk, to_host(ctx.output(out, info)))
    sched = C.make_schedule(ctx.n, ctx.p, N, 1, t)
    w, e = C.band_slots(sched, ans, 0)
    idx, got = hc.decompress(ctx.p, N, sched.s, w, [e])
    want = [int(i) + 1 for i in np.nonzero(v)[0]]
    assert idx == want and got[0] == [int(vals[0][i - 1]) for i in want]
