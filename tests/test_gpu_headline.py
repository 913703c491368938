"""Correctness at the large workload's own parameters: ring 2^16, 24 x 55-bit
ciphertext primes + 3 x 60-bit special primes, p = 786433.

* ring-level operations at full size against oracle results stored by
  tests/golden/make_ring65536.py (SHA-256 of every word plus sampled words):
  keygen, encryption, a Galois key, plain and hoisted rotation with all 27
  primes, Mask at 24 primes, the 24 -> 3 prime switch, a rotation with the key
  restricted to 3 primes, the 3 -> 1 prime answer switch;
* a whole compression of one ciphertext of records (t = 16, 4 columns) at those
  parameters, bit-identical to the oracle's (stored the same way);
* the whole benchmark query (2^20 records in 16 ciphertexts, t = 1024, 4 value
  columns, 2 groups x 3 streams, 1549 key switches): its answer decrypts to the
  Vandermonde products of Eq. (1) in every band and decompresses (Alg. 6) to every
  matched record and value; the noise left at the Comp level and in the one-prime
  answer is measured against the decryption budget.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, oracle_params, to_dev, to_host, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RING = "ring-65536"


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def check(got, ref, what):
    a = np.ascontiguousarray(got, dtype=np.uint64)
    flat = a.reshape(-1)
    assert list(a.shape) == ref["shape"], (what, a.shape, ref["shape"])
    bad = [(i, int(flat[i]), w) for i, w in zip(ref["sample_index"], ref["sample"]) if int(flat[i]) != w]
    assert not bad, (what, bad[:4])
    assert hashlib.sha256(flat.astype("<u8").tobytes()).hexdigest() == ref["sha256"], what


def test_ring65536_operations_match_oracle():
    from tests.golden.make_ring65536 import OPS_ENC, OPS_GK, OPS_SK, ops_inputs
    gold = load("ring65536_ops.json")
    ctx = context(RING)
    pr = oracle_params(RING)
    say("ring 2^16 operations")
    m, col = ops_inputs(pr)
    k1, k2 = gold["elements"]
    sk, pk = ctx.keygen(OPS_SK)
    assert [int(x) for x in ctx.export_sk(sk)[:64]] == gold["sk"]
    check(ctx.export_pk(pk), gold["pk"], "pk")
    ct = ctx.encrypt(pk, m, OPS_ENC)
    check(to_host(ct).reshape(2, ctx.L, ctx.n), gold["ct"], "encrypt")
    gk = ctx.galois_keygen(sk, [k1, k2], OPS_GK)
    check(ctx.export_gk(gk, k1), gold["gk_k1"], "galois key")
    rot = to_host(ctx.rotate(gk, k1, ct)).reshape(2, ctx.L, ctx.n)
    check(rot, gold["rotate_k1"], "rotate, 27 primes")
    assert np.array_equal(ctx.decrypt(sk, rot), np.roll(m, -1, axis=1))
    hs = to_host(ctx.rotate_hoisted(gk, [k1, k2], ct))
    check(hs, gold["hoisted_k1_k2"], "hoisted rotations, 27 primes")
    mp = ctx.mul_plain(ct, col)
    check(to_host(mp).reshape(2, ctx.L, ctx.n), gold["mul_plain"], "Mask product, 24 primes")
    ms = ctx.mod_switch(mp, ctx.L, 3)
    check(to_host(ms).reshape(2, 3, ctx.n), gold["switch_24_3"], "switch 24 -> 3")
    rl = ctx.rotate_level(gk, k1, 3, ms)
    check(to_host(rl).reshape(2, 3, ctx.n), gold["rotate_level3_k1"], "rotate, key restricted to 3 primes")
    o1 = to_host(ctx.mod_switch(rl, 3, 1)).reshape(2, 1, ctx.n)
    check(o1, gold["switch_3_1"], "switch 3 -> 1")
    assert np.array_equal(ctx.decrypt(sk, o1), np.roll(m * col % pr.p, -1, axis=1))


def test_reduced_large_parameters_bit_identical_to_oracle():
    """One ciphertext of records (2^16), t = 16, 4 columns at the full ring-2^16
    parameters: the answer at the Comp level (3 primes) and switched to one prime."""
    from oracle import slots
    gold = load("ring65536_reduced.json")
    wl = W.WORKLOADS["reduced-65536"]
    ctx = context(RING)
    say("reduced large instance")
    v, db = W.query_inputs(wl)
    keys, info = ctx.plan(wl.N, wl.ncol, wl.t)
    assert keys == gold["keys"] and info["s"] == gold["s"] and info["bands"] == gold["bands"]
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    vm = slots.vector_to_slot_matrices(v, ctx.n, 1)
    cts = ctx.ct_tensor(1)
    ctx.encrypt(pk, vm[0], W.seed32("enc", 0, 0), out=cts[0])
    out, info = ctx.compress(gk, dbh, cts, wl.N, wl.t)
    assert info["level"] == gold["level"] == 3
    check(to_host(ctx.output(out, info)), gold["compress_level3"], "compression at 3 primes")
    out1, info1 = ctx.compress(gk, dbh, cts, wl.N, wl.t, out_level=1)
    assert info1["level"] == 1 and info1["comp_level"] == 3
    check(to_host(ctx.output(out1, info1)), gold["compress_level1"], "compression, one-prime answer")
    say("oracle noise bits: level 3 %d of %d, level 1 %d of %d" % (
        gold["noise_bits_level3"], gold["budget_bits_level3"], gold["noise_bits_level1"], gold["budget_bits_level1"]))


def test_reduced_large_batch_equals_single_calls():
    """Three queries of the reduced instance (own index vectors, one ciphertext each) in
    one batched call at the full ring-2^16 parameters, so one launch of the fused Mask /
    inverse-transform pass serves every query's jobs: each answer equals its query's
    single call, and the first query's equals the oracle's stored digest."""
    from oracle import slots
    from paper_2408_17063_amd import hc
    gold = load("ring65536_reduced.json")
    wl = W.WORKLOADS["reduced-65536"]
    ctx = context(RING)
    say("reduced large instance, batch of 3")
    v0, db = W.query_inputs(wl)
    keys, _ = ctx.plan(wl.N, wl.ncol, wl.t)
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    vs = [v0] + [W.query_inputs(wl, query=q)[0] for q in (1, 2)]
    qs = []
    for qi, v in enumerate(vs):
        vm = slots.vector_to_slot_matrices(v, ctx.n, 1)
        cts = ctx.ct_tensor(1)
        ctx.encrypt(pk, vm[0], W.seed32("enc", 0, 0) if qi == 0 else W.seed32("enc", 7, qi), out=cts[0])
        qs.append((cts, wl.N, wl.t, ctx.ct_tensor(1)[0]))
    st, statuses, infos = ctx.compress_batch(gk, dbh, qs)
    assert st == hc.HC_OK and all(x == hc.HC_OK for x in statuses)
    for qi, ((cts, N, t, o), inf) in enumerate(zip(qs, infos)):
        alone, ainfo = ctx.compress(gk, dbh, cts, N, t)
        got = to_host(ctx.output(o, inf))
        assert np.array_equal(got, to_host(ctx.output(alone, ainfo))), qi
        if qi == 0:
            check(got, gold["compress_level3"], "batched reduced instance at 3 primes")


def test_headline_query_decrypts_and_decompresses():
    """The benchmark query itself (resident diagonals, as timed): the one-prime answer
    decrypts to Eq. (1)'s products in all 6 bands and decompresses exactly; the
    on-the-fly path gives the same bits; noise margins are measured."""
    from oracle import bfv, compress as C, slots
    from paper_2408_17063_amd import hc
    wl = W.WORKLOADS["large-65536"]
    ctx = context(RING)
    pr = oracle_params(RING)
    say("headline query: keys")
    v, db = W.query_inputs(wl)
    keys, plan = ctx.plan(wl.N, wl.ncol, wl.t)
    assert len(keys) == 145 and plan["n_keyswitch"] == 1549 and plan["bands"] == 6
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    n_ct = -(-wl.N // ctx.n)
    vm = slots.vector_to_slot_matrices(v, ctx.n, n_ct)
    cts = ctx.ct_tensor(n_ct)
    for i in range(n_ct):
        ctx.encrypt(pk, vm[i], W.seed32("enc", 0, i), out=cts[i])
    say("headline query: on the fly")
    fly, finfo = ctx.compress(gk, dbh, cts, wl.N, wl.t)
    fly3 = to_host(ctx.output(fly, finfo)).copy()
    say("headline query: resident")
    try:
        ctx.diag_prepare(wl.N, wl.ncol, wl.t)
        out, info = ctx.compress(gk, dbh, cts, wl.N, wl.t, out_level=1)
        assert info["n_diag"] == 0 and info["level"] == 1 and info["comp_level"] == 3
        ans = to_host(ctx.output(out, info)).copy()
        out3, info3 = ctx.compress(gk, dbh, cts, wl.N, wl.t)
        assert np.array_equal(to_host(ctx.output(out3, info3)), fly3)
    finally:
        ctx.diag_release()
    # the answer is the level-3 result switched to one prime
    sw = to_host(ctx.mod_switch(to_dev(fly3), 3, 1)).reshape(2, 1, ctx.n)
    assert np.array_equal(sw, ans)
    say("headline query: decrypt and decompress")
    sched = C.make_schedule(ctx.n, ctx.p, wl.N, wl.ncol, wl.t)
    dec = ctx.decrypt(sk, ans)
    assert np.array_equal(dec, ctx.decrypt(sk, fly3))
    exp = C.expected_bands(sched, v, db)
    for b in range(sched.bands):
        assert C.band_slots(sched, dec, b) == exp[b], b
    S = len(sched.streams)
    for gi, grp in enumerate(sched.groups):
        rows = []
        for st in range(S):
            rows += list(C.band_slots(sched, dec, gi * S + st))
        idx, vals = hc.decompress(ctx.p, grp.n_rec, sched.s, rows[0], rows[1:1 + wl.ncol])
        seg = v[grp.rec_start:grp.rec_start + grp.n_rec]
        want = [int(i) + 1 for i in np.nonzero(seg)[0]]
        assert idx == want and len(want) > 400
        for c in range(wl.ncol):
            assert vals[c] == [int(db[c][grp.rec_start + i - 1]) % ctx.p for i in want]
    # noise left (the oracle's secret equals the library's, checked above)
    osk = bfv.SecretKey(ctx.export_sk(sk))
    p3 = bfv.at_level(pr, 3)
    p1 = bfv.at_level(pr, 1, keyswitch=False)
    n3 = bfv.noise_bits(p3, osk, bfv.Ciphertext.from_stack(fly3, p3.q))
    n1 = bfv.noise_bits(p1, osk, bfv.Ciphertext.from_stack(ans, p1.q))
    say("headline noise bits: level 3 %d of %d, one-prime answer %d of %d" % (
        n3, bfv.noise_budget_bits(p3), n1, bfv.noise_budget_bits(p1)))
    assert n3 < bfv.noise_budget_bits(p3) - 20 and n1 < bfv.noise_budget_bits(p1) - 8
