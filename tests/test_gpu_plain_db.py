"""The unencrypted-database form (hc_compress_plain_db; Sec. 5.2, remark on an
unencrypted database): [C; C diag(DB)] v on the index vector alone. Bit-identical to
the oracle's compress_plain_db on small rings (one or several groups and streams,
answers at the Comp level or switched to one prime); at ring 2^15 and at the large
workload's parameters the answer decrypts to Eq. (1)'s products and decompresses."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, oracle_params, to_host, say

pytestmark = pytest.mark.gpu


def run_lib(wl_name, out_level=0, resident=False):
    from oracle import slots
    wl = W.WORKLOADS[wl_name]
    ctx = context(wl.ring)
    v, db = W.query_inputs(wl)
    keys, plan = ctx.plan_plain_db(wl.N, wl.ncol, wl.t, out_level=out_level)
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    n_ct = -(-wl.N // ctx.n)
    vm = slots.vector_to_slot_matrices(v, ctx.n, n_ct)
    cts = ctx.ct_tensor(n_ct)
    for i in range(n_ct):
        ctx.encrypt(pk, vm[i], W.seed32("enc", 0, i), out=cts[i])
    out, info = ctx.compress_plain_db(gk, dbh, cts, wl.N, wl.t, out_level=out_level)
    return dict(ctx=ctx, wl=wl, v=v, db=db, keys=keys, plan=plan, sk=sk, out=to_host(ctx.output(out, info)).copy(),
                info=info)


def check_decrypts(run):
    from oracle import compress as C
    from paper_2408_17063_amd import hc
    ctx, wl, v, db = run["ctx"], run["wl"], run["v"], run["db"]
    sched = C.make_schedule(ctx.n, ctx.p, wl.N, wl.ncol, wl.t)
    dec = ctx.decrypt(run["sk"], run["out"])
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
        assert idx == want
        for c in range(wl.ncol):
            assert vals[c] == [int(db[c][grp.rec_start + i - 1]) % ctx.p for i in want]


@pytest.mark.parametrize("wl_name,out_level", [("tiny-1024", 0), ("multi-2048", 0), ("multi-2048", 1),
                                               ("plain-4096", 1), ("fold-1024-q60", 0)])
def test_plain_db_bit_identical_to_oracle(wl_name, out_level):
    from oracle import bfv, compress as C, slots
    say("plain db parity", wl_name, out_level)
    run = run_lib(wl_name, out_level)
    wl = run["wl"]
    pr = oracle_params(wl.ring)
    sched = C.make_schedule(pr.n, pr.p, wl.N, wl.ncol, wl.t)
    assert run["keys"] == C.plain_db_schedule(sched).keys
    osk, opk = bfv.keygen(pr, W.seed32("sk", 0))
    gks = {k: bfv.galois_keygen(pr, osk, k, W.seed32("gk", 0)) for k in run["keys"]}
    vm = slots.vector_to_slot_matrices(run["v"], pr.n, sched.n_ct)
    octs = [bfv.encrypt(pr, opk, vm[i], W.seed32("enc", 0, i)) for i in range(sched.n_ct)]
    want = C.compress_plain_db(pr, sched, octs, run["db"], gks, out_level=out_level or None)
    assert np.array_equal(run["out"], want.stack())
    assert run["info"]["n_keyswitch"] == run["plan"]["n_keyswitch"]
    check_decrypts(run)


@pytest.mark.parametrize("wl_name", ["single-32768", "large-65536"])
def test_plain_db_full_size_decrypts(wl_name):
    say("plain db full size", wl_name)
    run = run_lib(wl_name, out_level=1)
    assert run["info"]["level"] == 1
    check_decrypts(run)
