"""The int8 matrix-core multiply-accumulate (resident tables in the digit layout)
against the oracle and against the split-word vector kernel: the same words."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, to_host, say
from tests.test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu

RING = "ring-1024-p12289"
# three queries of one (s, B) class: s = 64, B = 2, 24 u-blocks -> J = 48 terms (less than
# one 64-term block), 32 giants (two tiles), 3 pairs each -> 9 pairs, two groups of 8
SPECS = [(12 * 1024, 40), (12 * 1024 - 300, 60), (11 * 1024, 33)]
NCOL = 4
SEED = 31


def digit_table_bytes(levels, n, J, G):
    return levels * n * (-(-G // 16)) * (-(-J // 64)) * 7 * 1024


def test_digit_layout_batch_matches_oracle_and_split_layout():
    from paper_2408_17063_amd import hc
    from tests.oracle_runs import oracle_outputs
    say("mfma: batch of 9 pairs at ring 1024")
    ctx = context(RING)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, RING, SPECS, NCOL, SEED)
    keys, plan = ctx.plan(SPECS[0][0], NCOL, SPECS[0][1])
    assert plan["s"] == 64 and plan["bands"] == 3
    batch = lambda outs: [(q["cts"], q["N"], q["t"], o) for q, o in zip(qs, outs)]
    outs = {}
    try:
        for layout in (hc.DIAG_LAYOUT_AUTO, hc.DIAG_LAYOUT_SPLIT):
            ctx.diag_release()
            ctx.diag_layout(layout)
            held = ctx.diag_prepare(SPECS[0][0], NCOL, 64)
            if layout == hc.DIAG_LAYOUT_AUTO:
                assert held == digit_table_bytes(plan["level"], ctx.n, 48, 32)
            else:
                assert held == plan["level"] * ctx.n * 48 * 32 * 8
            o = [ctx.ct_tensor(1)[0] for _ in qs]
            st, statuses, infos = ctx.compress_batch(gk, dbh, batch(o))
            assert st == hc.HC_OK and all(x == hc.HC_OK for x in statuses)
            assert all(i["n_diag"] == 0 for i in infos)
            outs[layout] = [to_host(ctx.output(x, i)).copy() for x, i in zip(o, infos)]
            # single-query calls (one pair group) from the same table
            for q, want in zip(qs, outs[layout]):
                alone, ainfo = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
                assert np.array_equal(to_host(ctx.output(alone, ainfo)), want)
    finally:
        ctx.diag_release()
        ctx.diag_layout(hc.DIAG_LAYOUT_AUTO)
    for a, b in zip(outs[hc.DIAG_LAYOUT_AUTO], outs[hc.DIAG_LAYOUT_SPLIT]):
        assert np.array_equal(a, b)
    say("mfma: oracle")
    want = oracle_outputs(RING, SPECS, NCOL, SEED, db)
    for qi in range(len(SPECS)):
        assert np.array_equal(outs[hc.DIAG_LAYOUT_AUTO][qi], want[qi]), qi


def test_digit_layout_full_shape_ring_32768_two_blocks():
    """A class with 128 terms (two 64-term blocks) and 64 giants at ring 2^15: the
    digit-layout compression equals the on-the-fly one and decrypts to Eq. (1)."""
    from oracle import compress as C
    from paper_2408_17063_amd import hc
    say("mfma: ring 32768, 128 terms")
    ring = "ring-32768"
    specs = [(8 << 15, 1500)]
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, specs, 1, 33, values="u16")
    q = qs[0]
    fly, finfo = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
    fly = to_host(ctx.output(fly, finfo)).copy()
    _, plan = ctx.plan(q["N"], 1, q["t"])
    try:
        held = ctx.diag_prepare(q["N"], 1, q["t"])
        sched = C.make_schedule(ctx.n, ctx.p, q["N"], 1, q["t"])
        J = max(g.k for g in sched.groups) * sched.groups[0].B
        G = sched.s // sched.groups[0].B
        assert (J, G) == (128, 64)
        assert held == digit_table_bytes(plan["level"], ctx.n, J, G)
        out, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
        assert info["n_diag"] == 0
        got = to_host(ctx.output(out, info))
    finally:
        ctx.diag_release()
    assert np.array_equal(got, fly)
    dec = ctx.decrypt(sk, got)
    exp = C.expected_bands(sched, q["v"], db)
    for b in range(sched.bands):
        assert C.band_slots(sched, dec, b) == exp[b]


def test_layout_argument_checked():
    from paper_2408_17063_amd import hc
    ctx = context(RING)
    with pytest.raises(hc.HcError):
        ctx.diag_layout(2)
