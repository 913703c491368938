"""The autotuner's kernel variants are bit-neutral: every multiply-accumulate variant
(terms per stage x stages in flight) and every 64-bit NTT variant (register budgets,
persistent grid) gives the same compressed ciphertext as the default, which the
oracle pins; hc_autotune times them all and keeps the fastest."""
import numpy as np
import pytest

from tests.gpu_common import context, to_host, say
from tests.test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu


def outputs_for_variants(ring, specs, ncol, seed, values, variants, resident=False):
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, specs, ncol, seed, values)
    res = {}
    try:
        if resident:
            for N, t in specs:
                ctx.diag_prepare(N, ncol, t)
        for mv, nv in variants:
            ctx.tune_set(mv, nv)
            outs = []
            for q in qs:
                o, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
                outs.append(to_host(ctx.output(o, info)).copy())
            res[(mv, nv)] = outs
    finally:
        ctx.tune_set(0, 0)
        if resident:
            ctx.diag_release()
    return ctx, sk, gk, dbh, db, qs, res


@pytest.mark.parametrize("resident", [False, True])
def test_mac_variants_bit_identical_small_ring(resident):
    from tests.oracle_runs import oracle_outputs
    say("mac variants", resident)
    specs = [(7 * 2048, 13), (3 * 2048, 40)]
    variants = [(v, 0) for v in range(3)]
    ctx, sk, gk, dbh, db, qs, res = outputs_for_variants("ring-2048-p12289", specs, 4, 61, "zp", variants, resident)
    want = oracle_outputs("ring-2048-p12289", specs, 4, 61, db)
    for key, outs in res.items():
        for qi in range(len(specs)):
            assert np.array_equal(outs[qi], want[qi]), (key, qi)


def test_ntt_and_mac_variants_bit_identical_ring_32768():
    """At ring 2^15 (two-pass NTT: every NTT variant is used) all combinations agree."""
    say("ntt variants")
    specs = [(1 << 15, 64), (2 << 15, 16)]
    variants = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 3), (2, 1)]
    ctx, sk, gk, dbh, db, qs, res = outputs_for_variants("ring-32768", specs, 1, 62, "u16", variants)
    base = res[(0, 0)]
    for key, outs in res.items():
        for qi in range(len(specs)):
            assert np.array_equal(outs[qi], base[qi]), (key, qi)


def test_autotune_picks_fastest_and_keeps_bits():
    from paper_2408_17063_amd import hc
    say("autotune")
    ring = "ring-32768"
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, [(1 << 15, 64)], 1, 63, "u16")
    q = qs[0]
    o, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
    base = to_host(ctx.output(o, info)).copy()
    try:
        rep = ctx.autotune(gk, dbh, q["cts"], q["N"], q["t"])
        assert all(x > 0 for x in rep["mac_ms"]) and all(x > 0 for x in rep["ntt_ms"])
        assert rep["mac_ms"][rep["mac_variant"]] == min(rep["mac_ms"])
        assert rep["ntt_ms"][rep["ntt_variant"]] == min(rep["ntt_ms"])
        assert ctx.tune_get() == (rep["mac_variant"], rep["ntt_variant"])
        o, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
        assert np.array_equal(to_host(ctx.output(o, info)), base)
        with pytest.raises(hc.HcError):
            ctx.tune_set(3, 0)
        with pytest.raises(hc.HcError):
            ctx.tune_set(0, 4)
    finally:
        ctx.tune_set(0, 0)
