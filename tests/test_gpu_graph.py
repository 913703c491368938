"""Captured compressions (hc_graph_*): a batch recorded once into a HIP graph and
replayed. Every replay is checked against the eager batched call on the same
inputs (and the first against the oracle), with the buffers refilled with other
queries and eager work and synchronisations between replays."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, to_host, say
from tests.test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu


def refill(ctx, pk, q, seed, qi, rep):
    """Encrypt a fresh index vector of the same shape into the query's ct_v buffer."""
    from oracle import slots
    v = W.index_vector(W.rng_for(seed, 1000 + 10 * rep + qi), q["N"], q["t"])
    n_ct = q["cts"].shape[0]
    vm = slots.vector_to_slot_matrices(v, ctx.n, n_ct)
    for i in range(n_ct):
        ctx.encrypt(pk, vm[i], W.seed32("enc", seed, 1000 + rep, qi, i), out=q["cts"][i])
    return v


@pytest.mark.parametrize("out_level", [0, 1])
def test_graph_replays_equal_eager_and_oracle(out_level):
    import torch
    from paper_2408_17063_amd import hc
    from tests.oracle_runs import oracle_outputs
    say("graph replays", out_level)
    ring, seed = "ring-2048-p12289", 51
    specs = [(3 * 2048, 5), (7 * 2048, 13), (1000, 1)]
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, specs, 4, seed)
    outs = [ctx.ct_tensor(1)[0] for _ in qs]
    g = ctx.graph(gk, dbh, [(q["cts"], q["N"], q["t"], o) for q, o in zip(qs, outs)], out_level=out_level)
    assert g.nodes() > 20
    want0 = oracle_outputs(ring, specs, 4, seed, db, out_level=out_level or None)
    other = ctx.ct_tensor(1)[0]
    for rep in range(4):
        if rep > 0:
            for qi, q in enumerate(qs):
                refill(ctx, pk, q, seed, qi, rep)
        g.launch()
        torch.cuda.synchronize()
        got = [to_host(ctx.output(o, i)).copy() for o, i in zip(outs, g.infos)]
        # eager batched call on the same inputs, into other buffers
        eouts = [ctx.ct_tensor(1)[0] for _ in qs]
        st, _, einfos = ctx.compress_batch(gk, dbh, [(q["cts"], q["N"], q["t"], o) for q, o in zip(qs, eouts)],
                                           out_level=out_level)
        assert st == hc.HC_OK and einfos == g.infos
        for qi in range(len(qs)):
            assert np.array_equal(got[qi], to_host(ctx.output(eouts[qi], einfos[qi]))), (rep, qi)
            if rep == 0:
                assert np.array_equal(got[qi], want0[qi]), qi
        # unrelated eager work between replays
        ctx.compress(gk, dbh, qs[0]["cts"], qs[0]["N"], qs[0]["t"], out=other)
        torch.cuda.synchronize()


def test_graph_single_query_resident_ring_32768():
    """A one-query graph at ring 2^15 reading resident diagonal tables decrypts to the
    Vandermonde products on every replay and equals the eager call."""
    import torch
    from oracle import compress as C
    say("graph ring 32768")
    ring, seed = "ring-32768", 52
    specs = [(1 << 15, 256)]
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, specs, 1, seed, values="u16")
    q = qs[0]
    try:
        ctx.diag_prepare(q["N"], 1, q["t"])
        out = ctx.ct_tensor(1)[0]
        g = ctx.graph(gk, dbh, [(q["cts"], q["N"], q["t"], out)])
        assert g.infos[0]["n_diag_resident"] > 0
        for rep in range(3):
            v = q["v"] if rep == 0 else refill(ctx, pk, q, seed, 0, rep)
            g.launch()
            eager, einfo = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
            got = to_host(ctx.output(out, g.infos[0]))
            assert np.array_equal(got, to_host(ctx.output(eager, einfo))), rep
            sched = C.make_schedule(ctx.n, ctx.p, q["N"], 1, q["t"])
            dec = ctx.decrypt(sk, got)
            assert C.band_slots(sched, dec, 0) == C.expected_bands(sched, v, db)[0], rep
            torch.cuda.synchronize()
        del g
    finally:
        ctx.diag_release()
