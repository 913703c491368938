"""The serving loop (hc_server_*): requests submitted as they arrive are answered by
continuous batching, and every result is bit-identical to the same query
compressed alone and to the oracle's compression of that query."""
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, to_host, say
from tests.test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu


def run_server(ring, specs, ncol, seed, values, delays_ms, lanes=2, max_batch=4, prepare=True, out_level=0):
    from paper_2408_17063_amd import hc
    from tests.oracle_runs import oracle_outputs
    ctx = context(ring)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, ring, specs, ncol, seed, values)
    oracle = oracle_outputs(ring, specs, ncol, seed, db, out_level=out_level or None)
    alone = []
    for q in qs:
        o, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"], out_level=out_level)
        alone.append((to_host(ctx.output(o, info)), info))
    for (want, _), ow in zip(alone, oracle):
        assert np.array_equal(want, ow)
    if prepare:
        for N, t in specs:
            ctx.diag_prepare(N, ncol, t)
    srv = hc.Server(ctx, gk, dbh, lane_bytes=2 << 30, lanes=lanes, max_batch=max_batch, out_level=out_level)
    try:
        outs = [ctx.ct_tensor(1)[0] for _ in qs]
        ids = []
        for q, o, d in zip(qs, outs, delays_ms):
            if d:
                time.sleep(d / 1e3)
            ids.append(srv.submit(q["cts"], q["N"], q["t"], o))
        results = {}
        deadline = time.time() + 60
        while len(results) < len(ids) and time.time() < deadline:
            for r in srv.poll(cap=16, timeout_ms=100):
                results[r["id"]] = r
        stats = srv.stats()
    finally:
        srv.close()
        ctx.diag_release()
    assert len(results) == len(ids)
    for qi, (rid, o, (want, ainfo)) in enumerate(zip(ids, outs, alone)):
        r = results[rid]
        assert r["status"] == hc.HC_OK
        assert r["submit_ns"] <= r["start_ns"] <= r["done_ns"]
        assert r["info"]["level"] == ainfo["level"] and r["info"]["s"] == ainfo["s"]
        got = to_host(ctx.output(o, r["info"]))
        assert np.array_equal(got, want), rid
        assert np.array_equal(got, oracle[qi]), rid
    return stats, results


def test_server_results_equal_alone_small_ring():
    say("server ring 2048")
    specs = [(3 * 2048, 5), (7 * 2048, 13), (1000, 1), (7 * 2048 - 100, 30), (2048, 2), (5 * 2048, 9),
             (4 * 2048, 16), (6 * 2048, 3), (2 * 2048, 7), (7 * 2048, 11), (2048, 1), (3 * 2048 + 17, 20)]
    rng = np.random.default_rng(5)
    # a burst of six, then arrivals a few milliseconds apart
    delays = [0] * 6 + [float(x) for x in rng.exponential(3.0, size=len(specs) - 6)]
    stats, results = run_server("ring-2048-p12289", specs, 4, 31, "zp", delays)
    assert stats["submitted"] == stats["completed"] == len(specs)
    assert stats["max_batch_seen"] >= 2          # requests shared a batch
    assert stats["max_lanes_busy"] >= 2          # two batches on the device at once
    assert stats["batches"] < len(specs)


def test_server_on_the_fly_diagonals_and_one_lane():
    """Without resident tables and with one lane the results are still exact."""
    say("server on the fly")
    specs = [(2 * 2048, 5), (7 * 2048, 13), (2048, 3), (4 * 2048, 8)]
    stats, _ = run_server("ring-2048-p12289", specs, 4, 32, "zp", [0, 0, 1.0, 0], lanes=1, max_batch=3,
                          prepare=False)
    assert stats["completed"] == len(specs) and stats["max_lanes_busy"] == 1


def test_server_one_prime_answers():
    """Answers switched to one prime after the merge, served in a mix."""
    say("server one-prime answers")
    specs = [(3 * 2048, 5), (7 * 2048, 13), (2048, 2), (5 * 2048, 9), (6 * 2048, 3)]
    stats, _ = run_server("ring-2048-p12289", specs, 4, 33, "zp", [0, 0, 0, 2.0, 0], out_level=1)
    assert stats["completed"] == len(specs)


def test_server_rejects_bad_requests():
    from paper_2408_17063_amd import hc
    say("server errors")
    ctx = context("ring-1024-p12289")
    sk, pk = ctx.keygen(W.seed32("sk", 7))
    keys, _ = ctx.plan(1024, 1, 5)
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 7))
    db = ctx.db_upload(np.zeros((1, 1024), dtype=np.uint32))
    srv = hc.Server(ctx, gk, db, lane_bytes=64 << 20, lanes=1, max_batch=2)
    try:
        cts = ctx.ct_tensor(1)
        out = ctx.ct_tensor(1)[0]
        with pytest.raises(hc.HcError) as e:
            srv.submit(cts, 2048, 5, out)          # more records than the database holds
        assert e.value.status == hc.HC_EINVAL
        with pytest.raises(hc.HcError) as e:
            srv.submit(cts, 1024, 300, out)        # needs Galois keys gk lacks
        assert e.value.status in (hc.HC_ENOKEY, hc.HC_EINVAL)
        assert srv.stats()["submitted"] == 0
    finally:
        srv.close()
