"""Per-launch kernel timing (hc_timing_*) and the device probes (hc_probe_*): the timed
kernel classes of a compression report launches and durations that fit inside the
compression's own device time, timing leaves the output unchanged, and the probes run
and check their arguments."""
import numpy as np
import pytest
import torch

from tests.gpu_common import context, to_host, say
from tests.test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu

RING = "ring-2048-p12289"


def test_timed_classes_fit_the_compression_and_leave_the_output_unchanged():
    from paper_2408_17063_amd import hc
    say("timing: one compression at ring 2048")
    ctx = context(RING)
    sk, pk, gk, dbh, db, qs = make_queries(ctx, RING, [(7 * 2048, 13)], 4, 5)
    q = qs[0]
    base, info = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
    want = to_host(ctx.output(base, info)).copy()
    torch.cuda.synchronize()
    ctx.timing(True)
    try:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out, info2 = ctx.compress(gk, dbh, q["cts"], q["N"], q["t"])
        e1.record()
        torch.cuda.synchronize()
        total = e0.elapsed_time(e1)
        recs = {name: ctx.timing_read(kind) for kind, name in hc.KT_NAMES.items()}
    finally:
        ctx.timing(False)
    assert np.array_equal(to_host(ctx.output(out, info2)), want)
    timed = {name: r for name, r in recs.items() if r["launches"]}
    assert {"ntt_forward", "ntt_inverse", "keyswitch_inner", "diag_mac"} <= set(timed), recs
    for name, r in timed.items():
        assert r["ms"] > 0 and r["bytes"] > 0 and r["ops"] > 0, (name, r)
    # one stream: the timed kernels ran one after another inside the bracketing events
    assert sum(r["ms"] for r in timed.values()) <= total * 1.02 + 0.05, (timed, total)
    # a fresh enable clears the records
    ctx.timing(True)
    ctx.timing(False)
    assert all(ctx.timing_read(kind)["launches"] == 0 for kind in hc.KT_NAMES)


def test_probes_run_and_check_their_arguments():
    from paper_2408_17063_amd import hc
    ctx = context(RING)
    assert ctx.probe_stream(64 << 20, 8 << 20, 2) > 0
    assert ctx.probe_stream(64 << 20, 0, 1) > 0  # reads only
    with pytest.raises(hc.HcError):
        ctx.probe_stream(8, 0, 1)
    with pytest.raises(hc.HcError):
        ctx.probe_stream(1 << 20, 0, 0)
    ctx.probe_copy(1 << 20)
    assert ctx.probe_mul32_rate(5.0) > 1e12
