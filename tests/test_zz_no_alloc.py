"""The allocation-free rotation (hc_rotate_level_noalloc) against hc_rotate_level,
through the C ABI: two calls in a row per ring, the second on a smaller input
(fewer primes), each bit-identical to the allocating entry point and decrypting
to the rotated slots; a call beyond the fixed scratch is refused."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import context, to_host, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ring,levels", [("ring-2048-p12289", (4, 2)), ("ring-65536", (9, 3))])
def test_noalloc_rotation_equals_rotate_level(ring, levels):
    import torch
    from paper_2408_17063_amd import hc
    ctx = context(ring)
    say("no-alloc rotation", ring, levels)
    r = np.random.default_rng(40)
    k = pow(3, 3, 2 * ctx.n)
    sk, pk = ctx.keygen(W.seed32("sk", 40))
    gk = ctx.galois_keygen(sk, [k], W.seed32("gk", 40))
    slots = r.integers(0, ctx.p, size=(2, ctx.nh))
    ct = ctx.encrypt(pk, slots, W.seed32("enc", 40))
    for lvl in levels:
        src = ct if lvl == ctx.L else ctx.mod_switch(ct, ctx.L, lvl)
        want = ctx.rotate_level(gk, k, lvl, src)
        out = torch.empty(2 * lvl * ctx.n, dtype=torch.int64, device="cuda")
        ctx.rotate_level_noalloc(gk, k, lvl, src, out)
        got = to_host(out)
        assert np.array_equal(got, to_host(want)), (ring, lvl)
        assert np.array_equal(ctx.decrypt(sk, got), np.roll(slots, -3, axis=1)), (ring, lvl)
    if ring == "ring-65536":
        out = torch.empty(2 * ctx.L * ctx.n, dtype=torch.int64, device="cuda")
        with pytest.raises(hc.HcError) as e:
            ctx.rotate_level_noalloc(gk, k, ctx.L, ct, out)
        assert e.value.status == hc.HC_ESCRATCH
