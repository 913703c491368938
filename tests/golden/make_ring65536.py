"""Writes tests/golden/ring65536_ops.json and tests/golden/ring65536_reduced.json:
expected outputs at the large workload's ring and moduli (n = 2^16, 24 x 55-bit
ciphertext primes, 3 x 60-bit special primes, p = 786433), computed by the CPU
oracle alone (oracle/ and the input generators in workloads/; nothing else).

Each stored value is the SHA-256 of the result's words in the library's exchange
layout (little-endian uint64, coefficient domain, canonical residues) plus a few
sampled words, so a test can compare a device result bit for bit without
keeping megabytes of expected data.

  python tests/golden/make_ring65536.py [ops|reduced|all]

ops:     keygen, encryption, one Galois key, plain and hoisted rotation with all 27
         primes, a plaintext product at 24 primes (Mask), the 24 -> 3 prime switch,
         a rotation with the key restricted to 3 primes, the 3 -> 1 prime switch.
reduced: one whole compression (Mask + Comp, Alg. 7) of 2^16 records, t = 16,
         4 value columns, at the Comp level of 3 primes, and its answer switched
         to one prime.
"""
import hashlib
import json
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import bfv, compress as C  # noqa: E402
from oracle.params import make_params  # noqa: E402

RING = "ring-65536"
SAMPLE = 48  # sampled words per result


def params():
    r = W.RINGS[RING]
    return make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)


def digest(arr):
    a = np.ascontiguousarray(arr, dtype=np.uint64)
    flat = a.reshape(-1)
    idx = np.linspace(0, flat.size - 1, SAMPLE).astype(np.int64)
    return {"shape": list(a.shape), "sha256": hashlib.sha256(flat.astype("<u8").tobytes()).hexdigest(),
            "sample_index": [int(i) for i in idx], "sample": [int(flat[i]) for i in idx]}


def gk_stack(gk):
    return np.stack([np.stack([b.c, a.c]) for b, a in gk.digits])


def _keygen_one(args):
    k, seed = args
    pr = params()
    sk, _ = bfv.keygen(pr, W.seed32("sk", 0) if seed == "reduced" else OPS_SK)
    return k, bfv.galois_keygen(pr, sk, k, W.seed32("gk", 0) if seed == "reduced" else OPS_GK)


OPS_SK = W.seed32("sk", 65536)
OPS_GK = W.seed32("gk", 65536)
OPS_ENC = W.seed32("enc", 65536)


def ops_inputs(pr):
    rng = W.rng_for(65536, 1)
    m = rng.integers(0, pr.p, size=(2, pr.nh), dtype=np.int64)
    col = rng.integers(0, 1 << 16, size=(2, pr.nh), dtype=np.int64)  # a Mask operand
    return m, col


def make_ops():
    pr = params()
    t0 = time.time()
    sk, pk = bfv.keygen(pr, OPS_SK)
    m, col = ops_inputs(pr)
    k1, k2 = bfv.rot_row_element(pr, 1), bfv.rot_row_element(pr, 2)
    with get_context("spawn").Pool(2) as pool:
        gks = dict(pool.map(_keygen_one, [(k1, "ops"), (k2, "ops")]))
    print("keys", time.time() - t0, flush=True)
    ct = bfv.encrypt(pr, pk, m, OPS_ENC)
    out = {"_source": __doc__.strip().splitlines()[0], "ring": RING, "seeds": ["sk 65536", "gk 65536",
                                                                                 "enc 65536"],
           "elements": [k1, k2]}
    out["sk"] = [int(x) for x in sk.s[:64]]
    out["pk"] = digest(np.stack([pk.b.c, pk.a.c]))
    out["ct"] = digest(ct.stack())
    out["gk_k1"] = digest(gk_stack(gks[k1]))
    rot = bfv.rotate(pr, ct, gks[k1])
    out["rotate_k1"] = digest(rot.stack())
    print("rotate", time.time() - t0, flush=True)
    hs = bfv.rotate_hoisted(pr, ct, [gks[k1], gks[k2]])
    out["hoisted_k1_k2"] = digest(np.stack([h.stack() for h in hs]))
    print("hoisted", time.time() - t0, flush=True)
    mp = bfv.mul_plain(pr, ct, bfv.plain_poly(pr, col))
    out["mul_plain"] = digest(mp.stack())
    ms = bfv.mod_switch(pr, mp, 3)
    out["switch_24_3"] = digest(ms.stack())
    p3 = bfv.at_level(pr, 3)
    rl = bfv.rotate(p3, ms, bfv.key_at_level(pr, gks[k1], 3))
    out["rotate_level3_k1"] = digest(rl.stack())
    o1 = bfv.mod_switch(p3, rl, 1)
    out["switch_3_1"] = digest(o1.stack())
    print("done", time.time() - t0, flush=True)
    with open(os.path.join(HERE, "ring65536_ops.json"), "w") as f:
        json.dump(out, f, indent=1)


def make_reduced():
    pr = params()
    wl = W.WORKLOADS["reduced-65536"]
    t0 = time.time()
    v, db = W.query_inputs(wl)
    sched = C.make_schedule(pr.n, pr.p, wl.N, wl.ncol, wl.t)
    sk, pk = bfv.keygen(pr, W.seed32("sk", 0))
    with get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        gks = dict(pool.map(_keygen_one, [(k, "reduced") for k in sched.keys]))
    print("keys", len(gks), time.time() - t0, flush=True)
    from oracle import slots
    vm = slots.vector_to_slot_matrices(v, pr.n, sched.n_ct)
    cts = [bfv.encrypt(pr, pk, vm[i], W.seed32("enc", 0, i)) for i in range(sched.n_ct)]
    level = C.default_level(pr)
    res = C.compress(pr, sched, cts, db, gks, level=level)
    print("compress", time.time() - t0, flush=True)
    p3 = bfv.at_level(pr, level)
    one = bfv.mod_switch(p3, res, 1)
    out = {"_source": __doc__.strip().splitlines()[0], "workload": wl.name, "level": level,
           "keys": sched.keys, "s": sched.s, "bands": sched.bands,
           "compress_level3": digest(res.stack()), "compress_level1": digest(one.stack()),
           "noise_bits_level3": bfv.noise_bits(p3, sk, res), "budget_bits_level3": bfv.noise_budget_bits(p3),
           "noise_bits_level1": bfv.noise_bits(bfv.at_level(pr, 1, keyswitch=False), sk, one),
           "budget_bits_level1": bfv.noise_budget_bits(bfv.at_level(pr, 1, keyswitch=False))}
    dec = bfv.decrypt(bfv.at_level(pr, 1, keyswitch=False), sk, one)
    exp = C.expected_bands(sched, v, db)
    out["decrypts_to_vandermonde"] = all(C.band_slots(sched, dec, b) == exp[b] for b in range(sched.bands))
    print("done", time.time() - t0, out["decrypts_to_vandermonde"], flush=True)
    with open(os.path.join(HERE, "ring65536_reduced.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("ops", "all"):
        make_ops()
    if what in ("reduced", "all"):
        make_reduced()
