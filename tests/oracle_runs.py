"""Oracle compressions of many small queries, run in parallel worker processes.

Test infrastructure: each worker recomputes one query's inputs from its seeds
(the input generators in workloads/), the oracle's keys and encryptions, and the
oracle's compression; only CPU work happens there (the workers are started with
"spawn", so they share no device state with the test process)."""
import os
from multiprocessing import get_context

import numpy as np

import workloads as W


def _one(args):
    from oracle import bfv, compress as C, slots
    from oracle.params import make_params
    ring_name, N, t, ncol, seed, qi, db, level, out_level = args
    r = W.RINGS[ring_name]
    pr = make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)
    sched = C.make_schedule(pr.n, pr.p, N, ncol, t)
    sk, pk = bfv.keygen(pr, W.seed32("sk", seed))
    gks = {k: bfv.galois_keygen(pr, sk, k, W.seed32("gk", seed)) for k in sched.keys}
    v = W.index_vector(W.rng_for(seed, qi + 1), N, t)
    vm = slots.vector_to_slot_matrices(v, pr.n, sched.n_ct)
    cts = [bfv.encrypt(pr, pk, vm[i], W.seed32("enc", seed, qi, i)) for i in range(sched.n_ct)]
    return C.compress(pr, sched, cts, db, gks, level=level, out_level=out_level).stack()


def oracle_outputs(ring_name, specs, ncol, seed, db, level=None, out_level=None):
    """The oracle's output ciphertext ([2][level][n] uint64) of query qi = (N, t) of
    specs, with the inputs tests.test_gpu_batch.make_queries gives the library."""
    jobs = [(ring_name, N, t, ncol, seed, qi, np.asarray(db), level, out_level) for qi, (N, t) in enumerate(specs)]
    procs = max(1, min(8, os.cpu_count() or 1, len(jobs)))
    with get_context("spawn").Pool(procs) as pool:
        return pool.map(_one, jobs)
