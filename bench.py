"""Benchmark: compressions per second of the PDQ compression map on one MI355X.

Workload (one "step" = one full Answer of a PDQ query: Mask + Comp, Alg. 7):
ring degree 2^16, plaintext prime 786433, 24 x 55-bit ciphertext primes plus
3 x 60-bit special primes; 2^20 records in 16 ciphertexts; t = 1024 matches at
uniform random positions; 4 value columns of uniform 16-bit integers. Inputs
(ciphertexts, Galois keys, the encoded database) are resident in device
memory before the timed region; the output ciphertext stays on the device.

Prints one JSON line (see the README of the repository for the fields).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compressions/s at N=2^16,n=2^20,t=1024; batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def log_mem(tag):
    """Device memory free / total (GB) at a point of the run, with torch's cached share."""
    import torch
    free, total = torch.cuda.mem_get_info()
    log("memory %s: %.1f GB free of %.1f (torch holds %.1f GB)" % (tag, free / 1e9, total / 1e9,
                                                                   torch.cuda.memory_reserved() / 1e9))


def setup(wl_name):
    import numpy as np
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    wl = W.WORKLOADS[wl_name]
    r = W.RINGS[wl.ring]
    t0 = time.time()
    ctx = hc.Context(log_n=int(math.log2(r.n)), p=r.p, L=r.L, q_bits=r.q_bits, K=r.K, p_bits=r.p_bits)
    v, db = W.query_inputs(wl)
    keys, info = ctx.plan(wl.N, wl.ncol, wl.t)
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    n_ct = -(-wl.N // ctx.n)
    # record r -> ciphertext r / n, row (r % n) / (n/2), column r % (n/2)
    vm = np.zeros(n_ct * ctx.n, dtype=np.uint32)
    vm[:wl.N] = v
    vm = vm.reshape(n_ct, 2, ctx.nh)
    cts = ctx.ct_tensor(n_ct)
    for i in range(n_ct):
        ctx.encrypt(pk, vm[i], W.seed32("enc", 0, i), out=cts[i])
    torch.cuda.synchronize()
    log("setup %.1fs: %d Galois keys, %d ciphertexts, plan %s" % (time.time() - t0, len(keys), n_ct, info))
    return dict(ctx=ctx, sk=sk, pk=pk, gk=gk, db=dbh, cts=cts, v=v, dbv=db, wl=wl, info=info, keys=keys)


# VALU issue peak derived from the chip: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz =
# 39.3 T lane-instructions/s (a 64-wide VALU instruction occupies a 16-lane SIMD for 4
# cycles). The integer multiply-add the kernels use (v_mad_u64_u32) issues at that
# rate: the library's register-only probe (hc_probe_mul32_rate) measures ~35.5 T/s.
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12


def kernel_rooflines(ctx, hc):
    """Per-class totals over the timed region -> roofline objects."""
    out = {}
    for kind, name in hc.KT_NAMES.items():
        t = ctx.timing_read(kind)
        if t["launches"] == 0 or t["ms"] <= 0:
            continue
        sec = t["ms"] / 1e3
        out[name] = dict(t, sec=sec)
    rl = {}
    # the counts of the NTT pass variant in use (each variant is its own code object)
    rec = valu_per_launch()
    valu = {k: v["valu_lane_instr_per_launch"]
            for k, v in rec.get("variants", {}).get(str(ctx.tune_get()[1]), {}).items()}
    for name, t in out.items():
        if name.startswith("ntt") or name == "conv_fused":
            # VALU lane-instructions per launch counted by rocprofv3 on this same workload
            # (SQ_INSTS_VALU x 64, mean over the class's launches of a compression), times
            # the launches, over the live device time
            vpl = valu.get(name)
            ach = vpl * t["launches"] / t["sec"] / 1e12 if vpl else None
            rl[name] = {"bound": "alu", "achieved": round(ach, 3) if ach else None, "peak": round(VALU_PEAK_T, 3),
                        "unit": "T VALU lane-instr/s", "frac": round(ach / VALU_PEAK_T, 4) if ach else None,
                        "traffic": None, "valu_lane_instr_per_launch": vpl,
                        "butterflies_per_s_T": round(t["ops"] / t["sec"] / 1e12, 4),
                        "avg_launch_us": round(t["ms"] * 1e3 / t["launches"], 2),
                        "launches": t["launches"], "ms": round(t["ms"], 2)}
        else:
            ach = t["bytes"] / t["sec"] / 1e9
            rl[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_us": round(t["ms"] * 1e3 / t["launches"], 2),
                        "launches": t["launches"], "ms": round(t["ms"], 2)}
    return rl


def choose_baby(s, k):
    """The planner's baby-step count: the power of two B in [1, s] minimising
    k (B - 1) + (s / B - 1), ties to the larger B."""
    best, bb, B = None, 1, 1
    while B <= s:
        cost = k * (B - 1) + (s // B - 1)
        if best is None or cost <= best:
            best, bb = cost, B
        B *= 2
    return bb


def mac_stream_ceiling(ctx, t, info):
    """The diagonal multiply-accumulate's read and write bytes per launch (digit layout,
    one B class) replayed by the library's stream probe: contiguous reads with the same
    share of contiguous writes mixed in, an upper bound for the kernel's own pattern
    (its writes are 64-byte runs into every (pair, giant) output). t: the kernel class's
    timing record over the timed steps."""
    if t["launches"] == 0:
        return None
    s = info["s"]
    nd = info["n_diag_resident"] or info["n_diag"]
    if nd == 0 or nd % s:
        return None
    k = nd // s
    B = choose_baby(s, k)
    J, ga = k * B, s // B
    npairs = info["groups"] * info["streams"]
    ln = info["comp_level"] * ctx.n
    per_launch = t["bytes"] / t["launches"]
    expect = ln * (7.0 * J * ga + 16.0 * npairs * J + 16.0 * npairs * ga)
    if abs(per_launch - expect) > 1e-9 * expect:
        log("MAC stream probe skipped: the launches are not all of the digit-layout headline shape")
        return None
    write = ln * 16.0 * npairs * ga
    read = expect - write
    ms = ctx.probe_stream(int(read), int(write), 3)
    ceil_gbs = (read + write) / ms * 1e-6
    mac_gbs = per_launch * t["launches"] / t["ms"] * 1e-6
    return {"read_bytes": int(read), "write_bytes": int(write), "probe_ms": round(ms, 4),
            "ceiling_GBps": round(ceil_gbs, 1), "mac_GBps": round(mac_gbs, 1),
            "mac_frac_of_ceiling": round(mac_gbs / ceil_gbs, 4)}


def sources_current(rec):
    import hashlib
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest() == rec["sources_sha256"]


def valu_per_launch():
    """The committed rocprofv3 counter summary of this benchmark's own compressions:
    VALU lane-instructions per launch of each transform class, per NTT pass variant;
    empty when missing or when the kernels' sources changed since."""
    path = os.path.join(ROOT, "profiles", "valu_large-65536.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    if not sources_current(rec):
        log("VALU counter summary is stale (kernel sources changed): transform rooflines reported as null")
        return {}
    return rec


def measured_traffic(workload):
    """HBM bytes per launch from the committed counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), per kernel class;
    empty when the summary is missing or the kernels' sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        log("traffic summary is stale (kernel sources changed): traffic reported as null")
        return {}
    return {k: v["traffic_bytes_per_launch"] for k, v in rec["kernels"].items()}


def _cpu_sample(args):
    """One worker of the CPU baseline: the oracle's keys and one ciphertext at ring
    2^16, then one timed run of each sampled operation (single thread)."""
    level, seed = args
    import numpy as np
    import workloads as W
    from oracle import bfv, compress as C
    from oracle.params import make_params
    r = W.RINGS["ring-65536"]
    pr = make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)
    sk, pk = bfv.keygen(pr, W.seed32("sk", seed))
    k = bfv.rot_row_element(pr, 8)
    gk = bfv.galois_keygen(pr, sk, k, W.seed32("gk", seed))
    ct = bfv.encrypt(pr, pk, np.zeros((2, pr.nh), dtype=np.uint64), W.seed32("enc", seed, 0))
    dbm = bfv.plain_poly(pr, C.db_slots(np.arange(pr.n, dtype=np.uint32) % 65536, pr.n, 0))
    t = {}
    t0 = time.perf_counter()
    bfv.mul_plain(pr, ct, dbm)
    t["mask"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    lo = bfv.mod_switch(pr, ct, level) if level < pr.L else ct
    t["switch"] = time.perf_counter() - t0
    plo = bfv.at_level(pr, level)
    gklo = bfv.key_at_level(pr, gk, level)
    t0 = time.perf_counter()
    bfv.rotate(plo, lo, gklo)
    t["keyswitch"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    m = bfv.plain_poly(plo, C.diagonal_slots(pr.p, pr.nh, 1024, 8, 3, 5, 2))
    t["encode"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    bfv.mul_plain(plo, lo, m)
    t["ptct"] = time.perf_counter() - t0
    return t


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(info):
    """The CPU oracle on a bounded sample of the same workload, run on the host's cores.

    The oracle runs the same schedule as the library: Mask at the full modulus, a
    modulus switch of each ciphertext, then the rest at the Comp level. Sample: one
    Mask product and one modulus switch at the full modulus; one rotation (key switch),
    one diagonal encoding and one diagonal product at the Comp level; all at ring 2^16.
    The compression's operations are independent across ciphertexts, limbs and
    rotations of one phase, so the oracle parallelises over them: P worker processes
    (one per usable core, at most 16) each run the sample at once, and the host's rate
    is P compressions per the sample-scaled time of one (the workers' mean, measured
    while all run). Labelled extrapolated: no whole compression is run."""
    from multiprocessing import get_context
    model, ncpu, usable = host_cpu()
    P = max(1, min(16, usable))
    level = info["comp_level"]
    t_wall = time.perf_counter()
    with get_context("spawn").Pool(P) as pool:
        samples = pool.map(_cpu_sample, [(level, 1000 + i) for i in range(P)])
        pool.close()
        pool.join()  # every worker has exited before the result line is printed
    wall = time.perf_counter() - t_wall
    t = {k: sum(x[k] for x in samples) / P for k in samples[0]}
    n_mask = 4 * 16                      # value columns x input ciphertexts
    n_switch = 16 * (1 + 4)
    per_query = (n_mask * t["mask"] + n_switch * t["switch"] + info["n_keyswitch"] * t["keyswitch"] +
                 info["n_diag"] * t["encode"] + (info["n_ptct"] - n_mask) * t["ptct"])
    log("cpu oracle sample (%d workers, %.0fs): %s -> %.0f s per compression per core" % (
        P, wall, {a: round(b, 3) for a, b in t.items()}, per_query))
    return {"value": P / per_query, "unit": "compressions/s", "cores": P, "kind": "oracle",
            "host_cpus": ncpu, "usable_cpus": usable, "cpu_model": model,
            "sample": "oracle at ring 2^16 in %d parallel worker processes: one Mask product and one modulus "
                      "switch at 24 primes, one rotation, one diagonal encoding and one diagonal product at %d "
                      "primes per worker (mean %s s), scaled by the step's %d Mask products, %d switches, %d key "
                      "switches, %d diagonal encodings and %d other plaintext products, times %d workers"
                      % (P, level, ", ".join("%s %.3f" % kv for kv in t.items()), n_mask, n_switch,
                         info["n_keyswitch"], info["n_diag"], info["n_ptct"] - n_mask, P),
            "extrapolated": True, "wall_s": round(wall, 1)}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def answer_groups(n, p, N):
    """(first record, records) of each record group of an answer: whole ciphertexts of
    n records, balanced, at most p - 1 records per group (one band per group and stream)."""
    n_ct = -(-N // n)
    per = (p - 1) // n
    G = -(-n_ct // per)
    out, ct = [], 0
    for g in range(G):
        cnt = n_ct // G + (1 if g < n_ct % G else 0)
        out.append((ct * n, min(N, (ct + cnt) * n) - ct * n))
        ct += cnt
    return out


def answer_recovers(hc, ctx, dec, N, ncol, s, v, db):
    """Decompress every group of a decrypted answer (library decompression) and compare
    the recovered (index, values) with the query's own matching records. Band b of group
    g and stream sigma is b = g * streams + sigma, in slots [b s, (b + 1) s) of both
    slot rows (slot 0 on with a single band); streams pair [v, d_1, ..., d_ncol]."""
    import numpy as np
    groups = answer_groups(ctx.n, ctx.p, N)
    S = (ncol + 2) // 2
    bands = len(groups) * S
    for gi, (r0, nr) in enumerate(groups):
        rows = []
        for sv in range(S):
            off = (gi * S + sv) * s if bands > 1 else 0
            rows.append([int(x) for x in dec[0][off:off + s]])
            rows.append([int(x) for x in dec[1][off:off + s]])
        idx, vals = hc.decompress(ctx.p, nr, s, rows[0], rows[1:1 + ncol])
        want = [int(i) + 1 for i in np.nonzero(np.asarray(v)[r0:r0 + nr])[0]]
        if idx != want:
            return False
        for c in range(ncol):
            if vals[c] != [int(db[c][r0 + i - 1]) % ctx.p for i in want]:
                return False
    return True


def encrypt_query(ctx, pk, v, n_ct, seed_ints):
    import numpy as np
    import workloads as W
    vm = np.zeros(n_ct * ctx.n, dtype=np.uint32)
    vm[:len(v)] = v
    vm = vm.reshape(n_ct, 2, ctx.nh)
    cts = ctx.ct_tensor(n_ct)
    for i in range(n_ct):
        ctx.encrypt(pk, vm[i], W.seed32("enc", *seed_ints, i), out=cts[i])
    return cts


def batched_large(st, Q, steps, out_level=0):
    """Q queries of the headline workload (own index vectors) in one hc_compress_batch."""
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    ctx, wl = st["ctx"], st["wl"]
    pk = st["pk"]
    qs = []
    for qi in range(Q):
        v, _ = W.query_inputs(wl, query=100 + qi)
        qs.append((encrypt_query(ctx, pk, v, st["cts"].shape[0], (100 + qi,)), wl.N, wl.t, ctx.ct_tensor(1)[0]))
    ctx.compress_batch(st["gk"], st["db"], qs, out_level=out_level)  # warm-up (workspace)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ctx.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        rc, stats, _ = ctx.compress_batch(st["gk"], st["db"], qs, out_level=out_level)
        assert rc == hc.HC_OK
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for name, r in kernel_rooflines(ctx, hc).items():
        log("  batched %-16s %8.1f ms per batch %6d launches  %s %s of peak" % (
            name, r["ms"] / steps, r["launches"] // steps, r["bound"], r["frac"]))
    ctx.timing(False)
    del qs
    torch.cuda.empty_cache()
    return {"queries": Q, "ms_per_batch": round(ms, 2), "value": round(Q / (ms / 1e3), 4),
            "unit": "compressions/s"}


def plain_db_leg(st, eager_out, steps, comp_level, out_level):
    """The unencrypted-database form (hc_compress_plain_db) on the headline query: no
    Mask, [C; C diag(DB)] v with its diagonals encoded on the fly (they depend on the
    database); its answer must decrypt like the Mask + Comp answer."""
    import numpy as np
    import torch
    ctx, wl = st["ctx"], st["wl"]
    keys, plan = ctx.plan_plain_db(wl.N, wl.ncol, wl.t, comp_level, out_level)
    if not set(keys) <= set(st["keys"]):
        return {"skipped": "key set differs"}
    out = ctx.ct_tensor(1)[0]
    ctx.compress_plain_db(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=comp_level,
                          out_level=out_level)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        _, info = ctx.compress_plain_db(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=comp_level,
                                        out_level=out_level)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    a = ctx.decrypt(st["sk"], ctx.output(out, info).cpu().numpy().view(np.uint64))
    b = ctx.decrypt(st["sk"], ctx.output(eager_out, info).cpu().numpy().view(np.uint64))
    s = info["s"]
    same = all(np.array_equal(a[:, k * s:(k + 1) * s], b[:, k * s:(k + 1) * s]) for k in range(info["bands"]))
    del out
    torch.cuda.empty_cache()
    return {"steps": steps, "ms_per_step": round(ms, 3), "value": round(1e3 / ms, 4), "unit": "compressions/s",
            "key_switches": info["n_keyswitch"], "diagonals_encoded": info["n_diag"],
            "decrypts_like_mask_and_comp": bool(same)}


def products_leg(st, reps, out_level):
    """Ciphertext products at the headline parameters (ring 2^16, 24 primes): one
    hc_mul, one Power_{p-1} (x^3 then 18 squarings at p = 786433), and a whole PDQ
    Answer with Match (Alg. 7): hc_match of a query key against 2^20 record keys (16
    ciphertexts, one Power_{p-1} each), then Mask + Comp of its index vector with the
    headline database; the answer must decompress to the matching records."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    ctx, wl = st["ctx"], st["wl"]
    t0 = time.perf_counter()
    rk = ctx.relin_keygen(st["sk"], W.seed32("rk", 0))
    keygen_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    a, b = st["cts"][0], st["cts"][1]
    out = ctx.ct_tensor(1)[0]

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    mul_ms = timed(lambda: ctx.mul(rk, a, b, out=out), reps)
    pow_ms = timed(lambda: ctx.power(rk, a, ctx.p - 1, out=out), 1)
    keys, x, v = W.match_inputs(wl.N, wl.t, ctx.p, seed=5)
    kdb = ctx.db_upload(keys.reshape(1, -1))
    cx = ctx.encrypt(st["pk"], np.full((2, ctx.nh), x), W.seed32("enc-match", 0))
    ctv = ctx.ct_tensor(st["cts"].shape[0])
    match_ms = timed(lambda: ctx.match(rk, kdb, cx, wl.N, out=ctv), 1)
    ans = ctx.ct_tensor(1)[0]
    comp_ms = timed(lambda: ctx.compress(st["gk"], st["db"], ctv, wl.N, wl.t, out=ans, out_level=out_level), 1)
    _, info = ctx.compress(st["gk"], st["db"], ctv, wl.N, wl.t, out=ans, out_level=out_level)
    dec = ctx.decrypt(st["sk"], ctx.output(ans, info).cpu().numpy().view(np.uint64))
    ok = answer_recovers(hc, ctx, dec, wl.N, wl.ncol, info["s"], v, st["dbv"])
    rk.close()
    kdb.close()
    del ctv, ans
    torch.cuda.empty_cache()
    return {"relin_keygen_s": round(keygen_s, 2), "mul_ms": round(mul_ms, 3), "power_p_minus_1_ms": round(pow_ms, 2),
            "match_ms": round(match_ms, 1), "match_records": wl.N, "answer_after_match_ms": round(comp_ms, 2),
            "pdq_answer_with_match_per_s": round(1e3 / (match_ms + comp_ms), 4), "recovers_matches": bool(ok)}


def graph_leg(st, eager_out, steps, comp_level, out_level):
    """The headline compression captured once into a HIP graph (hc_graph_create) and
    replayed: same inputs, its output must equal the eager run's bit for bit."""
    import torch
    ctx, wl = st["ctx"], st["wl"]
    gout = ctx.ct_tensor(1)[0]
    t0 = time.perf_counter()
    g = ctx.graph(st["gk"], st["db"], [(st["cts"], wl.N, wl.t, gout)], comp_level=comp_level, out_level=out_level)
    cap_s = time.perf_counter() - t0
    g.launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gi = g.infos[0]
    same = bool(torch.equal(ctx.output(gout, gi), ctx.output(eager_out, gi)))
    res = {"steps": steps, "ms_per_step": round(ms, 3), "value": round(1e3 / ms, 4), "unit": "compressions/s",
           "nodes": g.nodes(), "capture_s": round(cap_s, 2), "equals_eager": same}
    g.close()
    del gout
    return res


def on_the_fly(st, resident_out, steps, comp_level, out_level=0):
    """The same compression with the resident tables released: every step encodes its
    diagonals itself. Its output must equal the resident run's bit for bit."""
    import torch
    ctx, wl = st["ctx"], st["wl"]
    ref = resident_out.clone()
    ctx.diag_release()
    out = ctx.ct_tensor(1)[0]
    ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=comp_level, out_level=out_level)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        _, info = ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=comp_level,
                               out_level=out_level)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    same = bool(torch.equal(ctx.output(out, info), ctx.output(ref, info)))
    del out, ref
    torch.cuda.empty_cache()
    return {"steps": steps, "ms_per_step": round(ms, 3), "value": round(1e3 / ms, 4),
            "unit": "compressions/s", "n_diag_encoded_per_step": info["n_diag"], "equals_resident": same}


def mixed_batch(count=64):
    """The batched configuration: `count` independent compressions over the 2^15 ring
    (14 x 55-bit + 2 x 60-bit primes), ciphertexts per query uniform in 1..32, t
    log-uniform in [16, 1024], one value column; one hc_compress_batch call vs the
    same queries as `count` sequential hc_compress calls."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    r = W.RINGS["ring-32768"]
    ctx = hc.Context(log_n=15, p=r.p, L=r.L, q_bits=r.q_bits, K=r.K, p_bits=r.p_bits)
    specs = W.batched_queries(count=count, seed=0, max_ct=32, n=ctx.n)
    Nmax = 32 * ctx.n
    rng = W.rng_for(0xBA7C, 1)
    db = W.value_columns(rng, Nmax, 1, "u16", ctx.p)
    sk, pk = ctx.keygen(W.seed32("sk", 4))
    keys = set()
    for N, t in specs:
        keys.update(ctx.plan(N, 1, t)[0])
    gk = ctx.galois_keygen(sk, sorted(keys), W.seed32("gk", 4))
    dbh = ctx.db_upload(db)
    qs = []
    for qi, (N, t) in enumerate(specs):
        v = W.index_vector(W.rng_for(0xBA7C, 2, qi), N, t)
        qs.append((encrypt_query(ctx, pk, v, N // ctx.n, (0xBA7C, qi)), N, t, ctx.ct_tensor(1)[0]))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # sequential plain calls (after one warm-up pass of the largest query)
    big = max(range(count), key=lambda i: specs[i][0])
    ctx.compress(gk, dbh, qs[big][0], qs[big][1], qs[big][2])
    lat = []
    t0 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    evs = []
    for (cts, N, t, out) in qs:
        e = torch.cuda.Event(enable_timing=True)
        ctx.compress(gk, dbh, cts, N, t, out=out)
        e.record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    prev = t0
    for e in evs:
        lat.append(prev.elapsed_time(e))
        prev = e
    seq_ms = t0.elapsed_time(evs[-1])
    singles = [out.clone() for (_, _, _, out) in qs]
    # one batched call
    ctx.compress_batch(gk, dbh, qs)
    torch.cuda.synchronize()
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    rc, stats, infos = ctx.compress_batch(gk, dbh, qs)
    b1.record(stream)
    torch.cuda.synchronize()
    assert rc == hc.HC_OK
    batch_ms = b0.elapsed_time(b1)
    same = all(torch.equal(ctx.output(out, info), ctx.output(ref, info))
               for (_, _, _, out), ref, info in zip(qs, singles, infos))
    # the same batch captured once into a graph and replayed
    log_mem("before the mixed batch's graph")
    gouts = [ctx.ct_tensor(1)[0] for _ in qs]
    g = ctx.graph(gk, dbh, [(cts, N, t, o) for (cts, N, t, _), o in zip(qs, gouts)])
    g.launch()
    torch.cuda.synchronize()
    b0.record(stream)
    g.launch()
    b1.record(stream)
    torch.cuda.synchronize()
    graph_ms = b0.elapsed_time(b1)
    same_g = all(torch.equal(ctx.output(o, info), ctx.output(ref, info))
                 for o, ref, info in zip(gouts, singles, g.infos))
    graph_nodes = g.nodes()
    g.close()
    del gouts
    # the same queries with every class's diagonals resident
    t0p = time.perf_counter()
    held = 0
    for N, t in specs:
        held = ctx.diag_prepare(N, 1, t)
    prep_s = time.perf_counter() - t0p
    ctx.compress(gk, dbh, qs[big][0], qs[big][1], qs[big][2])
    torch.cuda.synchronize()
    r0 = torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    rlat, prev = [], r0
    for (cts, N, t, out) in qs:
        ctx.compress(gk, dbh, cts, N, t, out=out)
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        rlat.append(e)
    torch.cuda.synchronize()
    rseq_ms = r0.elapsed_time(rlat[-1])
    rl_ms = []
    for e in rlat:
        rl_ms.append(prev.elapsed_time(e))
        prev = e
    same_r = all(torch.equal(ctx.output(out, info), ctx.output(ref, info))
                 for (_, _, _, out), ref, info in zip(qs, singles, infos))
    ctx.compress_batch(gk, dbh, qs)
    torch.cuda.synchronize()
    b0.record(stream)
    rc, stats, infos = ctx.compress_batch(gk, dbh, qs)
    b1.record(stream)
    torch.cuda.synchronize()
    assert rc == hc.HC_OK
    rbatch_ms = b0.elapsed_time(b1)
    same_rb = all(torch.equal(ctx.output(out, info), ctx.output(ref, info))
                  for (_, _, _, out), ref, info in zip(qs, singles, infos))
    resident = {"prepare_s": round(prep_s, 3), "bytes": held, "sequential_ms": round(rseq_ms, 2),
                "batched_ms": round(rbatch_ms, 2), "sequential_value": round(count / (rseq_ms / 1e3), 3),
                "batched_value": round(count / (rbatch_ms / 1e3), 3), "speedup": round(rseq_ms / rbatch_ms, 3),
                "sequential_p50_ms": round(percentile(rl_ms, 50), 2),
                "sequential_p99_ms": round(percentile(rl_ms, 99), 2),
                "equals_on_the_fly": bool(same_r and same_rb)}
    ctx.diag_release()
    res = {"queries": count, "ring_degree": ctx.n, "records_min": min(N for N, _ in specs),
           "records_max": max(N for N, _ in specs), "t_min": min(t for _, t in specs),
           "t_max": max(t for _, t in specs),
           "sequential_ms": round(seq_ms, 2), "batched_ms": round(batch_ms, 2),
           "sequential_value": round(count / (seq_ms / 1e3), 3), "batched_value": round(count / (batch_ms / 1e3), 3),
           "speedup": round(seq_ms / batch_ms, 3), "unit": "compressions/s",
           "graph_ms": round(graph_ms, 2), "graph_value": round(count / (graph_ms / 1e3), 3),
           "graph_speedup": round(seq_ms / graph_ms, 3), "graph_nodes": graph_nodes,
           "graph_equals_sequential": bool(same_g),
           "sequential_p50_ms": round(percentile(lat, 50), 2), "sequential_p99_ms": round(percentile(lat, 99), 2),
           "batch_equals_sequential": bool(same), "resident": resident}
    del qs, singles
    ctx.close()
    torch.cuda.empty_cache()
    return res


def serving(st, rates, requests, lane_gb=40, lanes=2, max_batch=16, out_level=0):
    """The serving configuration: a seeded Poisson stream of PDQ requests at the
    headline parameters (ring 2^16, 24 + 3 primes). Each request draws its record
    count from {2^15, 2^17, 2^20} (a prefix of the resident 2^20 x 4 database) and t
    log-uniform in [16, 1024]. Galois keys for the whole mix, the database and the
    diagonal tables of every class stay resident; the server admits requests by
    workspace footprint and batches them continuously on two streams. Latency is
    scheduled arrival -> result final on the device, as seen by the host. Each rate
    is a fraction of the plain (one query at a time, back to back) throughput of the
    same request list, measured just before it is served."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    ctx, wl = st["ctx"], st["wl"]
    sizes = [1 << 15, 1 << 17, 1 << 20]
    st["gk"].close()
    ctx.trim()
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    keys = set()
    for N in sizes:
        for sv in (16, 32, 64, 128, 256, 512, 1024):
            keys.update(ctx.plan(N, wl.ncol, sv)[0])
    gk = ctx.galois_keygen(st["sk"], sorted(keys), W.seed32("gk-serve", 0))
    held = 0
    for N in sizes:
        for sv in (16, 32, 64, 128, 256, 512, 1024):
            held = ctx.diag_prepare(N, wl.ncol, sv)
    setup_s = time.perf_counter() - t0
    log("serving setup %.1fs: %d Galois keys, %.1f GB resident diagonals" % (setup_s, len(keys), held / 1e9))
    # a pool of encrypted index vectors per record count (16 matches: valid for every t >= 16)
    pool = {}
    for N in sizes:
        pool[N] = []
        for j in range(3):
            v = W.index_vector(W.rng_for(0x5E7E, N, j), N, 16)
            pool[N].append(encrypt_query(ctx, st["pk"], v, -(-N // ctx.n), (0x5E7E, N, j)))
    rng = W.rng_for(0x5E7E, 1)

    def draw(count):
        Ns = rng.choice(sizes, size=count)
        ts = np.rint(np.exp(rng.uniform(np.log(16), np.log(1024), size=count))).astype(int)
        return [(int(N), int(t), pool[int(N)][i % 3]) for i, (N, t) in enumerate(zip(Ns, ts))]

    out = ctx.ct_tensor(1)[0]
    stream = torch.cuda.current_stream()

    def plain_ms(reqs):
        """The same requests one at a time, back to back (GPU events)."""
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for N, t, cts in reqs:
            ctx.compress(gk, st["db"], cts, N, t, out=out, out_level=out_level)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    warm = draw(6)
    plain_ms(warm)
    ctx.trim()
    torch.cuda.empty_cache()
    srv = hc.Server(ctx, gk, st["db"], lane_bytes=int(lane_gb) << 30, lanes=lanes, max_batch=max_batch,
                    out_level=out_level)
    res = {"requests_per_rate": requests, "lanes": lanes, "lane_gb": lane_gb, "max_batch": max_batch,
           "galois_keys": len(keys), "resident_diagonal_gb": round(held / 1e9, 2), "setup_s": round(setup_s, 1),
           "rates": []}
    try:
        for frac in rates:
            reqs = draw(requests)
            pms = plain_ms(reqs)  # the same request list, plain, for the capacity and the comparison
            capacity = requests / (pms / 1e3)
            lam = frac * capacity
            gaps = rng.exponential(1.0 / lam, size=requests)
            start = time.monotonic_ns() + 20_000_000
            arrive = start + np.cumsum(gaps * 1e9).astype(np.int64)
            arrival_of, lat, done_last, batch_sizes = {}, [], 0, []
            i = 0
            while len(lat) < requests:
                now = time.monotonic_ns()
                while i < requests and arrive[i] <= now:
                    N, t, cts = reqs[i]
                    rid = srv.submit(cts, N, t, ctx.ct_tensor(1)[0])
                    arrival_of[rid] = int(arrive[i])
                    i += 1
                wait_ms = 5.0 if i >= requests else max(0.0, min(5.0, (arrive[i] - time.monotonic_ns()) / 1e6))
                for r in srv.poll(cap=64, timeout_ms=wait_ms):
                    assert r["status"] == hc.HC_OK
                    lat.append((r["done_ns"] - arrival_of[r["id"]]) / 1e6)
                    done_last = max(done_last, r["done_ns"])
                    batch_sizes.append(r["batch_size"])
            span = (done_last - int(arrive[0])) / 1e9
            row = {"fraction_of_plain_capacity": frac, "plain_per_s": round(capacity, 3), "offered_per_s": round(lam, 3),
                   "throughput_per_s": round(requests / span, 3), "p50_ms": round(percentile(lat, 50), 2),
                   "p99_ms": round(percentile(lat, 99), 2), "mean_batch": round(float(np.mean(batch_sizes)), 2)}
            log("serving at %.2f x plain capacity: %s" % (frac, row))
            res["rates"].append(row)
        res["server_stats"] = srv.stats()
    finally:
        srv.close()
    return res


def small_config_latency(wl_name, reps=20, config=None):
    """Latency of one compression of a smaller benchmark configuration (ring 4096:
    configuration 1; ring 2^15: configuration 2), plain calls and graph replays, with
    the answer decrypted and decompressed to the query's matching records once."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2408_17063_amd import hc
    wl = W.WORKLOADS[wl_name]
    r = W.RINGS[wl.ring]
    ctx = hc.Context(log_n=int(math.log2(r.n)), p=r.p, L=r.L, q_bits=r.q_bits, K=r.K, p_bits=r.p_bits)
    v, db = W.query_inputs(wl)
    keys, info = ctx.plan(wl.N, wl.ncol, wl.t)
    sk, pk = ctx.keygen(W.seed32("sk", 0))
    gk = ctx.galois_keygen(sk, keys, W.seed32("gk", 0))
    dbh = ctx.db_upload(db)
    n_ct = -(-wl.N // ctx.n)
    cts = encrypt_query(ctx, pk, v, n_ct, (0,))
    out = ctx.ct_tensor(1)[0]
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1))
        return lat

    res = {"workload": wl_name, "config": config, "ring_degree": ctx.n, "records": wl.N, "t": wl.t}
    try:
        plain = timed(lambda: ctx.compress(gk, dbh, cts, wl.N, wl.t, out=out))
        ref = out.clone()
        _, info = ctx.compress(gk, dbh, cts, wl.N, wl.t, out=out)
        dec = ctx.decrypt(sk, ctx.output(out, info).cpu().numpy().view(np.uint64))
        ok = answer_recovers(hc, ctx, dec, wl.N, wl.ncol, info["s"], v, db)
        gout = ctx.ct_tensor(1)[0]
        g = ctx.graph(gk, dbh, [(cts, wl.N, wl.t, gout)])
        graph = timed(lambda: g.launch())
        same = bool(torch.equal(ctx.output(gout, g.infos[0]), ctx.output(ref, info)))
        res.update({"plain_p50_ms": round(percentile(plain, 50), 3), "plain_p99_ms": round(percentile(plain, 99), 3),
                    "graph_p50_ms": round(percentile(graph, 50), 3), "graph_p99_ms": round(percentile(graph, 99), 3),
                    "reps": reps, "key_switches": info["n_keyswitch"], "answer_recovers_matches": bool(ok),
                    "graph_equals_plain": same, "graph_nodes": g.nodes()})
        g.close()
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large-65536")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-queries", type=int, default=8,
                    help="queries of the headline workload per batched call (0: skip)")
    ap.add_argument("--mixed-batch", type=int, default=64,
                    help="queries of the mixed 2^15-ring batch (0: skip)")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="skip the read/write stream probe run beside the multiply-accumulate's roofline")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="launch one plain copy kernel of this many MiB (counter calibration)")
    ap.add_argument("--comp-level", type=int, default=0,
                    help="ciphertext primes kept for Comp (0: the library default; 24: no switching)")
    ap.add_argument("--diagonals", choices=["resident", "on-the-fly"], default="resident",
                    help="resident: precompute the query-independent diagonals once (hc_diag_prepare) "
                         "before timing; on-the-fly: encode them inside every compression")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,0.9,1.0,1.25",
                    help="serving arrival rates as fractions of the plain capacity ('' to skip)")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per serving rate")
    ap.add_argument("--serve-lanes", type=int, default=2, help="concurrent batches of the server")
    ap.add_argument("--serve-max-batch", type=int, default=16, help="queries per server batch")
    ap.add_argument("--on-the-fly-steps", type=int, default=2,
                    help="with resident diagonals, also time this many steps encoding them on the fly")
    ap.add_argument("--out-level", type=int, default=1,
                    help="primes of the answer (1: one prime, the answer form of Sec. 6.2; 0: the Comp level)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel variants")
    ap.add_argument("--ntt-variant", type=int, default=-1,
                    help="set this NTT pass variant after tuning (counter collection per variant)")
    ap.add_argument("--graph-steps", type=int, default=20,
                    help="also time this many replays of the headline compression captured in a graph (0: skip)")
    ap.add_argument("--plain-db-steps", type=int, default=2,
                    help="also time the unencrypted-database form on the headline query (0: skip)")
    ap.add_argument("--products", type=int, default=1,
                    help="also time ciphertext products, Power_{p-1} and a PDQ Answer with Match (0: skip)")
    ap.add_argument("--small-configs", type=int, default=20,
                    help="latency repetitions of the ring-4096 and ring-2^15 configurations (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the compression path here is built and measured on a single "
              "MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_17063_amd import hc
    st = setup(args.workload)
    ctx, wl = st["ctx"], st["wl"]
    out = ctx.ct_tensor(1)[0]
    stream = torch.cuda.current_stream()
    prep = None
    if args.diagonals == "resident":
        t0 = time.perf_counter()
        held = ctx.diag_prepare(wl.N, wl.ncol, wl.t, args.comp_level)
        prep = {"seconds": round(time.perf_counter() - t0, 3), "bytes": held}
        log("resident diagonals: %.2f GB prepared in %.2fs" % (held / 1e9, prep["seconds"]))
    info = st["info"]
    ol = args.out_level
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune = ctx.autotune(st["gk"], st["db"], st["cts"], wl.N, wl.t, args.comp_level)
        tune["seconds"] = round(time.perf_counter() - t0, 2)
        log("autotune:", tune)
    if args.ntt_variant >= 0:
        ctx.tune_set(ctx.tune_get()[0], args.ntt_variant)
    for _ in range(args.warmup):
        _, info = ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=args.comp_level,
                               out_level=ol)
    torch.cuda.synchronize()
    ctx.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    step_ev = []
    for _ in range(args.steps):
        ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=args.comp_level, out_level=ol)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        step_ev.append(ev)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    lat, prev = [], e0
    for ev in step_ev:
        lat.append(prev.elapsed_time(ev))
        prev = ev
    ms_per_step = gpu_ms / args.steps
    value = args.steps / (gpu_ms / 1000.0)
    log("timed %d steps: %.1f ms/step (events), wall %.2fs" % (args.steps, ms_per_step, wall))
    # the last timed answer, decrypted and decompressed on the host (the client's side)
    import numpy as np
    dec = ctx.decrypt(st["sk"], ctx.output(out, info).cpu().numpy().view(np.uint64))
    recovered = answer_recovers(hc, ctx, dec, wl.N, wl.ncol, info["s"], st["v"], st["dbv"])
    log("timed answer decrypts and decompresses to the query's %d matches: %s" % (wl.t, recovered))
    rl = kernel_rooflines(ctx, hc)
    mac_timing = ctx.timing_read(hc.KT_DIAG_MAC)
    ctx.timing(False)
    for name, tb in measured_traffic(args.workload).items():
        if name in rl:
            rl[name]["traffic"] = tb
    if args.copy_probe_mb:
        ctx.probe_copy(args.copy_probe_mb << 20)
    for name, r in rl.items():
        log("  %-16s %8.1f ms %6d launches  %s %s of peak" % (name, r["ms"], r["launches"], r["bound"],
                                                              r["frac"]))
    dominant = max(rl, key=lambda k: rl[k]["ms"])
    probe = ctx.probe_mul32_rate(50.0) / 1e12
    log("  32-bit multiply-add probe: %.2f T/s (derived peak %.2f T/s)" % (probe, VALU_PEAK_T))

    rec = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "compressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "PDQ compression, ring 2^16, 2^20 records in 16 ciphertexts, t=1024, "
                               "4 value columns, Q=24x55-bit, P=3x60-bit, p=786433",
                   "records": wl.N, "t": wl.t, "ring_degree": ctx.n, "value_columns": wl.ncol,
                   "key_switches_per_step": st["info"]["n_keyswitch"],
                   "ptct_per_step": st["info"]["n_ptct"],
                   "comp_level_primes": info["comp_level"], "answer_primes": info["level"],
                   "answer_bytes": 2 * info["level"] * ctx.n * 8},
    }
    rec["answer_recovers_matches"] = bool(recovered)
    if tune is not None:
        rec["autotune"] = tune
    rec["latency_ms"] = {"p50": round(percentile(lat, 50), 2), "p99": round(percentile(lat, 99), 2),
                         "kind": "plain, one query at a time"}
    if prep is not None:
        rec["config"]["diagonals"] = "resident (query-independent, prepared once before timing)"
        rec["diag_prepare"] = prep
    else:
        rec["config"]["diagonals"] = "encoded on the fly inside every step"
    if args.graph_steps:
        log_mem("before graph")
        rec["graph"] = graph_leg(st, out, args.graph_steps, args.comp_level, ol)
        log("graph replay: %s" % rec["graph"])
    if args.products:
        log_mem("before products")
        rec["products"] = products_leg(st, 5, ol)
        log("products, Power and Match: %s" % rec["products"])
    if args.plain_db_steps:
        log_mem("before plain_db")
        rec["plain_db"] = plain_db_leg(st, out, args.plain_db_steps, args.comp_level, ol)
        log("unencrypted-database form: %s" % rec["plain_db"])
    if args.batch_queries:
        log_mem("before batched")
        rec["batched"] = batched_large(st, args.batch_queries, max(1, args.steps // 2), ol)
        log("batched %d queries: %.1f ms per batch, %.3f compressions/s" % (
            args.batch_queries, rec["batched"]["ms_per_batch"], rec["batched"]["value"]))
    if prep is not None and args.on_the_fly_steps:
        log_mem("before on_the_fly")
        rec["on_the_fly"] = on_the_fly(st, out, args.on_the_fly_steps, args.comp_level, ol)
        log("diagonals on the fly: %.1f ms/step; output equals resident: %s" % (
            rec["on_the_fly"]["ms_per_step"], rec["on_the_fly"]["equals_resident"]))
    if prep is not None and not args.on_the_fly_steps:
        st["ctx"].diag_release()  # the legs below hold their own tables and batch workspaces
    st["ctx"].trim()  # and the headline context's per-call workspace (the batched leg's is the largest)
    torch.cuda.empty_cache()
    if args.small_configs:
        log_mem("before small_configs")
        rec["small_configs"] = [small_config_latency("plain-4096", args.small_configs, 1),
                                small_config_latency("single-32768", args.small_configs, 2)]
        log("smaller configurations:", rec["small_configs"])
    if args.mixed_batch:
        log_mem("before mixed_batch")
        rec["mixed_batch"] = mixed_batch(args.mixed_batch)
        log("mixed batch:", rec["mixed_batch"])
    if args.serve_rates:
        log_mem("before serving")
        rec["serving"] = serving(st, [float(x) for x in args.serve_rates.split(",")], args.serve_requests,
                                 lanes=args.serve_lanes, max_batch=args.serve_max_batch, out_level=ol)
    if "diag_mac" in rl and not args.no_stream_probe:
        # last: the probe holds 27 GB of device memory while it runs
        try:
            sp = mac_stream_ceiling(ctx, mac_timing, info)
        except hc.HcError as e:
            sp = {"skipped": str(e)}
        if sp:
            rl["diag_mac"]["stream_probe"] = sp
            log("  MAC vs a contiguous stream of the same read/write mix: %s" % sp)
    rec["roofline"] = dict(rl[dominant], kernel=dominant)
    rec["rooflines"] = rl
    rec["mul32_probe_T"] = round(probe, 3)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(st["info"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
