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
    return dict(ctx=ctx, sk=sk, gk=gk, db=dbh, cts=cts, v=v, dbv=db, wl=wl, info=info, keys=keys)


# 32-bit integer multiply peak derived from the chip: 256 CUs x 4 SIMDs x 16 lanes
# at 2.4 GHz = 39.3 T lane-operations/s for full-rate VALU work. On gfx950 the
# 32 x 32 -> 64-bit multiply-add (v_mad_u64_u32) issues at full rate: the
# library's register-only probe (hc_probe_mul32_rate) measures ~35.5 T/s.
MUL32_PEAK_T = 256 * 64 * 2.4e9 / 1e12
# One lazy Shoup butterfly multiplies two 64-bit words: the high half of x*w'
# needs 4 32x32 partial products, the low halves of x*w and qhat*q 3 each.
MUL32_PER_BUTTERFLY = 10


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
    for name, t in out.items():
        if name.startswith("ntt"):
            ach = t["ops"] * MUL32_PER_BUTTERFLY / t["sec"] / 1e12
            rl[name] = {"bound": "alu", "achieved": round(ach, 3), "peak": round(MUL32_PEAK_T, 3),
                        "unit": "Tmul32/s", "frac": round(ach / MUL32_PEAK_T, 4), "traffic": None,
                        "avg_launch_us": round(t["ms"] * 1e3 / t["launches"], 2),
                        "launches": t["launches"], "ms": round(t["ms"], 2)}
        else:
            ach = t["bytes"] / t["sec"] / 1e9
            rl[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                        "avg_launch_us": round(t["ms"] * 1e3 / t["launches"], 2),
                        "launches": t["launches"], "ms": round(t["ms"], 2)}
    return rl


def cpu_baseline(info):
    """The CPU oracle on a bounded sample of the same workload: one plain
    rotation (key switch), one diagonal encoding and one plaintext product at
    the full ring size, scaled by the step's operation counts."""
    import numpy as np
    import workloads as W
    from oracle import bfv, compress as C
    from oracle.params import make_params
    r = W.RINGS["ring-65536"]
    pr = make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)
    sk, pk = bfv.keygen(pr, W.seed32("sk", 0))
    k = bfv.rot_row_element(pr, 8)
    gk = bfv.galois_keygen(pr, sk, k, W.seed32("gk", 0))
    ct = bfv.encrypt(pr, pk, np.zeros((2, pr.nh), dtype=np.uint64), W.seed32("enc", 0, 0))
    t0 = time.perf_counter()
    bfv.rotate(pr, ct, gk)
    t_ks = time.perf_counter() - t0
    t0 = time.perf_counter()
    m = bfv.plain_poly(pr, C.diagonal_slots(pr.p, pr.nh, 1024, 8, 3, 5, 2))
    t_enc = time.perf_counter() - t0
    t0 = time.perf_counter()
    bfv.mul_plain(pr, ct, m)
    t_pt = time.perf_counter() - t0
    per_query = info["n_keyswitch"] * t_ks + info["n_diag"] * t_enc + info["n_ptct"] * t_pt
    log("cpu oracle sample: keyswitch %.1fs, diagonal encode %.2fs, ptct %.2fs -> %.0fs per compression"
        % (t_ks, t_enc, t_pt, per_query))
    return {"value": 1.0 / per_query, "unit": "compressions/s", "cores": 1, "kind": "oracle",
            "sample": "oracle (single thread) timed on one plain rotation, one diagonal encoding and "
                      "one plaintext-ciphertext product at ring 2^16 / 24+3 primes "
                      "(%.1f s, %.2f s, %.2f s), scaled by the step's %d key switches, %d diagonal "
                      "encodings and %d plaintext products" % (t_ks, t_enc, t_pt, info["n_keyswitch"],
                                                               info["n_diag"], info["n_ptct"]),
            "extrapolated": True}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large-65536")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--comp-level", type=int, default=0,
                    help="ciphertext primes kept for Comp (0: the library default; 24: no switching)")
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
    for _ in range(args.warmup):
        _, info = ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=args.comp_level)
    torch.cuda.synchronize()
    ctx.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.compress(st["gk"], st["db"], st["cts"], wl.N, wl.t, out=out, comp_level=args.comp_level)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = gpu_ms / args.steps
    value = args.steps / (gpu_ms / 1000.0)
    log("timed %d steps: %.1f ms/step (events), wall %.2fs" % (args.steps, ms_per_step, wall))
    rl = kernel_rooflines(ctx, hc)
    ctx.timing(False)
    for name, r in rl.items():
        log("  %-16s %8.1f ms %6d launches  %s %.3f of peak" % (name, r["ms"], r["launches"], r["bound"],
                                                               r["frac"]))
    dominant = max(rl, key=lambda k: rl[k]["ms"])
    probe = ctx.probe_mul32_rate(50.0) / 1e12
    log("  32-bit multiply-add probe: %.2f T/s (derived peak %.2f T/s)" % (probe, MUL32_PEAK_T))

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
                   "comp_level_primes": info["level"]},
    }
    rec["roofline"] = dict(rl[dominant], kernel=dominant)
    if "keyswitch_inner" in rl:
        rec["roofline_keyswitch"] = dict(rl["keyswitch_inner"], kernel="keyswitch_inner")
    rec["kernels"] = {k: {"ms": v["ms"], "frac": v["frac"], "bound": v["bound"]} for k, v in rl.items()}
    rec["mul32_probe_T"] = round(probe, 3)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(st["info"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
