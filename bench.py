#!/usr/bin/env python3
"""Benchmark of the MI355X Pi_MatMul path; prints one JSON line.

Headline workload (the default): the BERT-large / GPT-2-medium-shaped stack of 24 encoder
layers, each with four private linear products at sequence 512 (QKV 1024x3072, attn-out
1024x1024, FFN 1024x4096 and 4096x1024), RNS-BFV with N = 8192, three 50-bit primes,
t = 2^41, W = floor(N(0, 0.02) * 2^14), client share X uniform over Z_{2^41}, block area
1024.  Synthetic seeded inputs (workloads.py).  Every layer has its own weight cache (pi_A
blocks in NTT form), built at weight-load time outside the timed region and resident at once.

A step is one pass of the whole stack: for each of the 96 products encode (client), encrypt
(client), ciphertext-plaintext product with accumulation, re-randomisation, mask and sparse
reply (server, one fused call), decrypt and decode (client).  value = useful
multiply-accumulates (seq * d_in * d_out summed over the stack) per second of wall time over
the timed passes.  HIP events recorded on the stream at every layer boundary give the pass
and per-layer latencies (p50 / p99).

roofline: the product kernel (k_mac_sk), whose launches are bracketed with HIP events on their
own stream during the timed passes; at this shape (64 column blocks per weight block) it is
bound by the FP64 vector unit, so achieved = slot-wise modular multiply-accumulates per launch
(2 L N P) x 14 (7 FP64 instructions, each counted at the FMA rate the peak assumes) over the
average launch duration, against 78.6 TFLOP/s.

cpu_baseline: the oracle (plain C + Python big integers, OpenMP) on a bounded sample of the
stack (the FFN2 product's first column block), with the host's CPU model.

Extra keys: bert_base_layer (the BERT-base layer at seq 128, N = 4096, two primes, fewest-wire
plan, with the product's HBM roofline) and batched_vs_plain (64 uneven BERT-base products:
one batched pass against one call per product).

Other workloads (each prints one JSON line of its own): --workload layer (the BERT-base layer
alone, with its oracle baseline), stack, batch, serve (a Poisson stream of requests through a
12-layer stack with continuous batching, p50/p99 per arrival rate), peak (the device's
streaming and arithmetic ceilings), pareto (the layer at several block areas: GPU time against
wire bytes) and attention (the cross terms of a BERT-base layer's attention, Pi_MatMul on
uniform shares at N = 8192).
"""
import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ct-pt MatMul int-MAC/s and layer-stack p50/p99 latency, batched vs plain"
HBM_PEAK_GBS = 8000.0
# Operation ids of the autotuners' trial encryptions: far above every step's ids, so that no
# (seed, op_id) pair is used for two different inputs.
AUTOTUNE_OP = 1 << 31


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mac_traffic_bert_base_seq128.md")
MAC_SOURCES = [os.path.join(ROOT, "paper_2305_18396_amd", "csrc", f) for f in ("mac.h", "mac.hip")]


STACK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mac_mfma_traffic_bert_large_seq512.md")
MFMA_SOURCES = [os.path.join(ROOT, "paper_2305_18396_amd", "csrc", f) for f in ("mfma.h", "mfma.hip")]


def measured_traffic(schedules, path=TRAFFIC_FILE, sources=MAC_SOURCES):
    """HBM bytes per product launch from the committed counter summary, or None when the
    product's sources or schedules differ from the ones the counters were taken on."""
    import hashlib

    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in sources)).hexdigest()
    want = ";".join(",".join(str(v) for v in sch) for sch in schedules)
    if fields.get("mac_sources_sha256") != h or fields.get("product_schedules") != want:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(seconds: float):
    import numpy as np

    from oracle import oracle as orc
    from paper_2305_18396_amd import workloads

    wl = workloads.bert_base_layer(128)[0]  # QKV 768x2304
    n, r, m = wl.shape
    pyp = orc.Params(4096, 2, 37, 12)
    plan = orc.plan_comm(4096, n, r, m)
    cseed, sseed = workloads.seed("client", 900), workloads.seed("server", 900)
    s, pk = orc.keygen(pyp, cseed)
    ptA = orc.encode_weights(plan, wl.W)
    t0 = time.perf_counter()
    pt = orc.encode_input(plan, wl.X)
    ct = orc.encrypt(pyp, s, cseed, 0, pt)
    t_enc = time.perf_counter() - t0
    threads = orc.max_threads()
    done, t_out = 0, 0.0
    macs = 0
    while done < plan.O and t_out + t_enc < seconds:
        outs = np.arange(done, min(plan.O, done + threads), dtype=np.uint32)
        t1 = time.perf_counter()
        acc = orc.matmul(pyp, plan, ptA, ct, outs)
        acc = orc.rerandomize(pyp, pk, sseed, 0, acc, outs)
        c1, c0s, sm = orc.mask_extract(pyp, plan, sseed, 0, acc, outs)
        orc.decrypt(pyp, plan, s, c1, c0s, outs)
        t_out += time.perf_counter() - t1
        for y in outs.tolist():
            ib, kb = divmod(y, plan.K)
            rows = min(plan.nb, n - kb * plan.nb)
            cols = min(plan.mb, m - ib * plan.mb)
            macs += rows * cols * r
        done += len(outs)
    elapsed = t_out + t_enc * done / plan.O
    return {"value": macs / elapsed, "unit": "int-MAC/s", "cores": threads, "kind": "oracle",
            "sample": f"QKV 768x2304 product at seq 128 (N=4096, 2 primes): {done} of {plan.O} output "
                      f"ciphertexts through product, re-randomisation, mask and decryption, "
                      f"encryption of all {plan.I} inputs counted pro rata; {elapsed:.1f} s"}


def bench_batch(args):
    """Uneven batch: `count` independent products, lengths uniform in [16, 512], shapes uniform
    over the four BERT-base products, block area d_fix (one weight cache per shape, one client key
    per product).  Times the server's product step (forward NTT, slot-wise products, inverse NTT)
    for every item: one batched pass (autotuned schedule) against one pimm_matmul call per item."""
    import torch

    from paper_2305_18396_amd import pimm, workloads

    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True, device=0)
    wts, items = workloads.batched_uneven(count=args.batch_count)
    caches, rows = {}, []
    useful = wire = slot = 0
    for k, it in enumerate(items):
        r, m, W = wts[it.shape_index]
        plan = pimm.Plan(ctx, it.seq, r, m, d_fix=args.d_fix)
        if (r, m) not in caches:
            caches[(r, m)] = pimm.Weights(plan, pimm.to_device_u64(W))
        cseed = workloads.seed("client", 2000 + k)
        sk, _ = pimm.keygen(ctx, cseed)
        ct = pimm.encrypt(plan, sk, cseed, k, pimm.encode_input(plan, pimm.to_device_u64(it.X)))
        acc = torch.empty((plan.O, 2, 2, 4096), dtype=torch.int64, device="cuda")
        rows.append((plan, caches[(r, m)], ct, acc))
        useful += it.seq * r * m
        wire += plan.info.ct_bytes + plan.info.c1_bytes + plan.info.c0s_bytes
        slot += 2 * 2 * 4096 * plan.info.P
    torch.cuda.synchronize()
    log(f"batch: {len(rows)} items, {useful / 1e9:.2f} G useful MACs, d_fix {args.d_fix}")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # The plain form runs each product with its own autotuned schedule (one tuning per
    # distinct plan shape).
    tuned = {}
    for plan, w, ct, acc in rows:
        key = (plan.r, plan.m, plan.n)
        if key not in tuned:
            plan.autotune(w, ct, acc, reps=1)
            tuned[key] = plan.tuning()
        plan.set_tuning(*tuned[key])
    torch.cuda.synchronize()
    log(f"plain form: {len(tuned)} plan shapes autotuned")

    def plain():
        for plan, w, ct, acc in rows:
            pimm.matmul(plan, w, ct, acc)

    def phases(fn, reps):
        """Kernel-class milliseconds per pass, from the library's HIP events."""
        kinds = ("ntt_fwd", "mac", "ntt_inv", "fused")
        for k in kinds:
            pimm.profile_read(k)
        pimm.profile_enable(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        pimm.profile_enable(False)
        return {k: round(pimm.profile_read(k)[1] / reps, 3) for k in kinds}

    t_plain = timed(plain, args.steps)
    plain_phases = phases(plain, 2)
    ref = [acc.clone() for *_, acc in rows]
    batch = pimm.Batch(rows)
    best_ms = batch.autotune(reps=2)
    t_batch = timed(batch.run, args.steps)
    batch_phases = phases(batch.run, 2)
    batch.status()
    same = all(torch.equal(acc, r) for (*_, acc), r in zip(rows, ref))
    graph_t = None
    ws = batch.workspace()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        batch.run(ws=ws, stream=s)
    graph_t = timed(g.replay, args.steps)
    batch.status(ws=ws)
    sched = dict(zip(("schedule", "mac_rows", "mac_cols", "xcd_map", "grid"), batch.get_schedule()))
    # Roofline of the phased pass's product (k_batch_mac): each weight cache is read once per
    # column tile of its group (the products sharing it line up their column blocks), every
    # input and accumulator word once.
    L, N = 2, 4096
    groups = collections.defaultdict(list)
    for plan, w, ct, acc in rows:
        groups[id(w)].append(plan)
    KB = max(1, sched["mac_cols"])
    mac_bytes = 0
    for plans in groups.values():
        cols = sum(p.K for p in plans)
        mac_bytes += plans[0].Wb * L * N * 8 * (-(-cols // KB))
        mac_bytes += sum((2 * p.I + 2 * p.O) * L * N * 8 for p in plans)
    mac_s = batch_phases["mac"] / 1e3
    achieved = mac_bytes / mac_s / 1e9 if mac_s > 0 else 0.0
    # The persistent single launch on the same tile, and the bytes its per-product units read
    # (each product reads its weight cache itself, once per column tile of its own).
    persistent_ms = None
    persistent_bytes = sum(p.Wb * L * N * 8 * (-(-p.K // KB)) + (2 * p.I + 2 * p.O) * L * N * 8
                           for p, *_ in rows)
    if sched["schedule"] == pimm.PHASED:
        batch.set_schedule(pimm.PERSISTENT, sched["mac_rows"], sched["mac_cols"], sched["xcd_map"], 0)
        persistent_ms = timed(batch.run, args.steps) * 1e3
        batch.status()
        batch.set_schedule(pimm.PHASED, sched["mac_rows"], sched["mac_cols"], sched["xcd_map"],
                           sched["grid"])
    return {"workload": f"{len(rows)} products, seq uniform in [16, 512], BERT-base shapes, "
                        f"N=4096, 2 primes, block area {args.d_fix}",
            "useful_macs": useful, "slot_macs": slot, "wire_bytes": wire,
            "plain_ms": t_plain * 1e3, "batched_ms": t_batch * 1e3,
            "graph_ms": graph_t * 1e3, "autotune_best_ms": best_ms,
            "plain_int_mac_per_s": useful / t_plain, "batched_int_mac_per_s": useful / t_batch,
            "graph_int_mac_per_s": useful / graph_t, "speedup": t_plain / t_batch,
            "schedule": sched, "bitexact_vs_plain": bool(same),
            "plain_schedule_counts": {",".join(map(str, t)): c for t, c in
                                      collections.Counter(tuned.values()).most_common()},
            "plain_kernel_ms": plain_phases, "batched_kernel_ms": batch_phases,
            "persistent_ms": persistent_ms, "persistent_product_alg_bytes": persistent_bytes,
            "roofline": {"kernel": "k_batch_mac (the phased pass's product)", "bound": "hbm",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_pass": mac_bytes,
                         "product_ms_per_pass": batch_phases["mac"]}}


def bench_serve(args):
    """Served stream: Poisson arrivals of requests with prompt length log-uniform in [32, 512],
    each a 12-layer BERT-base-shaped stack of 4 products (block area d_fix), keys and
    ciphertexts resident on the device, admission by an HBM budget.  Sweeps the arrival rate on
    a geometric grid until p99 latency saturates; at every rate the same trace also runs in the
    plain form, one request at a time in arrival order."""
    import numpy as np
    import torch

    from paper_2305_18396_amd import pimm, workloads

    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True, device=0)
    shapes = [(r, m) for _, r, m in workloads.BERT_BASE_SHAPES]
    weights = []
    for layer in range(args.layers):
        for wl in workloads.bert_base_layer(1, seed_=workloads.MASTER_SEED + layer):
            n, r, m = wl.shape
            plan = pimm.Plan(ctx, 1, r, m, d_fix=args.d_fix)
            weights.append(pimm.Weights(plan, pimm.to_device_u64(wl.W)))
    torch.cuda.synchronize()
    budget = int(args.serve_budget_gb * (1 << 30))
    log(f"serve: {args.layers} layers, weight caches built, budget {args.serve_budget_gb} GB")

    def run(rate, count, max_active):
        srv = pimm.Server(ctx, args.layers, shapes, weights, args.d_fix, budget, max_active,
                          schedule=pimm.PHASED, mac_rows=args.serve_tile[0],
                          mac_cols=args.serve_tile[1], min_batch=args.serve_min_batch)
        trace = workloads.poisson_trace(rate, count)
        reqs = [(q.rid, q.seq, q.arrival_s, workloads.seed("client", 7000 + q.rid),
                 workloads.seed("server", 7000 + q.rid)) for q in trace]
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        lat = np.array([r["done_s"] - r["arrival_s"] for r in res]) * 1e3
        macs = sum(r["useful_macs"] for r in res)
        srv.close()
        return {"rate_per_s": rate, "requests": count, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "int_mac_per_s": macs / wall,
                "wall_s": wall, "max_active": max_active}

    def both(rate):
        """Continuous batching and the plain form (one request at a time, in arrival order) on
        the same trace."""
        cb = run(rate, args.serve_requests, args.serve_max_active)
        plain = run(rate, args.serve_requests, 1)
        log(f"serve rate {rate:.2f}/s: batched p50/p99 {cb['p50_ms']:.1f}/{cb['p99_ms']:.1f} ms "
            f"{cb['int_mac_per_s'] / 1e9:.1f} G MAC/s; plain p50/p99 {plain['p50_ms']:.1f}/"
            f"{plain['p99_ms']:.1f} ms {plain['int_mac_per_s'] / 1e9:.1f} G MAC/s")
        return {"rate_per_s": rate, "batched": cb, "plain": plain}

    sweep = []
    workload = (f"Poisson stream, prompt length log-uniform in [32, 512], {args.layers}-layer "
                f"BERT-base linear stack, N=4096, 2 primes, block area {args.d_fix}")
    if args.serve_rates:
        # Explicit rates only (no saturation search).
        for rate in args.serve_rates:
            sweep.append(both(rate))
        return {"product_tile": list(args.serve_tile), "min_batch": args.serve_min_batch,
                "workload": workload, "sweep": sweep}
    rate = args.serve_rate0
    while True:
        r = both(rate)
        sweep.append(r)
        if len(sweep) >= 2 and (r["batched"]["p99_ms"] > 4 * sweep[0]["batched"]["p99_ms"]
                                or len(sweep) >= 6):
            break
        rate *= 2
    return {"product_tile": list(args.serve_tile), "min_batch": args.serve_min_batch,
            "workload": workload, "sweep": sweep}


FP64_ISSUE_PER_S = 39.3e12  # FP64 VALU instruction issues per second (78.6 TFLOP/s counts an FMA as 2)
FP64_ISSUES_PER_SLOT_MAC = 7  # mul, fma, mul, rint, fma, add of the modular product + the accumulation


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_stack(seconds: float):
    """The oracle on a bounded sample of the BERT-large stack: column blocks of the FFN2
    4096x1024 product (block plan (16, 64, 8), N = 8192, three primes; a column block is 8
    sequence rows: 64 input and 64 output ciphertexts), one after another until about `seconds`
    have passed, each through encryption of its inputs, product, re-randomisation, mask and
    decryption of its outputs (output ciphertexts in chunks of the thread count; the last block
    may stop part-way, its encryption then counted pro rata)."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2305_18396_amd import workloads

    wl = workloads.bert_large_layer(512)[3]  # FFN2 4096x1024
    n, r, m = wl.shape
    pyp = orc.Params(8192, 3, 41, 14)
    full = orc.plan_fix(8192, 1024, n, r, m)
    plan = orc.Plan(full.nb, r, m, full.mb, full.rb, full.nb, 8192)  # one column block (K = 1)
    cseed, sseed = workloads.seed("client", 901), workloads.seed("server", 901)
    s, pk = orc.keygen(pyp, cseed)
    ptA = orc.encode_weights(plan, wl.W)
    threads = orc.max_threads()
    elapsed, macs, blocks, outs_done = 0.0, 0, 0, 0
    for kb in range(full.K):
        if elapsed >= seconds:
            break
        X = wl.X[kb * full.nb:(kb + 1) * full.nb]
        t0 = time.perf_counter()
        ct = orc.encrypt(pyp, s, cseed, kb, orc.encode_input(plan, X))
        t_enc = time.perf_counter() - t0
        done, t_out = 0, 0.0
        while done < plan.O and elapsed + t_out + t_enc * done / plan.O < seconds:
            outs = np.arange(done, min(plan.O, done + threads), dtype=np.uint32)
            t1 = time.perf_counter()
            acc = orc.matmul(pyp, plan, ptA, ct, outs)
            acc = orc.rerandomize(pyp, pk, sseed, kb, acc, outs)
            c1, c0s, sm = orc.mask_extract(pyp, plan, sseed, kb, acc, outs)
            orc.decrypt(pyp, plan, s, c1, c0s, outs)
            t_out += time.perf_counter() - t1
            for y in outs.tolist():
                macs += plan.nb * min(plan.mb, m - y * plan.mb) * r
            done += len(outs)
        elapsed += t_out + t_enc * done / plan.O
        blocks += 1
        outs_done += done
    return {"value": macs / elapsed, "unit": "int-MAC/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"BERT-large FFN2 4096x1024 product (N=8192, 3 primes, block plan "
                      f"({full.mb},{full.rb},{full.nb})): {outs_done} output ciphertexts of "
                      f"{blocks} column block(s) (of {full.K}) through encryption of their inputs, "
                      f"product, re-randomisation, mask and decryption; {elapsed:.1f} s"}


def bench_stack(args):
    """BERT-large / GPT-2-medium-shaped stack: `--stack-layers` encoder layers (24 by default) of
    four products each at seq 512 (QKV 1024x3072, attn-out 1024x1024, FFN 1024x4096 and
    4096x1024), N = 8192, three 50-bit primes, t = 2^41, 14 fractional bits, block area 1024.
    Every layer has its own weights and weight cache (all resident at once); a step is one pass
    of the whole stack, each product through encode, encrypt, fused server step and decrypt.
    HIP events on the stream at every layer boundary give the pass and layer latencies; the
    product launches are bracketed for the roofline."""
    import numpy as np
    import torch

    from paper_2305_18396_amd import pimm, workloads

    N, L, ell, f, D = 8192, 3, 41, 14, 1024
    ctx = pimm.Context(N, L, ell, f, rerandomize=True, device=0)
    dev = torch.device("cuda", 0)
    cseed, sseed = workloads.seed("client", 11), workloads.seed("server", 11)
    sk, pk = pimm.keygen(ctx, cseed)
    shapes = workloads.BERT_LARGE_SHAPES
    seq = 512
    plans, bufs = [], []
    for name, r, m in shapes:
        plan = pimm.Plan(ctx, seq, r, m, d_fix=D)
        fi = plan.info
        plans.append(plan)
        bufs.append(dict(
            pt=torch.empty((fi.I, N), dtype=torch.int64, device=dev),
            ct=torch.empty((fi.I, 2, L, N), dtype=torch.int64, device=dev),
            c1=torch.empty((fi.O, L, N), dtype=torch.int64, device=dev),
            c0s=torch.empty((fi.O, L, fi.mb * fi.nb), dtype=torch.int64, device=dev),
            c1s=torch.empty((fi.O, L - 1, N), dtype=torch.int64, device=dev),
            c0ss=torch.empty((fi.O, L - 1, fi.mb * fi.nb), dtype=torch.int64, device=dev),
            y0=torch.empty((seq, m), dtype=torch.int64, device=dev),
            y1=torch.empty((seq, m), dtype=torch.int64, device=dev)))
    switched = args.reply == "switched"
    layers = []
    cache = 0
    t_setup = time.perf_counter()
    for k in range(args.stack_layers):
        ops = workloads.bert_large_layer(seq, layer_index=k)
        row = []
        for i, wl in enumerate(ops):
            w = pimm.Weights(plans[i], pimm.to_device_u64(wl.W))
            row.append((w, pimm.to_device_u64(wl.X)))
            cache += plans[i].info.weights_bytes
        layers.append(row)
    torch.cuda.synchronize()
    log(f"stack: {args.stack_layers} layers, weight caches {cache / 1e9:.1f} GB "
        f"({time.perf_counter() - t_setup:.1f} s)")
    useful_layer = sum(seq * r * m for _, r, m in shapes)
    useful = args.stack_layers * useful_layer
    slot_per_product = [2 * L * N * p.info.P for p in plans]
    slot = args.stack_layers * sum(slot_per_product)
    # One schedule per product shape, tuned on layer 0's buffers (or given by --schedules).
    for i, plan in enumerate(plans):
        if args.schedules:
            plan.set_tuning(*(int(v) for v in args.schedules.split(";")[i].split(",")))
            continue
        b = bufs[i]
        pimm.encrypt(plan, sk, cseed, AUTOTUNE_OP + i,
                     pimm.encode_input(plan, layers[0][i][1], b["pt"]), b["ct"])
        acc = torch.empty((plan.O, 2, L, N), dtype=torch.int64, device=dev)
        best = plan.autotune(layers[0][i][0], b["ct"], acc, reps=1)
        log(f"  {shapes[i][0]}: plan ({plan.mb},{plan.rb},{plan.nb}) K={plan.K} "
            f"schedule {plan.tuning()} {best:.2f} ms")
        del acc
    torch.cuda.empty_cache()

    def product(t, k, i):
        w, X = layers[k][i]
        plan, b = plans[i], bufs[i]
        op = (t * args.stack_layers + k) * 4 + i
        pimm.encrypt_input(plan, sk, cseed, op, X, b["ct"])  # Alg. 1 steps 1 and 2 in one pass
        pimm.matmul_share(plan, w, pk, sseed, op, b["ct"], b["c1"], b["c0s"], b["y1"])
        if switched:
            # The reply crosses the wire with its last prime dropped.
            pimm.mod_switch(plan, w, b["c1"], b["c0s"], b["c1s"], b["c0ss"])
            pimm.decrypt_switched(plan, sk, b["c1s"], b["c0ss"], b["y0"])
        else:
            pimm.decrypt(plan, sk, b["c1"], b["c0s"], b["y0"])

    def step(t, marks=None):
        for k in range(args.stack_layers):
            for i in range(len(plans)):
                product(t, k, i)
            if marks is not None:
                marks.append(torch.cuda.Event(enable_timing=True))
                marks[-1].record()

    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    pimm.profile_read("mac")
    pimm.profile_select(["mac"])
    pimm.profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for t in range(args.steps):
        step(args.warmup + t, marks)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    pimm.profile_enable(False)
    pimm.profile_select(None)
    cnt, mac_ms = pimm.profile_read("mac")
    # Latencies from the layer-boundary events (device time, no host synchronisation).
    ends = [start.elapsed_time(e) for e in marks]
    layer_ms = np.diff([0.0] + ends)
    pass_ms = np.diff([0.0] + ends[args.stack_layers - 1::args.stack_layers])
    log(f"stack: {el * 1e3:.1f} ms per pass, {useful / el / 1e9:.1f}e9 int-MAC/s")

    # Per-class breakdown from one untimed pass with every class recorded.
    classes = ("mac", "ntt_fwd", "ntt_inv", "sample", "encode", "decode", "mask_extract",
               "mod_switch")
    for kname in classes:
        pimm.profile_read(kname)
    pimm.profile_enable(True)
    step(10_000)
    torch.cuda.synchronize()
    pimm.profile_enable(False)
    breakdown = {}
    for kname in classes:
        c_, ms_ = pimm.profile_read(kname)
        breakdown[kname] = {"launches_per_pass": c_, "ms_per_pass": round(ms_, 3)}

    mac_avg_s = mac_ms / 1e3 / max(1, cnt)
    slot_per_launch = sum(slot_per_product) / len(plans)
    slot_rate = slot_per_launch / mac_avg_s if cnt else 0.0
    schedules = [p.tuning() for p in plans]
    if all(sch == (0, 0, 0) for sch in schedules):
        # Matrix-core product: the algorithmic bytes are the query ciphertexts (both components,
        # read in place in evaluation form, 8 bytes a residue), the digit form of the weight fragments (7 bytes a residue, padded to 16 rows x 64 inner
        # blocks) and the accumulators (FP64), each once; the int8 work is 49 digit-pair
        # products of 2 x 16 x 16 x 64 operations per tile, slot and prime.
        byts, ops = [], []
        for p in plans:
            fi = p.info
            mt = (fi.M + 15) // 16
            byts.append(16 * L * N * (fi.I + fi.O) + 7 * L * N * mt * 1024)
            ops.append(L * N * mt * ((2 * fi.K + 15) // 16) * 49 * 2 * 16 * 16 * 64)
        bytes_per_launch, ops_per_launch = sum(byts) / len(byts), sum(ops) / len(ops)
        achieved = bytes_per_launch / mac_avg_s / 1e9 if cnt else 0.0
        roofline = {
            "kernel": "k_mac_mfma (the slot-wise product on the matrix cores)", "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(schedules, STACK_TRAFFIC_FILE, MFMA_SOURCES),
            "alg_bytes_per_launch": bytes_per_launch, "avg_launch_ms": mac_avg_s * 1e3,
            "int8_ops_per_launch": ops_per_launch,
            "int8_TOPS": ops_per_launch / mac_avg_s / 1e12 if cnt else 0.0,
            "int8_peak_TOPS": 5000.0,
            "note": "HBM is the binding roofline: the launch's bytes at 8 TB/s take longer than "
                    "its int8 operations at 5.0 POP/s",
        }
    else:
        flop_per_slot = 2 * FP64_ISSUES_PER_SLOT_MAC
        achieved_tf = slot_rate * flop_per_slot / 1e12
        roofline = {
            "kernel": "k_mac_sk (the slot-wise product)", "bound": "alu",
            "achieved": achieved_tf, "peak": 78.6, "unit": "TFLOP/s",
            "frac": achieved_tf / 78.6, "traffic": None,
            "work_per_launch_slot_macs": slot_per_launch,
            "flop_per_slot_mac": flop_per_slot,
            "avg_launch_ms": mac_avg_s * 1e3,
            "note": "FP64 vector issue rate: each slot-wise modular multiply-accumulate is 7 FP64 "
                    "instructions (counted at the FMA rate of the 78.6 TFLOP/s peak, i.e. 2 each); "
                    "peak = 5.61e12 slot-MAC/s",
        }
    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    return {
        "workload": f"BERT-large-shaped stack, {args.stack_layers} layers x 4 products at seq "
                    f"{seq} (QKV 1024x3072, attn-out 1024x1024, FFN 1024x4096 and 4096x1024); "
                    f"RNS-BFV N={N}, {L}x50-bit primes, t=2^{ell}, {f} fractional bits, block "
                    f"area {D}; weight caches resident",
        "plans": [[p.mb, p.rb, p.nb] for p in plans],
        "product_schedules": [list(p.tuning()) for p in plans],
        "weight_cache_bytes": cache, "useful_macs_per_step": useful,
        "s_per_step": el, "ms_per_layer": el * 1e3 / args.stack_layers,
        "int_mac_per_s": useful / el, "slot_mac_per_s": slot / el,
        "stack_latency_ms": {"p50": float(np.percentile(pass_ms, 50)),
                             "p99": float(np.percentile(pass_ms, 99)),
                             "samples": int(len(pass_ms))},
        "layer_latency_ms": {"p50": float(np.percentile(layer_ms, 50)),
                             "p99": float(np.percentile(layer_ms, 99)),
                             "samples": int(len(layer_ms))},
        "product_ms_per_step": mac_ms / args.steps,
        "product_slot_mac_per_s": slot_rate,
        "reply": ("switched: the last prime dropped before the reply is sent, decrypted with "
                  f"{L - 1} primes" if switched else f"full: {L} primes"),
        "wire_bytes_per_step": {
            "upload": args.stack_layers * sum(p.info.ct_bytes for p in plans),
            "reply_full": args.stack_layers * sum(p.info.c1_bytes + p.info.c0s_bytes for p in plans),
            "reply_switched": args.stack_layers * sum(p.info.c1_bytes + p.info.c0s_bytes
                                                      for p in plans) * (L - 1) // L},
        "kernels_untimed_pass": breakdown,
        "roofline": roofline,
    }


def bench_pareto(args):
    """Protocol-level plan selection: the BERT-base layer at each block area D (0 = the
    fewest-wire plan), the GPU time of a whole step and of the server's part against the bytes
    on the wire; the points no other point beats on both, and the D that minimises the step
    time plus the wire time over links of a few speeds."""
    import torch

    from paper_2305_18396_amd import pimm, workloads

    dev = torch.device("cuda", 0)
    N, L, ell, f = 4096, 2, 37, 12
    ctx = pimm.Context(N, L, ell, f, rerandomize=True, device=0)
    ops = workloads.bert_base_layer(args.seq)
    cseed, sseed = workloads.seed("client", 1), workloads.seed("server", 1)
    sk, pk = pimm.keygen(ctx, cseed)
    points = []
    for D in args.pareto_d:
        state, wire = [], 0
        for i, wl in enumerate(ops):
            n, r, m = wl.shape
            plan = pimm.Plan(ctx, n, r, m, d_fix=D)
            w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
            fi = plan.info
            X = pimm.to_device_u64(wl.X)
            ct = pimm.encrypt(plan, sk, cseed, i, pimm.encode_input(plan, X))
            acc = torch.empty((fi.O, 2, L, N), dtype=torch.int64, device=dev)
            plan.autotune(w, ct, acc, reps=2)
            del acc
            state.append(dict(plan=plan, w=w, X=X, ct=ct, op=i, ws=plan.workspace(),
                              pt=torch.empty((fi.I, N), dtype=torch.int64, device=dev),
                              c1=torch.empty((fi.O, L, N), dtype=torch.int64, device=dev),
                              c0s=torch.empty((fi.O, L, fi.mb * fi.nb), dtype=torch.int64,
                                              device=dev),
                              y0=torch.empty((n, m), dtype=torch.int64, device=dev),
                              y1=torch.empty((n, m), dtype=torch.int64, device=dev)))
            wire += fi.ct_bytes + fi.c1_bytes + fi.c0s_bytes

        def step(k, server_only=False):
            for st in state:
                p, op = st["plan"], k * 8 + st["op"]
                if not server_only:
                    pimm.encode_input(p, st["X"], st["pt"])
                    pimm.encrypt(p, sk, cseed, op, st["pt"], st["ct"], st["ws"])
                pimm.matmul_share(p, st["w"], pk, sseed, op, st["ct"], st["c1"], st["c0s"],
                                  st["y1"], st["ws"])
                if not server_only:
                    pimm.decrypt(p, sk, st["c1"], st["c0s"], st["y0"], st["ws"])

        times = {}
        for mode in (False, True):
            for k in range(args.warmup):
                step(k, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                step(args.warmup + k, mode)
            torch.cuda.synchronize()
            times[mode] = (time.perf_counter() - t0) / args.steps
        pt = {"d": D or "fewest-wire", "plans": [[s["plan"].mb, s["plan"].rb, s["plan"].nb] for s in state],
              "step_ms": times[False] * 1e3, "server_ms": times[True] * 1e3, "wire_bytes": wire,
              "weight_cache_bytes": sum(s["plan"].info.weights_bytes for s in state)}
        log(f"D={pt['d']}: step {pt['step_ms']:.2f} ms, server {pt['server_ms']:.2f} ms, "
            f"wire {wire / 1e6:.0f} MB")
        points.append(pt)
        del state
        torch.cuda.empty_cache()
    for a in points:
        a["pareto"] = not any(b is not a and b["server_ms"] <= a["server_ms"] and
                              b["wire_bytes"] <= a["wire_bytes"] and
                              (b["server_ms"] < a["server_ms"] or b["wire_bytes"] < a["wire_bytes"])
                              for b in points)
    # Link speed above which each point of the front beats the next one with fewer bytes.
    front = sorted((q for q in points if q["pareto"]), key=lambda q: q["wire_bytes"])
    for lo, hi in zip(front, front[1:]):
        dt = lo["step_ms"] - hi["step_ms"]
        hi["beats_previous_above_Gbit_per_s"] = (
            (hi["wire_bytes"] - lo["wire_bytes"]) * 8 / (dt * 1e-3) / 1e9 if dt > 0 else None)
    choice = {}
    for gbps in (1, 10, 100, 400, 1600):
        best = min(points, key=lambda q: q["step_ms"] + q["wire_bytes"] * 8 / (gbps * 1e9) * 1e3)
        choice[f"{gbps}_Gbit_per_s"] = {"d": best["d"], "total_ms": best["step_ms"] +
                                        best["wire_bytes"] * 8 / (gbps * 1e9) * 1e3}
    return {"workload": f"BERT-base-shaped layer, seq {args.seq}, N=4096, 2 primes; block area "
                        "swept", "points": points, "choice_by_link": choice}


def bench_select(args):
    """Protocol-level plan selection as the library does it (pimm_plan_select): for each product
    of the BERT-base layer at seq --seq and each link speed of --link-gbps, the block area among
    --pareto-d (0 = the fewest-wire plan) that minimises the measured server step plus the time
    the upload and the reply take on the link."""
    import torch

    from paper_2305_18396_amd import pimm, workloads

    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True, device=0)
    ops = workloads.bert_base_layer(args.seq)
    out = {"workload": f"BERT-base-shaped layer, seq {args.seq}, N=4096, 2 primes; block area "
                       "chosen per product and link speed by pimm_plan_select",
           "candidates": args.pareto_d, "links": {}}
    for gbps in args.link_gbps:
        row = {"choice": [], "server_ms": [], "wire_bytes": [], "total_ms": 0.0}
        for wl in ops:
            n, r, m = wl.shape
            best, ms, wire = pimm.plan_select(ctx, n, r, m, pimm.to_device_u64(wl.W), gbps * 1e9,
                                              args.pareto_d, reps=2)
            i = args.pareto_d.index(best)
            row["choice"].append(best)
            row["server_ms"].append(ms)
            row["wire_bytes"].append(wire)
            row["total_ms"] += ms[i] + wire[i] * 8 / (gbps * 1e9) * 1e3
        log(f"select at {gbps} Gbit/s: block areas {row['choice']} "
            f"(step + wire {row['total_ms']:.2f} ms)")
        out["links"][f"{gbps:g}_Gbit_per_s"] = row
        torch.cuda.empty_cache()
    return out


def bench_attention(args):
    """Attention cross terms of one BERT-base layer at seq `--seq` (Eq. 2): per head (12, head
    dimension 64) the score terms Q0 K1^T and K0 Q1^T (seq x 64 x seq) and the value terms A0 V1
    (seq x seq x 64) and V0^T A1^T (64 x seq x seq), each a Pi_MatMul whose plaintext operand is
    the server's uniform share, at N = 8192 with three primes and t = 2^41.  A step runs all 48
    products: the client's encode and encrypt, the server's re-encoding of its share into the
    weight cache (no allocation, no synchronisation), the fused server step, the decryption."""
    import numpy as np
    import torch

    from paper_2305_18396_amd import pimm, workloads

    dev = torch.device("cuda", 0)
    N, L, ell, f, heads, d = 8192, 3, 41, 14, 12, 64
    n = args.seq
    ctx = pimm.Context(N, L, ell, f, rerandomize=True, device=0)
    cseed, sseed = workloads.seed("client", 5), workloads.seed("server", 5)
    sk, pk = pimm.keygen(ctx, cseed)
    rng = np.random.default_rng(20230529)
    half = 1 << (ell - 1)
    shapes = [(n, d, n), (n, d, n), (n, n, d), (d, n, n)]
    state, useful, wire = [], 0, 0
    for h in range(heads):
        for t, (a, r, m) in enumerate(shapes):
            plan = pimm.Plan(ctx, a, r, m)
            fi = plan.info
            X = pimm.to_device_u64(rng.integers(0, 1 << ell, (a, r), dtype=np.uint64))
            W = torch.from_numpy(rng.integers(-half, half, (r, m), dtype=np.int64)).to(dev)
            w = pimm.Weights(plan, W)
            state.append(dict(plan=plan, w=w, X=X, W=W, op=h * 4 + t, ws=plan.workspace(),
                              pt=torch.empty((fi.I, N), dtype=torch.int64, device=dev),
                              ct=torch.empty((fi.I, 2, L, N), dtype=torch.int64, device=dev),
                              c1=torch.empty((fi.O, L, N), dtype=torch.int64, device=dev),
                              c0s=torch.empty((fi.O, L, fi.mb * fi.nb), dtype=torch.int64,
                                              device=dev),
                              y0=torch.empty((a, m), dtype=torch.int64, device=dev),
                              y1=torch.empty((a, m), dtype=torch.int64, device=dev)))
            useful += a * r * m
            wire += fi.ct_bytes + fi.c1_bytes + fi.c0s_bytes
    for st in state[:4]:
        # Operation ids from 2^31 up are kept for the autotuner's encryptions, apart from
        # the steps' ids, so that no (seed, op_id) pair serves two different inputs.
        ct0 = pimm.encrypt(st["plan"], sk, cseed, AUTOTUNE_OP + st["op"],
                           pimm.encode_input(st["plan"], st["X"]))
        acc0 = torch.empty((st["plan"].info.O, 2, L, N), dtype=torch.int64, device=dev)
        st["plan"].autotune(st["w"], ct0, acc0, reps=2)
        del ct0, acc0
    for st in state[4:]:
        st["plan"].set_tuning(*state[st["op"] % 4]["plan"].tuning())

    def step(k):
        for st in state:
            p, op = st["plan"], k * 64 + st["op"]
            pimm.encode_input(p, st["X"], st["pt"])
            pimm.encrypt(p, sk, cseed, op, st["pt"], st["ct"], st["ws"])
            st["w"].update(st["W"], half)
            pimm.matmul_share(p, st["w"], pk, sseed, op, st["ct"], st["c1"], st["c0s"], st["y1"],
                              st["ws"])
            pimm.decrypt(p, sk, st["c1"], st["c0s"], st["y0"], st["ws"])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    log(f"attention cross terms: {sec * 1e3:.2f} ms per layer, {useful / sec / 1e9:.1f}e9 int-MAC/s")

    # The products of each phase are independent (the 24 score terms, then after the softmax
    # the 24 value terms): run each phase over --att-streams streams, joined before the next phase.
    streams = [torch.cuda.Stream() for _ in range(args.att_streams)]

    def step_streams(k):
        main = torch.cuda.current_stream()
        for phase in (0, 1):
            for q in streams:
                q.wait_stream(main)
            for st in state:
                if (st["op"] % 4 >= 2) != bool(phase):
                    continue
                q = streams[(st["op"] // 4 + st["op"]) % len(streams)]
                p, op = st["plan"], k * 64 + st["op"]
                pimm.encode_input(p, st["X"], st["pt"], stream=q)
                pimm.encrypt(p, sk, cseed, op, st["pt"], st["ct"], st["ws"], stream=q)
                st["w"].update(st["W"], half, stream=q)
                pimm.matmul_share(p, st["w"], pk, sseed, op, st["ct"], st["c1"], st["c0s"],
                                  st["y1"], st["ws"], stream=q)
                pimm.decrypt(p, sk, st["c1"], st["c0s"], st["y0"], st["ws"], stream=q)
            for q in streams:
                main.wait_stream(q)

    step_streams(800)
    torch.cuda.synchronize()
    ref_s = [(st["y0"].clone(), st["y1"].clone()) for st in state]
    step(800)
    torch.cuda.synchronize()
    streams_same = all(torch.equal(st["y0"], a) and torch.equal(st["y1"], b)
                       for st, (a, b) in zip(state, ref_s))
    t0 = time.perf_counter()
    for k in range(args.steps):
        step_streams(args.warmup + k)
    torch.cuda.synchronize()
    ssec = (time.perf_counter() - t0) / args.steps
    log(f"  over {len(streams)} streams per phase: {ssec * 1e3:.2f} ms per layer "
        f"(same shares: {streams_same})")

    # The same step captured once into a HIP graph (the calls allocate nothing and record no
    # memset) and replayed; every replay is checked against the eager step with the same ids.
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step(900)
    torch.cuda.synchronize()
    ref = [(st["y0"].clone(), st["y1"].clone()) for st in state]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        step(900)
    same = True
    for _ in range(3):
        for st in state:
            st["y0"].zero_()
            st["y1"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same = same and all(torch.equal(st["y0"], a) and torch.equal(st["y1"], b)
                            for st, (a, b) in zip(state, ref))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    gsec = (time.perf_counter() - t0) / args.steps
    log(f"  as a HIP graph: {gsec * 1e3:.2f} ms per layer (replays bit-exact: {same})")

    # Grouped: the products of one shape in a phase as one grouped plan (the 24 score terms;
    # the 12 A0 V1 and the 12 V0^T A1^T terms), every call doing all of them in one set of
    # launches.  Operation ids from 2^30 up keep its randomness apart from the steps above.
    terms = [[0, 1], [2], [3]]
    gstate = []
    for gi, ts in enumerate(terms):
        members = [st for st in state if st["op"] % 4 in ts]
        a, r, m = shapes[ts[0]]
        G = len(members)
        plan = pimm.Plan(ctx, a, r, m, groups=G)
        fi = plan.info
        Xg = torch.stack([st["X"] for st in members]).contiguous()
        Wg = torch.stack([st["W"] for st in members]).contiguous()
        w = pimm.Weights(plan, Wg)
        g = dict(plan=plan, w=w, X=Xg, W=Wg, members=members, ws=plan.workspace(),
                 pt=torch.empty((fi.I, N), dtype=torch.int64, device=dev),
                 ct=torch.empty((fi.I, 2, L, N), dtype=torch.int64, device=dev),
                 c1=torch.empty((fi.O, L, N), dtype=torch.int64, device=dev),
                 c0s=torch.empty((fi.O, L, fi.mb * fi.nb), dtype=torch.int64, device=dev),
                 y0=torch.empty((G, a, m), dtype=torch.int64, device=dev),
                 y1=torch.empty((G, a, m), dtype=torch.int64, device=dev))
        pimm.encrypt(plan, sk, cseed, AUTOTUNE_OP + 100 + gi, pimm.encode_input(plan, Xg, g["pt"]), g["ct"])
        acc0 = torch.empty((fi.O, 2, L, N), dtype=torch.int64, device=dev)
        plan.autotune(w, g["ct"], acc0, reps=2)
        del acc0
        gstate.append(g)

    def gstep(k):
        for gi, g in enumerate(gstate):
            p, op = g["plan"], (1 << 30) + k * 8 + gi
            pimm.encode_input(p, g["X"], g["pt"])
            pimm.encrypt(p, sk, cseed, op, g["pt"], g["ct"], g["ws"])
            g["w"].update(g["W"], half)
            pimm.matmul_share(p, g["w"], pk, sseed, op, g["ct"], g["c1"], g["c0s"], g["y1"], g["ws"])
            pimm.decrypt(p, sk, g["c1"], g["c0s"], g["y0"], g["ws"])

    # The grouped shares add up to the same products as the per-product shares of step 800.
    step(800)
    gstep(800)
    torch.cuda.synchronize()
    mask = (1 << ell) - 1
    grouped_same = all(
        torch.equal((g["y0"][i] + g["y1"][i]) & mask, (st["y0"] + st["y1"]) & mask)
        for g in gstate for i, st in enumerate(g["members"]))
    for k in range(args.warmup):
        gstep(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        gstep(args.warmup + k)
    torch.cuda.synchronize()
    grsec = (time.perf_counter() - t0) / args.steps
    log(f"  grouped (3 plans of 24, 12, 12 products): {grsec * 1e3:.2f} ms per layer, "
        f"{useful / grsec / 1e9:.1f}e9 int-MAC/s (same products: {grouped_same})")
    return {"workload": f"BERT-base attention cross terms, seq {n}: 12 heads x (2 x {n}x64x{n} "
                        f"+ {n}x{n}x64 + 64x{n}x{n}), plaintext operand a uniform share; "
                        "RNS-BFV N=8192, 3x50-bit primes, t=2^41",
            "plans": [[s["plan"].mb, s["plan"].rb, s["plan"].nb] for s in state[:4]],
            "product_schedules": [list(s["plan"].tuning()) for s in state[:4]],
            "ms_per_layer": sec * 1e3, "useful_macs_per_layer": useful,
            "int_mac_per_s": useful / sec, "wire_bytes_per_layer": wire,
            "graph_ms_per_layer": gsec * 1e3, "graph_int_mac_per_s": useful / gsec,
            "graph_replays_bitexact": bool(same),
            "streams": len(streams), "streams_ms_per_layer": ssec * 1e3,
            "streams_int_mac_per_s": useful / ssec, "streams_same_shares": bool(streams_same),
            "grouped_ms_per_layer": grsec * 1e3, "grouped_int_mac_per_s": useful / grsec,
            "grouped_plans": [[g["plan"].groups, g["plan"].mb, g["plan"].rb, g["plan"].nb]
                              for g in gstate],
            "grouped_product_schedules": [list(g["plan"].tuning()) for g in gstate],
            "grouped_same_products": bool(grouped_same)}


def bench_peak(args):
    """Sustained device rates next to the published peaks: the HBM read and copy
    bandwidth of plain streaming kernels (and of torch's own sum and copy), the FP64
    fma rate, and the modular-product rates of the FP64 form the library uses and of
    the 64-bit integer Barrett and Shoup forms."""
    import torch

    from paper_2305_18396_amd import pimm

    out = {"spec_hbm_GBps": HBM_PEAK_GBS, "spec_fp64_TFLOPs": 78.6}
    gib = 1 << 30
    out["read_GBps"] = pimm.probe(pimm.PROBE_READ, 8 * gib, args.steps) / 1e9
    out["read8_GBps"] = pimm.probe(pimm.PROBE_READ8, 8 * gib, args.steps) / 1e9
    out["copy_GBps"] = pimm.probe(pimm.PROBE_COPY, 4 * gib, args.steps) / 1e9
    out["fma64_TFLOPs"] = pimm.probe(pimm.PROBE_FMA64, 4096, args.steps) / 1e12
    out["modmul_f64_G_per_s"] = pimm.probe(pimm.PROBE_MODMUL_F64, 4096, args.steps) / 1e9
    out["modmul_barrett_u64_G_per_s"] = pimm.probe(pimm.PROBE_MODMUL_BARRETT, 1024, args.steps) / 1e9
    out["modmul_shoup_u64_G_per_s"] = pimm.probe(pimm.PROBE_MODMUL_SHOUP, 1024, args.steps) / 1e9
    x = torch.ones((8 * gib) // 8, dtype=torch.float64, device="cuda")
    x.sum()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.sum()
    torch.cuda.synchronize()
    out["torch_sum_GBps"] = 8 * gib / ((time.perf_counter() - t0) / args.steps) / 1e9
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    out["torch_copy_GBps"] = 2 * 8 * gib / ((time.perf_counter() - t0) / args.steps) / 1e9
    return out


def bench_layer(args):
    """BERT-base-shaped layer (the four products at sequence --seq, N = 4096, two primes,
    t = 2^37), the whole protocol per step; the product's HBM roofline, the server path alone,
    the FC completion, the seed-compressed upload's expansion, latency and graph replay."""
    import numpy as np
    import torch

    from paper_2305_18396_amd import pimm, workloads

    dev = torch.device("cuda", 0)
    N, L, ell, f = 4096, 2, 37, 12
    ctx = pimm.Context(N, L, ell, f, rerandomize=True, device=0)
    ops = workloads.bert_base_layer(args.seq)
    cseed, sseed = workloads.seed("client", 1), workloads.seed("server", 1)
    sk, pk = pimm.keygen(ctx, cseed)
    state = []
    useful = mac_bytes = slot_macs = butterflies = wire = wire_seeded = wire_switched = cache = 0
    switched = args.reply == "switched"
    for i, wl in enumerate(ops):
        n, r, m = wl.shape
        plan = pimm.Plan(ctx, n, r, m, d_fix=args.layer_d)
        w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
        fi = plan.info
        st = dict(
            plan=plan, w=w, X=pimm.to_device_u64(wl.X),
            pt=torch.empty((fi.I, N), dtype=torch.int64, device=dev),
            ct=torch.empty((fi.I, 2, L, N), dtype=torch.int64, device=dev),
            acc=torch.empty((fi.O, 2, L, N), dtype=torch.int64, device=dev),
            c1=torch.empty((fi.O, L, N), dtype=torch.int64, device=dev),
            c0s=torch.empty((fi.O, L, fi.mb * fi.nb), dtype=torch.int64, device=dev),
            c1s=torch.empty((fi.O, L - 1, N), dtype=torch.int64, device=dev),
            c0ss=torch.empty((fi.O, L - 1, fi.mb * fi.nb), dtype=torch.int64, device=dev),
            y0=torch.empty((n, m), dtype=torch.int64, device=dev),
            y1=torch.empty((n, m), dtype=torch.int64, device=dev),
            ws=plan.workspace(), op=i)
        state.append(st)
        if args.schedules:
            plan.set_tuning(*(int(v) for v in args.schedules.split(";")[i].split(",")))
        elif not args.no_autotune:
            # The product's schedule is picked by the library's autotuner on these buffers.
            ct0 = pimm.encrypt(plan, sk, cseed, AUTOTUNE_OP + i, pimm.encode_input(plan, st["X"]))
            acc0 = torch.empty((fi.O, 2, L, N), dtype=torch.int64, device=dev)
            best = plan.autotune(w, ct0, acc0, reps=2)
            st["tuning"] = plan.tuning()
            log(f"  autotuned product schedule (rows, column blocks, grid waves) = {st['tuning']}: "
                f"{best:.3f} ms")
            del ct0, acc0
        useful += n * r * m
        mac_bytes += (fi.Wb + 2 * fi.I + 2 * fi.O) * L * N * 8
        slot_macs += 2 * L * N * fi.P
        butterflies += L * (N // 2) * (N.bit_length() - 1) * (2 * fi.I + 2 * fi.O)
        wire += fi.ct_bytes + fi.c1_bytes + fi.c0s_bytes
        wire_seeded += fi.ct_bytes // 2 + 32 + fi.c1_bytes + fi.c0s_bytes
        wire_switched += fi.ct_bytes + (fi.c1_bytes + fi.c0s_bytes) * (L - 1) // L
        cache += fi.weights_bytes
        log(f"{wl.name}: plan ({fi.mb},{fi.rb},{fi.nb}) I={fi.I} O={fi.O} Wb={fi.Wb} "
            f"weights {fi.weights_bytes / 1e9:.2f} GB")
    torch.cuda.synchronize()

    def step(k):
        for st in state:
            p = st["plan"]
            pimm.encrypt_input(p, sk, cseed, k * 8 + st["op"], st["X"], st["ct"], st["ws"])
            pimm.matmul_share(p, st["w"], pk, sseed, k * 8 + st["op"], st["ct"], st["c1"],
                              st["c0s"], st["y1"], st["ws"])
            if switched:
                pimm.mod_switch(p, st["w"], st["c1"], st["c0s"], st["c1s"], st["c0ss"])
                pimm.decrypt_switched(p, sk, st["c1s"], st["c0ss"], st["y0"], st["ws"])
            else:
                pimm.decrypt(p, sk, st["c1"], st["c0s"], st["y0"], st["ws"])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    classes = ("mac", "ntt_fwd", "ntt_inv", "sample", "encode", "decode", "mask_extract",
               "mod_switch")
    for kname in classes:
        pimm.profile_read(kname)
    # Timed region: HIP events bracket the product launches only (an event recorded
    # between two dependent launches delays the second by a few microseconds).
    pimm.profile_select(["mac"])
    pimm.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pimm.profile_enable(False)
    elapsed = t1 - t0
    mac_cnt, mac_ms = pimm.profile_read("mac")
    log(f"timed {args.steps} steps in {elapsed:.4f} s")
    # Per-class breakdown from separate, untimed steps with every class recorded.
    pimm.profile_select(None)
    pimm.profile_enable(True)
    nb = max(2, min(5, args.steps))
    for k in range(nb):
        step(30_000 + k)
    torch.cuda.synchronize()
    pimm.profile_enable(False)
    kernels = {}
    for kname in classes:
        cnt, ms = pimm.profile_read(kname)
        kernels[kname] = {"launches_per_step": cnt / nb, "ms_per_step": round(ms / nb, 4)}

    # The server's part alone (rows A4-A9: forward NTT through the masked reply) on inputs
    # encrypted beforehand.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for st in state:
            pimm.matmul_share(st["plan"], st["w"], pk, sseed, (20_000 + k) * 8 + st["op"], st["ct"],
                              st["c1"], st["c0s"], st["y1"], st["ws"])
    torch.cuda.synchronize()
    server_s = (time.perf_counter() - t0) / args.steps

    # The server's completion of each fully connected layer (x1 W + b added to its share;
    # not part of the timed step): x1 and b are synthetic, the shares are the step's.
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    for st in state:
        fi = st["plan"].info
        st["x1"] = torch.randint(0, 1 << ell, (fi.n, fi.r), generator=gen, device=dev)
        st["b"] = torch.randint(-(1 << 30), 1 << 30, (fi.m,), generator=gen, device=dev)
    for st in state:
        pimm.fc_complete(st["plan"], st["w"], st["x1"], st["b"], st["y1"], st["ws"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for st in state:
            pimm.fc_complete(st["plan"], st["w"], st["x1"], st["b"], st["y1"], st["ws"])
    torch.cuda.synchronize()
    fc_s = (time.perf_counter() - t0) / args.steps

    # Seed-compressed upload: the server's rebuild of the ciphertexts from c0 and the public
    # seed (not part of the timed step, whose client uploads whole ciphertexts).
    aseed = workloads.seed("public", 1)
    for st in state:
        st["c0"] = st["ct"][:, 0].contiguous()
        st["ctx_"] = torch.empty_like(st["ct"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for st in state:
            pimm.ct_expand(st["plan"], aseed, st["op"], st["c0"], st["ctx_"])
    torch.cuda.synchronize()
    expand_s = (time.perf_counter() - t0) / args.steps

    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Per-step latency of the layer (each step synchronised), for p50/p99.
    lat = []
    for k in range(max(5, min(30, args.steps * 2))):
        torch.cuda.synchronize()
        a = time.perf_counter()
        step(10_000 + k)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)

    # The same step captured once into a HIP graph and replayed (the calls allocate nothing
    # and record no memset).  A replay repeats the captured operation ids, so it is reported
    # beside the measured step, not as it; every checked replay equals the eager step.
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        step(50_000)
    torch.cuda.synchronize()
    gref = [(st["y0"].clone(), st["y1"].clone()) for st in state]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        step(50_000)
    graph_same = True
    for _ in range(3):
        for st in state:
            st["y0"].zero_()
            st["y1"].zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        graph_same = graph_same and all(torch.equal(st["y0"], a) and torch.equal(st["y1"], b)
                                        for st, (a, b) in zip(state, gref))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / args.steps
    log(f"step as a HIP graph: {graph_s * 1e3:.3f} ms (replays bit-exact: {graph_same})")

    mac_avg_s = mac_ms / 1e3 / max(1, mac_cnt)
    bytes_per_launch = mac_bytes / len(state)
    achieved = bytes_per_launch / mac_avg_s / 1e9 if mac_cnt else 0.0
    value = useful * args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "int-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"BERT-base-shaped linear layer, seq {args.seq}: QKV 768x2304, "
                        "attn-out 768x768, FFN 768x3072 and 3072x768; RNS-BFV N=4096, "
                        "2x50-bit primes, t=2^37, 12 fractional bits; "
                        + ("fewest-wire plan" if not args.layer_d else
                           f"fixed block area {args.layer_d}") + "; weight cache built at load",
            "global_batch": 1, "seq_len": args.seq, "parallelism": "single GPU",
            "plans": [[s["plan"].mb, s["plan"].rb, s["plan"].nb] for s in state],
            "product_schedules": [list(s["plan"].tuning()) for s in state],
            "useful_macs_per_step": useful,
        },
        "server_path_ms": server_s * 1e3,
        "server_path_int_mac_per_s": useful / server_s,
        "graph_replay_ms_per_step": graph_s * 1e3,
        "graph_replays_bitexact": bool(graph_same),
        "fc_completion_ms": fc_s * 1e3,
        "fc_completion_int_mac_per_s": useful / fc_s,
        "wire_bytes_per_step_seeded_upload": wire_seeded,
        "reply": ("switched: the last prime dropped before the reply is sent, decrypted with "
                  f"{L - 1} prime" if switched else f"full: {L} primes"),
        "wire_bytes_per_step_switched_reply": wire_switched,
        "seeded_upload_expand_ms": expand_s * 1e3,
        "slot_mac_per_s": slot_macs * args.steps / elapsed,
        "server_ntt_butterflies_per_s": butterflies * args.steps / elapsed,
        "wire_bytes_per_step": wire,
        "weight_cache_bytes": cache,
        "layer_latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99)), "samples": len(lat)},
        "kernels_untimed_breakdown": kernels,
        "roofline": {
            "kernel": "k_mac_sk (the slot-wise product)", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic([s["plan"].tuning() for s in state]),
            "alg_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": mac_avg_s * 1e3,
        },
        "cpu_baseline": None,
    }
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seq", type=int, default=128)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB device to device "
                         "(a known-size reference for hardware byte counters)")
    ap.add_argument("--workload", choices=["default", "layer", "batch", "serve", "peak", "stack",
                                           "pareto", "attention", "select"],
                    default="default",
                    help="default: the BERT-large stack (headline) with the BERT-base layer and "
                         "the batched-versus-plain comparison as extra keys")
    ap.add_argument("--no-layer", action="store_true",
                    help="default workload: skip the BERT-base layer")
    ap.add_argument("--no-batch", action="store_true",
                    help="default workload: skip the batched-versus-plain comparison")
    ap.add_argument("--stack-layers", type=int, default=24)
    ap.add_argument("--reply", choices=["switched", "full"], default="switched",
                    help="stack and layer: send the reply with its last prime dropped (modulus "
                         "switching; the same shares) or with all primes")
    ap.add_argument("--serve-tile", type=lambda v: tuple(int(x) for x in v.split(",")),
                    default=(4, 8), help="serve: product tile 'rows,cols' of the batched launch")
    ap.add_argument("--pareto-d", type=lambda v: [int(x) for x in v.split(",")],
                    default=[0, 64, 128, 256, 1024],
                    help="block areas of the pareto workload (0: the fewest-wire plan)")
    ap.add_argument("--link-gbps", type=lambda v: [float(x) for x in v.split(",")],
                    default=[1, 10, 100, 400, 1600],
                    help="select: link speeds in Gbit/s")
    ap.add_argument("--att-streams", type=int, default=8,
                    help="streams per phase of the attention workload")
    ap.add_argument("--layer-d", type=int, default=0,
                    help="layer workload: fixed block area m_b*r_b (0: the fewest-wire plan)")
    ap.add_argument("--schedules", default="",
                    help="product schedules 'rows,cols,waves;...' per product (skips the autotuner)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default product schedule instead of autotuning it per product")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--d-fix", type=int, default=32)
    ap.add_argument("--layers", type=int, default=12)
    ap.add_argument("--serve-budget-gb", type=float, default=48.0)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-min-batch", type=int, default=8,
                    help="serve: fewest requests at one step that run as one batched pass")
    ap.add_argument("--serve-max-active", type=int, default=32)
    ap.add_argument("--serve-rate0", type=float, default=4.0)
    ap.add_argument("--serve-rates", type=lambda v: [float(x) for x in v.split(",")], default=None,
                    help="serve: run only these arrival rates (comma-separated)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); sharding Pi_MatMul "
              "over several GPUs is described, not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2305_18396_amd import pimm, workloads

    if args.workload == "batch":
        print(json.dumps({"metric": METRIC, "batch": bench_batch(args)}), flush=True)
        return
    if args.workload == "stack":
        print(json.dumps({"metric": METRIC, "stack": bench_stack(args)}), flush=True)
        return
    if args.workload == "peak":
        print(json.dumps({"metric": METRIC, "peak": bench_peak(args)}), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps({"metric": METRIC, "serve": bench_serve(args)}), flush=True)
        return
    if args.workload == "attention":
        print(json.dumps({"metric": METRIC, "attention": bench_attention(args)}), flush=True)
        return
    if args.workload == "pareto":
        print(json.dumps({"metric": METRIC, "pareto": bench_pareto(args)}), flush=True)
        return
    if args.workload == "select":
        if args.pareto_d == [0, 64, 128, 256, 1024]:
            args.pareto_d = [0, 64, 128, 256]
        print(json.dumps({"metric": METRIC, "select": bench_select(args)}), flush=True)
        return

    if args.workload == "layer":
        out = bench_layer(args)
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle) ...")
            out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        print(json.dumps(out), flush=True)
        return

    # Default: the BERT-large-shaped 24-layer stack is the headline (the largest configuration
    # that fits one GPU), with the BERT-base layer and the batched-versus-plain comparison as
    # extra keys.
    st = bench_stack(args)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": st["int_mac_per_s"],
        "unit": "int-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": st["s_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": st["workload"], "global_batch": 1, "seq_len": 512,
                   "parallelism": "single GPU", "plans": st["plans"],
                   "product_schedules": st["product_schedules"],
                   "useful_macs_per_step": st["useful_macs_per_step"]},
        "stack_latency_ms": st["stack_latency_ms"],
        "layer_latency_ms": st["layer_latency_ms"],
        "roofline": st["roofline"],
        "stack": {k: v for k, v in st.items() if k not in ("roofline", "workload", "plans",
                                                           "product_schedules",
                                                           "stack_latency_ms",
                                                           "layer_latency_ms")},
        "cpu_baseline": None,
    }
    if not args.no_layer:
        lay = bench_layer(args)
        out["bert_base_layer"] = {k: v for k, v in lay.items()
                                  if k not in ("metric", "unit", "n_gpus", "higher_is_better",
                                               "scaling", "vs_baseline", "dtype", "data",
                                               "cpu_baseline")}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if not args.no_batch:
        bsteps, args.steps = args.steps, min(args.steps, 5)
        b = bench_batch(args)
        args.steps = bsteps
        out["batched_vs_plain"] = b
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample of the stack) ...")
        out["cpu_baseline"] = cpu_baseline_stack(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
