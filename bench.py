#!/usr/bin/env python3
"""Benchmark: one encrypted bounding-box query per step on one MI355X.

Workload: 16-bit signed fixed-point latitude/longitude (9 integer + 7
fraction bits) against 16 encrypted boxes that tile a Korea-like region
(random guillotine widths), 32-bit encrypted payload per box; TFHE Torus32
parameters n=630, N=1024, k=1, Bg=2^7, l=3, key-switch base 2^2 with t=8.
The circuit (Algorithms 2-5) has 4112 gate bootstraps and 3088 key
switches in 24 depth levels.  Inputs and keys are resident on the GPU before
the timed region; a step is one full query evaluation.

Prints one JSON line: bootstraps/s (value), queries/s, p50/p99 latency, the
roofline of the blind-rotation kernel (event-timed live), the CPU oracle's
rate on a bounded sample of the same gate mix, and batched NAND throughput
against one bootstrap per launch.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gate bootstraps/s; bbox queries/s; p50/p99 query latency on 1 MI355X"
# MI355X: 256 CUs x 64 lanes x 2.4 GHz full-rate 32-bit VALU lane-ops
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of one blind-rotation launch: the bootstrapping key
# in the NTT domain once (630 x 6 x 2 x 1024 u64), plus per job its two
# LWE_n inputs and its extracted LWE_N output (u32 words).
BSK_NTT_BYTES = 630 * 6 * 2 * 1024 * 8
BR_JOB_BYTES = (2 * 631 + 1025) * 4
# Algorithmic integer work of one blind rotation in 32-bit VALU lane-cycles:
# 630 CMux steps x (6 forward + 2 inverse radix-2 1024-point NTTs = 40960
# butterflies, plus 12 x 1024 pointwise products) = 25.8 M butterflies and
# 7.74 M products; a Goldilocks mulmod costs 4 quarter-rate 32x32 multiplies
# (16 lane-cycles) + 12 ALU ops, an add or subtract mod p 6 ops, so a
# butterfly is 40 and a pointwise multiply-accumulate 35 lane-cycles.
ALG_LANE_CYCLES_PER_BR = 630 * ((6 + 2) * 5120 * 40 + 12 * 1024 * 35)
KERNEL_SOURCES = ["paper_2407_19871_amd/csrc/kernels.hip", "paper_2407_19871_amd/csrc/ntt32.h",
                  "paper_2407_19871_amd/csrc/ntt64.h", "paper_2407_19871_amd/csrc/gl64.h"]
# blind-rotation kernel of each launch shape (waves per bootstrap)
SHAPE_KERNEL = {1: "blind_rotate_kernel<1>", 2: "blind_rotate_pair_kernel", 3: "blind_rotate_kernel<3>",
                4: "blind_rotate_kernel<4>", 5: "blind_rotate_kernel<5>", 6: "blind_rotate_split_kernel"}
TUNE_BUCKETS = (1, 16, 32, 64, 128, 256, 384, 512, 768, 1024, 2048, 4096, 16384)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "blind_rotate_bbox16x16_traffic.txt")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "blind_rotate_valu_issue.txt")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Per-launch HBM bytes of one blind-rotation kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on these
    kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    txt = open(TRAFFIC_SUMMARY).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", txt, re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("kernels", {}).get(kernel)


def load_valu():
    """VALU issue fractions of the blind-rotation kernel from the committed
    rocprofv3 SQ_INSTS_VALU summary, if it was taken on this kernel."""
    if not os.path.exists(VALU_SUMMARY):
        return None
    m = re.search(r"^valu_json:\s*(\{.*\})\s*$", open(VALU_SUMMARY).read(), re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    return d if d.get("kernel_hash") == kernel_hash() else None


def cpu_baseline(seed: int):
    """The oracle as it stands, on a bounded sample of the query's gate mix:
    256 XNOR + 128 MUX gates (512 bootstraps, the comparator mix), OpenMP over
    every host thread."""
    import oracle as O
    keys = O.keygen(seed)
    ctx = O.Ctx(keys)
    rng = np.random.default_rng(seed)
    nx, nm = 256, 128
    bits = rng.integers(0, 2, 2 * nx + 3 * nm).astype(np.uint8)
    ct = O.encrypt_bits(keys, bits, seed=seed + 1)
    t0 = time.perf_counter()
    _, th1 = ctx.gate_batch("XNOR", ct[:nx], ct[nx:2 * nx])
    o = 2 * nx
    _, th2 = ctx.gate_batch("MUX", ct[o:o + nm], ct[o + nm:o + 2 * nm], ct[o + 2 * nm:o + 3 * nm])
    dt = time.perf_counter() - t0
    n_br = nx + 2 * nm
    # one thread: the oracle's single-gate entry, 8 XNOR + 4 MUX gates
    t0 = time.perf_counter()
    for k in range(8):
        ctx.gate("XNOR", ct[k], ct[nx + k])
    for k in range(4):
        ctx.gate("MUX", ct[o + k], ct[o + nm + k], ct[o + 2 * nm + k])
    dt1 = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(n_br / dt, 2), "unit": "bootstraps/s", "cores": int(max(th1, th2)), "kind": "oracle",
            "sample": f"{nx} XNOR + {nm} MUX gates = {n_br} bootstraps with key switching, "
                      f"same parameters, {dt:.1f} s", "host_cpus": os.cpu_count(), "cpu_model": model,
            "single_core": {"value": round(16 / dt1, 2), "unit": "bootstraps/s",
                            "sample": f"8 XNOR + 4 MUX gates = 16 bootstraps on one thread, {dt1:.1f} s"}}


def summarize_launches(launches, depth: int, l: int):
    """Per-kind totals, the time-weighted fraction of the chip's 1024 SIMDs
    that hold a blind-rotation wave, and the split of a query's time into
    the paper's Table 2 phases by depth level.  A query launches one blind
    rotation and one key switch per level, in level order; levels [0, l]
    are the comparators (the XNOR level and l MUX levels), the next three
    the validation ANDs (bounds, box, service), the rest the XOR tree.
    With an odd box count one box's chain runs a few levels late, so the
    split by level is then approximate."""
    tot = {k: {"launches": 0, "jobs": 0, "total_ms": 0.0} for k in ("blind_rotate", "keyswitch")}
    busy = 0.0
    per_level = np.zeros(depth)
    n_rot, level = 0, 0
    for r in launches:
        t = tot[r["name"]]
        t["launches"] += 1
        t["jobs"] += r["jobs"]
        t["total_ms"] += r["ms"]
        if r["name"] == "blind_rotate":
            busy += r["ms"] * min(r["jobs"] * r["shape"], 1024) / 1024
            level = n_rot % depth
            n_rot += 1
        per_level[level] += r["ms"]   # a key switch belongs to the rotation before it
    per_level /= max(1, n_rot // depth)
    br_ms = tot["blind_rotate"]["total_ms"]
    # rotation launches by shape (waves per bootstrap), i.e. by kernel
    by_shape = {}
    for r in launches:
        if r["name"] == "blind_rotate":
            t = by_shape.setdefault(r["shape"], {"launches": 0, "jobs": 0, "total_ms": 0.0})
            t["launches"] += 1
            t["jobs"] += r["jobs"]
            t["total_ms"] += r["ms"]
    tot["blind_rotate_by_shape"] = by_shape
    phases = {"comparison": per_level[:l + 1].sum(), "validation": per_level[l + 1:l + 4].sum(),
              "hom_add_xor": per_level[l + 4:].sum()}
    return tot, (busy / br_ms if br_ms else None), {k: round(float(v), 2) for k, v in phases.items()}


def microbench(lp, torch, sk, dk, sizes=(1, 64, 1024, 16384)):
    """Batched NAND bootstraps (one launch pair per batch) and the plain
    one-bootstrap-per-launch path."""
    res = {}
    rng = np.random.default_rng(3)
    for B in sizes:
        bits = rng.integers(0, 2, 2 * B).astype(np.uint8)
        ct = sk.encrypt_bits(bits, seed=30 + B)
        c1, c2 = lp.to_device(ct[:B]), lp.to_device(ct[B:])
        # warm up for at least a quarter second of work: after the light
        # launches before it, the first full-chip batches run while the
        # GPU's clocks are still ramping up
        t_w = time.perf_counter()
        while True:
            out = lp.bootstrap_batch(dk, "NAND", c1, c2)
            torch.cuda.synchronize()
            if time.perf_counter() - t_w >= 0.25:
                break
        reps = 3 if B <= 1024 else 1
        t0 = time.perf_counter()
        for _ in range(reps):
            out = lp.bootstrap_batch(dk, "NAND", c1, c2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        d, _ = sk.decrypt_bits(lp.to_host(out))
        assert (d == 1 - (bits[:B] & bits[B:])).all()
        res[str(B)] = round(B / dt, 1)
        print(f"bench: NAND batch {B}: {res[str(B)]} bootstraps/s", file=sys.stderr, flush=True)
    # one bootstrap per launch: 16 single-gate launches back to back
    ct = sk.encrypt_bits(rng.integers(0, 2, 32).astype(np.uint8), seed=99)
    cs = [(lp.to_device(ct[k:k + 1]), lp.to_device(ct[16 + k:17 + k])) for k in range(16)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in cs:
        lp.bootstrap_batch(dk, "NAND", a, b)
    torch.cuda.synchronize()
    one = 16 / (time.perf_counter() - t0)
    return {"batched_nand_bootstraps_per_s": res, "one_per_launch_bootstraps_per_s": round(one, 1)}


def serve_bench(requests_per_rate: int, tick_cap: int = 0, seed: int = 5):
    """Serving: requests with their own keys (a pool of client keys, each
    uploaded and converted on the GPU per request), 16- or 32-bit signed
    coordinates, 1..256 boxes log-uniform, 32-bit payloads.  A burst measures
    the saturated rate, then Poisson arrivals at 0.25/0.5/0.75/0.95 of it.
    tick_cap > 0 caps the blind rotations of a server tick; p50 is also
    given for requests of at most 16 boxes and for larger ones."""
    import math
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    rng = np.random.default_rng(seed)
    clients = [lp.keygen(None, 5000 + c) for c in range(8)]
    # launch shapes are per device, not per key: tune once with one client key
    lp.autotune(lp.DeviceKey(clients[0][1]), buckets=TUNE_BUCKETS, br_steps=64)

    def make_request(i):
        c = i % len(clients)
        l = 16 if rng.random() < 0.5 else 32
        nb = int(min(256, max(1, math.floor(math.exp(rng.uniform(0, math.log(257)))))))
        q = W.random_query(10000 + i, l, nb, 32, region=W.KOREA if i % 2 else W.ZERO_STRADDLE,
                           force_inside=bool(rng.random() < 0.8))
        xb, yb, bb, pb = q.plain_bits()
        sk, ck = clients[c]
        ct = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=20000 + i)
        L, N = q.l, q.n_boxes
        parts = (ct[:L], ct[L:2 * L], ct[2 * L:2 * L + 4 * L * N], ct[2 * L + 4 * L * N:])
        return q, c, parts

    def run(reqs, arrivals):
        srv = lp.Server(200 << 30, max_tick_rotations="auto" if tick_cap < 0 else tick_cap)
        t0 = time.perf_counter()
        tickets = []
        for (q, c, parts), at in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(clients[c][1], q.l, q.n_boxes, q.m, True, *parts))
        lats, ok = [], True
        for (q, c, parts), t in zip(reqs, tickets):
            st, out, lat = srv.poll(t)
            d, _ = clients[c][0].decrypt_bits(out)
            ok &= st == 0 and W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True)
            lats.append(lat)
        wall = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        n_br = sum(lp.bbox_counts(q.l, q.n_boxes, q.m)[0] for q, _, _ in reqs)
        small = [x for x, (q, _, _) in zip(lats, reqs) if q.n_boxes <= 16]
        large = [x for x, (q, _, _) in zip(lats, reqs) if q.n_boxes > 16]
        p50 = lambda v: round(float(np.percentile(v, 50)) * 1e3, 1) if v else None
        return {"queries_per_s": round(len(reqs) / wall, 3), "bootstraps_per_s": round(n_br / wall, 1),
                "p50_ms": p50(lats), "p99_ms": round(float(np.percentile(lats, 99)) * 1e3, 1),
                "p50_ms_upto16_boxes": p50(small), "p50_ms_over16_boxes": p50(large),
                "requests": len(reqs), "ticks": stats["ticks"], "widest_tick": stats["widest_tick"],
                "correct": bool(ok)}

    burst = [make_request(i) for i in range(requests_per_rate)]
    sat = run(burst, [0.0] * len(burst))
    print(f"serve: burst done, {sat['queries_per_s']} queries/s", file=sys.stderr, flush=True)
    res = {"metric": "serving: p50/p99 latency and queries/s under Poisson arrivals on 1 MI355X",
           "tick_cap": tick_cap, "saturated": sat, "rates": []}
    for k, f in enumerate((0.25, 0.5, 0.75, 0.95)):
        reqs = [make_request(1000 * (k + 1) + i) for i in range(requests_per_rate)]
        lam = f * sat["queries_per_s"]
        arr = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
        r = run(reqs, list(arr))
        print(f"serve: rate {f} done, p50 {r['p50_ms']} ms", file=sys.stderr, flush=True)
        r["offered_fraction"] = f
        r["offered_queries_per_s"] = round(lam, 3)
        res["rates"].append(r)
    print(json.dumps(res), flush=True)


def clients_bench(n_clients: int, steps: int, warmup: int, seed: int = 4):
    """Many clients at once, each with its own keys: the first half use 32-bit
    floor(deg * 1e6) signed coordinates, the second half 16-bit 9.7 ones; box
    counts uniform in 1..64; 32-bit payloads; the Korea-like region, the
    zero-straddling one for odd clients.  All queries run as one fused program:
    level L of every query is one blind-rotation and one key-switch launch,
    each replayed from its hipGraph.  Every result is checked against the
    plaintext predicate."""
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    lp.autotune(lp.DeviceKey(lp.keygen(None, 1000 * seed + 999)[1]), buckets=TUNE_BUCKETS, br_steps=64)
    keys, sks, qs, items = [], [], [], []
    n_br = n_ks = 0
    for c in range(n_clients):
        l = 32 if c < n_clients // 2 else 16
        nb = int(rng.integers(1, 65))
        q = W.random_query(40000 + c, l, nb, 32, region=W.ZERO_STRADDLE if c % 2 else W.KOREA)
        sk, ck = lp.keygen(None, 1000 * seed + c)
        keys.append(lp.DeviceKey(ck))
        del ck
        xb, yb, bb, pb = q.plain_bits()
        ct = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=50000 + c)
        L, N = q.l, q.n_boxes
        items.append((L, N, q.m, True, *[lp.to_device(a) for a in
                                         (ct[:L], ct[L:2 * L], ct[2 * L:2 * L + 4 * L * N], ct[2 * L + 4 * L * N:])]))
        sks.append(sk)
        qs.append(q)
        br, ks, _ = lp.bbox_counts(L, N, q.m)
        n_br += br
        n_ks += ks
        if (c + 1) % 32 == 0:
            print(f"clients: {c + 1} keys and queries on the device", file=sys.stderr, flush=True)
    setup = time.perf_counter() - t0
    outs = None
    for _ in range(warmup):
        outs = lp.eval_bbox_batch(keys, items, outs)
    torch.cuda.synchronize()
    print("clients: warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        outs = lp.eval_bbox_batch(keys, items, outs)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ok = True
    for sk, q, o in zip(sks, qs, outs):
        d, _ = sk.decrypt_bits(lp.to_host(o))
        ok &= W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True)
    res = {"metric": "fused queries of many clients with their own keys on 1 MI355X",
           "clients": n_clients, "bootstraps": n_br, "keyswitches": n_ks,
           "levels": max(lp.bbox_counts(q.l, q.n_boxes, q.m)[2] for q in qs),
           "device_key_gb": round(sum(k.bytes for k in keys) / 1e9, 2),
           "seconds_per_batch": round(wall, 3), "bootstraps_per_s": round(n_br / wall, 1),
           "queries_per_s": round(n_clients / wall, 3), "steps": steps, "warmup": warmup,
           "setup_s": round(setup, 1), "correct_vs_predicate": bool(ok)}
    print(json.dumps(res), flush=True)


def sweep_bench(reps: int = 3, seed: int = 6):
    """The paper's experiment shapes on the GPU, 8- to 32-bit synthetic
    queries over the Korea-like region (a continent-sized one at 8 bits), one
    query at a time: Fig. 4a (N = 10
    boxes, m = 9, l = 8/16/24/32), Table 2 (the nine city boxes and services
    printed in Table 1, N = m = 9, at l = 13 and 16, under both the lambda 128
    and the lambda 80 parameter sets, for a point in Seoul), Fig. 4b (l = 16,
    N = 10, m = 1 to 64; the paper prints no values for it) and a sweep over
    N at l = 16, m = 9.  The paper's CPU times (6-core Ryzen 5
    3500X, TFHE 1.1) are listed beside the Fig. 4a and Table 2 shapes as
    context, not as a target."""
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    keys = {}
    for name, params in (("lambda128", None), ("lambda80", lp.params_lambda80())):
        sk, ck = lp.keygen(params, seed)
        keys[name] = (sk, lp.DeviceKey(ck))
    lp.autotune(keys["lambda128"][1], buckets=TUNE_BUCKETS, br_steps=64)
    fig4a = {8: 3.256, 16: 6.139, 24: 8.764, 32: 11.670}  # seconds, Fig. 4a
    table2 = {"lambda128": {13: 4.88, 16: 5.67}, "lambda80": {13: 4.36, 16: 5.12}}  # seconds, Table 2
    shapes = [("fig4a", "lambda128", l, 10, 9, fig4a[l]) for l in (8, 16, 24, 32)]
    shapes += [("table2", ps, l, 9, 9, table2[ps][l]) for ps in ("lambda128", "lambda80") for l in (13, 16)]
    shapes += [("fig4b", "lambda128", 16, 10, m, None) for m in (1, 16, 32, 64)]
    shapes += [("boxes", "lambda128", 16, N, 9, None) for N in (1, 4, 16, 28)]
    with open(os.path.join(ROOT, "tests", "golden", "table1_covid_boxes.json")) as f:
        table1 = json.load(f)["rows"]
    rows = []
    for k, (kind, ps, l, N, m, paper_s) in enumerate(shapes):
        sk, dk = keys[ps]
        if kind == "table2":
            q = W.table1_query((37.55, 127.0), table1, l=l, m=m)
        else:
            # 8-bit codes step 2 degrees: a Korea-sized tiling of 10 boxes would
            # quantize to empty boxes, so that shape tiles a continent-sized region
            region = W.KOREA if l >= 13 else (-60.0, 60.0, -120.0, 120.0)
            q = W.random_query(60000 + k, l, N, m, region=region, force_inside=True)
        xb, yb, bb, pb = q.plain_bits()
        ct = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=61000 + k)
        parts = [lp.to_device(a) for a in (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])]
        out = lp.eval_bbox_query(dk, l, N, m, True, *parts)
        torch.cuda.synchronize()
        lp.profile_enable(True)
        lp.profile_collect_launches()
        t0 = time.perf_counter()
        for _ in range(reps):
            lp.eval_bbox_query(dk, l, N, m, True, *parts, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        launches = lp.profile_collect_launches()
        lp.profile_enable(False)
        d, _ = sk.decrypt_bits(lp.to_host(out))
        n_br, _, levels = lp.bbox_counts(l, N, m)
        _, busy, phases = summarize_launches(launches, levels, l)
        row = {"kind": kind, "params": ps, "l": l, "boxes": N, "m": m, "bootstraps": n_br, "levels": levels,
               "phases_ms": phases, "busy_simd_frac": round(busy, 3) if busy is not None else None,
               "inputs": "Table 1 boxes and services" if kind == "table2" else "synthetic tiling",
               "ms_per_query": round(dt * 1e3, 1), "bootstraps_per_s": round(n_br / dt, 1),
               "correct_vs_predicate": bool(W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m,
                                                                            True))}
        if paper_s is not None:
            row["paper_cpu_s"] = paper_s
        rows.append(row)
        print(f"sweep: {kind} {ps} l={l} N={N}: {row['ms_per_query']} ms", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "paper experiment shapes: bbox query latency on 1 MI355X", "rows": rows}), flush=True)


def small_query(lp, torch, reps: int = 5):
    """The 8-bit unsigned coordinates vs one box query with an 8-bit payload
    (107 bootstraps in 12 levels), with its own key."""
    from oracle import plain
    from paper_2407_19871_amd import workloads as W
    q = W.random_query_u8(1, force_inside=True)
    sk, ck = lp.keygen(None, 1)
    dk = lp.DeviceKey(ck)
    xb, yb, bb, pb = q.plain_bits()
    ct = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=1)
    l, N, m = q.l, q.n_boxes, q.m
    parts = [lp.to_device(a) for a in (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])]
    out = lp.eval_bbox_query(dk, l, N, m, False, *parts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lp.eval_bbox_query(dk, l, N, m, False, *parts, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    d, _ = sk.decrypt_bits(lp.to_host(out))
    n_br, _, levels = lp.bbox_counts(l, N, m)
    return {"workload": "8-bit unsigned point vs 1 encrypted box, 8-bit payload", "bootstraps": n_br,
            "levels": levels, "ms_per_query": round(dt * 1e3, 2), "bootstraps_per_s": round(n_br / dt, 1),
            "correct_vs_predicate": bool(W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m,
                                                                         False))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run device copies of this many bytes (traffic calibration)")
    ap.add_argument("--serve", type=int, default=0,
                    help="serving benchmark with this many requests per arrival rate (separate JSON line)")
    ap.add_argument("--tick-cap", type=int, default=0,
                    help="with --serve: blind rotations per server tick at most (0 = whole levels, "
                         "-1 = sized from the timed launch-shape table)")
    ap.add_argument("--sweep", action="store_true",
                    help="the paper's Fig. 4a / Table 2 query shapes and a box-count sweep (separate JSON line)")
    ap.add_argument("--clients", type=int, default=0,
                    help="fused queries of this many clients with their own keys (separate JSON line)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing them on this device first")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the gate-bootstrap path here runs on a single MI355X "
              f"and has no multi-GPU mode (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_bench(args.serve, args.tick_cap)
        return
    if args.clients:
        clients_bench(args.clients, args.steps, args.warmup)
        return
    if args.sweep:
        sweep_bench()
        return

    import torch

    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    seed = 2
    q = W.random_query(seed, 16, 16, 32, force_inside=True)
    sk, ck = lp.keygen(None, seed)
    xb, yb, bb, pb = q.plain_bits()
    cts = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=seed)
    l, N, m = q.l, q.n_boxes, q.m
    d_x = lp.to_device(cts[:l])
    d_y = lp.to_device(cts[l:2 * l])
    d_b = lp.to_device(cts[2 * l:2 * l + 4 * l * N])
    d_p = lp.to_device(cts[2 * l + 4 * l * N:])
    dk = lp.DeviceKey(ck)
    n_br, n_ks, levels = lp.bbox_counts(l, N, m)
    tune = None
    if not args.no_autotune:
        # launch shapes per batch size, timed on this device before anything
        # is measured (covers the query's level widths and the batch sizes)
        t0 = time.perf_counter()
        rows = lp.autotune(dk, buckets=TUNE_BUCKETS, br_steps=64)
        tune = {"seconds": round(time.perf_counter() - t0, 2), "br_steps_timed": 64, "rows": rows}
        print(f"bench: autotune done in {tune['seconds']} s", file=sys.stderr, flush=True)
    out = torch.empty((m, 631), dtype=torch.int32, device="cuda")

    def step():
        lp.eval_bbox_query(dk, l, N, m, True, d_x, d_y, d_b, d_p, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    d, _ = sk.decrypt_bits(lp.to_host(out))
    expect = plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m, True)
    correct = W.from_bits(d) == expect

    lp.profile_enable(True)
    lp.profile_collect_launches()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        step()
        ev[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = lp.profile_collect_launches()
    lp.profile_enable(False)
    stats, busy_simd, phases = summarize_launches(launches, levels, l)
    print(f"bench: {args.steps} queries timed, {wall * 1e3 / args.steps:.1f} ms each", file=sys.stderr, flush=True)
    lat = np.array([a.elapsed_time(b) for a, b in ev])

    br = stats.get("blind_rotate", {"launches": 0, "jobs": 0, "total_ms": 0.0})
    ks = stats.get("keyswitch", {"launches": 0, "jobs": 0, "total_ms": 0.0})
    by_shape = stats.get("blind_rotate_by_shape", {})

    def tops(jobs, ms):
        return ALG_LANE_CYCLES_PER_BR * jobs / (ms / 1e3) / 1e12 if ms else 0.0

    # the dominant kernel: the rotation shape with the most time in the query
    dom = max(by_shape, key=lambda w: by_shape[w]["total_ms"]) if by_shape else 3
    dk_ = by_shape.get(dom, {"launches": 0, "jobs": 0, "total_ms": 0.0})
    dom_avg_ms = dk_["total_ms"] / max(1, dk_["launches"])
    achieved = tops(dk_["jobs"], dk_["total_ms"])
    traffic = load_traffic(SHAPE_KERNEL[dom])
    valu = load_valu()
    roofline = {
        "bound": "alu", "kernel": SHAPE_KERNEL[dom],
        "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
        "frac": round(achieved / VALU_PEAK_TOPS, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "avg_launch_ms": round(dom_avg_ms, 3),
        "bootstraps_per_launch": round(dk_["jobs"] / max(1, dk_["launches"]), 1),
        "op_unit": "32-bit VALU lane-cycles, 1.30e9 per bootstrap (algorithmic count)",
        # every rotation launch of the query, by kernel, and all of them together
        "by_kernel": {SHAPE_KERNEL[w]: {"launches": v["launches"], "jobs": v["jobs"],
                                        "total_ms": round(v["total_ms"], 3),
                                        "avg_launch_ms": round(v["total_ms"] / max(1, v["launches"]), 3),
                                        "frac": round(tops(v["jobs"], v["total_ms"]) / VALU_PEAK_TOPS, 4)}
                      for w, v in sorted(by_shape.items())},
        "all_rotations_frac": round(tops(br["jobs"], br["total_ms"]) / VALU_PEAK_TOPS, 4),
        # HBM side of the same kernel: rocprofv3 bytes per launch over the live
        # launch time, and the algorithmic bytes (key once, job ciphertexts)
        "hbm_gbs_rocprof": round(traffic["bytes_per_launch"] / (dom_avg_ms / 1e3) / 1e9, 2)
        if traffic and dom_avg_ms else None,
        "hbm_frac_rocprof": round(traffic["bytes_per_launch"] / (dom_avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5)
        if traffic and dom_avg_ms else None,
        "alg_bytes_per_launch": int(BSK_NTT_BYTES + BR_JOB_BYTES * dk_["jobs"] / max(1, dk_["launches"])),
        # measured: rocprofv3 SQ_INSTS_VALU x 4 cycles / (kernel time x 2.4 GHz x 1024 SIMDs)
        "valu_issue_frac_rocprof": valu["query_valu_issue_frac"] if valu else None,
        # time-weighted share of the 1024 SIMDs holding a rotation wave (narrow
        # levels leave most of the chip idle), and the issue rate of those
        "busy_simd_frac": round(busy_simd, 4) if busy_simd is not None else None,
        "valu_issue_frac_busy_simds": round(valu["query_valu_issue_frac"] / busy_simd, 4)
        if valu and busy_simd else None,
    }

    res = {
        "metric": METRIC,
        "value": round(n_br * args.steps / wall, 1),
        "unit": "bootstraps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "bbox query, 16-bit signed fixed-point point vs 16 encrypted boxes (guillotine "
                               "tiling of a Korea-like region), 32-bit encrypted payloads; TFHE Torus32 n=630, "
                               "N=1024, k=1, Bg=2^7, l=3, KS base 2^2 t=8",
                   "bootstraps_per_query": n_br, "keyswitches_per_query": n_ks, "levels": levels, "seed": seed},
        "queries_per_s": round(args.steps / wall, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "correct_vs_predicate": bool(correct),
        "kernels": {"blind_rotate_ms": round(br["total_ms"], 3), "keyswitch_ms": round(ks["total_ms"], 3),
                    "launches": br["launches"] + ks["launches"]},
        "roofline": roofline,
        # the paper's Table 2 phases of one query, by depth level (ms)
        "phases_ms": phases,
        "autotune": tune,
    }
    if not args.no_micro:
        res["microbench"] = microbench(lp, torch, sk, dk)
        big = (valu or {}).get("launches", {}).get("1x16384")
        res["microbench"]["valu_issue_frac_rocprof_16384"] = big["valu_issue_frac"] if big else None
        res["small_query"] = small_query(lp, torch)
    if args.copy_probe:
        src = torch.empty(args.copy_probe // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = args.copy_probe
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(seed)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
