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
roofline of the blind-rotation kernel (event-timed live, its operation count
priced by field-operation rates measured live), the CPU oracle on the run's
own keys and ciphertexts, and beside them the other workloads: the 8-bit
one-box query, batched NAND gates against one bootstrap per launch, 256
clients with their own keys fused per depth level, serving under Poisson
arrivals with a fresh key per request, and the paper's Table 2 shapes.
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
# MI355X 32-bit VALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T
# lane-ops/s.  A SIMD is 16 lanes wide but issues two wave64 VALU
# instructions per four cycles (the SQ_ACTIVE_INST_VALU2 counter counts such
# quad-cycles); the same per-clock width gives the published fp32 vector
# rate, 157.3 TFLOP/s = 78.6 T FMA/s.  Measured 32-bit additions reach about
# three quarters of it (op_prices reports the ratio).
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of one blind-rotation launch: the bootstrapping key
# in the NTT domain once (630 x 6 x 2 x 1024 u64), plus per job its two
# LWE_n inputs and its extracted LWE_N output (u32 words).
BSK_NTT_BYTES = 630 * 6 * 2 * 1024 * 8
BR_JOB_BYTES = (2 * 631 + 1025) * 4
# The method's field operations per CMux step of one blind rotation, in this
# library's formulation of the external product (Sec. 2.2, Bootstrap): 6
# forward transforms (2 accumulator components x 3 gadget levels) of 1024
# points, each 32 columns x 48 shift-twiddle butterflies (pass-1 stages 4, 2,
# 1) + 32 rows x 80 (pass 2), 32 x 32 digit butterflies (pass-1 stages 16
# and 8 on gadget digits, in int64) and 1024 twist products; per output
# component and level 1024 sums a*b + c*d (own and cross key products), and
# the level sums (2 additions per coefficient and component); 2 inverse
# transforms of 2 x 32 x 80 butterflies and 1024 twist products each; and
# 32-bit work: the rotation X^a ACC - ACC (2048 subtractions), the digits
# (3 operations for each of 6144) and the lift into ACC (2 x 2048).
OPS_PER_STEP = {
    "fwd_butterfly": 6 * 32 * 128,
    "digit_butterfly": 6 * 32 * 32,
    "mulmod": 8 * 1024,
    "mulsum": 2 * 3 * 1024,
    "add": 2 * 2 * 1024,
    "inv_butterfly": 2 * 2 * 32 * 80,
    "u32_add": 2048 + 3 * 6144 + 2 * 2048,
}
N_STEPS = 630
KERNEL_SOURCES = ["paper_2407_19871_amd/csrc/kernels.hip", "paper_2407_19871_amd/csrc/split.hip",
                  "paper_2407_19871_amd/csrc/kernel_util.h", "paper_2407_19871_amd/csrc/ntt32.h",
                  "paper_2407_19871_amd/csrc/ntt64.h", "paper_2407_19871_amd/csrc/gl64.h",
                  "paper_2407_19871_amd/_build.py"]
# blind-rotation kernel of each launch shape (waves per bootstrap)
SHAPE_KERNEL = {1: "blind_rotate_kernel<1>", 2: "blind_rotate_pair_kernel", 3: "blind_rotate_kernel<3>",
                4: "blind_rotate_kernel<4>", 5: "blind_rotate_kernel<5>", 6: "blind_rotate_split_kernel",
                7: "blind_rotate_split_kernel<dual>"}
TUNE_BUCKETS = (1, 16, 32, 64, 128, 256, 384, 512, 768, 1024, 2048, 4096, 16384)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "blind_rotate_bbox16x16_traffic.txt")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "blind_rotate_valu_busy.txt")


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
    """VALU busy fractions of the blind-rotation kernels from the committed
    rocprofv3 SQ_ACTIVE_INST_VALU summary (busy VALU issue cycles over the
    chip's dual-issue capacity), if it was taken on these kernel sources."""
    if not os.path.exists(VALU_SUMMARY):
        return None
    m = re.search(r"^valu_json:\s*(\{.*\})\s*$", open(VALU_SUMMARY).read(), re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    return d if d.get("kernel_hash") == kernel_hash() else None


def op_prices(lp, n_steps: int = N_STEPS):
    """Prices the rotation's operation count with field-operation rates
    measured now on this device (lp_debug_field_op_rates: each operation alone
    at full occupancy).  The price of an operation in 32-bit VALU lane-cycles
    is the chip's peak lane-op rate over the operation's measured rate, so
    the count is the lane-cycles the method's operations take when each runs
    at its own best rate, and a launch's fraction of the peak is at most 1
    unless it executes them faster than they run alone."""
    rates = lp.field_op_rates(4.0)
    peak = VALU_PEAK_TOPS * 1e12
    price = {k: peak / rates[k]["per_s"] for k in OPS_PER_STEP}
    per_step = sum(OPS_PER_STEP[k] * price[k] for k in OPS_PER_STEP)
    return {"lane_cycles_per_bootstrap": n_steps * per_step,
            "lane_cycles_per_op": {k: round(v, 3) for k, v in price.items()},
            "ops_per_step": OPS_PER_STEP, "steps": n_steps,
            "rates_gops": {k: round(v["per_s"] / 1e9, 2) for k, v in rates.items()},
            "u32_rate_vs_peak": round(rates["u32_add"]["per_s"] / peak, 4)}


def _query_parts(ct, l, N):
    return ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:]


def cpu_baseline(runs):
    """The oracle as it stands on the GPU run's own work: its key (the
    oracle's KeyGen from the same seed, equal to the library's bit for bit)
    and its very ciphertexts, checked equal before timing.  Each run is one
    whole query (the headline 16-bit 16-box query and the 8-bit one-box
    query), OpenMP over the host's threads; its output is compared with the
    GPU's bit for bit.  runs: (name, seed, q, bits, cts, is_signed,
    gpu_out)."""
    import oracle as O
    out = {"kind": "oracle", "unit": "bootstraps/s", "queries": {}}
    threads = 1
    for name, seed, q, bits, cts, signed, gpu_out in runs:
        okeys = O.keygen(seed)
        same_inputs = bool(np.array_equal(O.encrypt_bits(okeys, bits, seed=seed), cts))
        octx = O.Ctx(okeys)
        l, N, m = q.l, q.n_boxes, q.m
        t0 = time.perf_counter()
        res = octx.bbox_query(l, N, m, signed, *_query_parts(cts, l, N))
        dt = time.perf_counter() - t0
        n_br = O.bbox_counts(l, N, m)[0]
        out["queries"][name] = {"bootstraps": int(n_br), "query_s": round(dt, 3),
                                "bootstraps_per_s": round(n_br / dt, 2), "same_inputs_as_gpu": same_inputs,
                                "equal_to_gpu": bool(np.array_equal(res, gpu_out))}
        print(f"bench: oracle {name} query {dt:.1f} s", file=sys.stderr, flush=True)
        if name == "bbox16x16":
            _, threads = octx.gate_batch("NAND", cts[:2], cts[2:4])
            # one thread: the oracle's single-gate entry on 8 XNOR gates of the same inputs
            t0 = time.perf_counter()
            for k in range(8):
                octx.gate("XNOR", cts[k], cts[k + 8])
            dt1 = time.perf_counter() - t0
            out["single_core"] = {"value": round(8 / dt1, 2), "unit": "bootstraps/s",
                                  "sample": f"8 XNOR gates on one thread, {dt1:.1f} s"}
    head = out["queries"]["bbox16x16"]
    out["value"] = head["bootstraps_per_s"]
    out["cores"] = int(threads)
    out["sample"] = ("the whole 16-bit 16-box query (4112 bootstraps) and the 8-bit one-box query (107), on the "
                     "GPU run's own keys and ciphertexts; value from the 16-box query")
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    out["host_cpus"] = os.cpu_count()
    out["cpu_model"] = model
    return out


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
            # SIMDs holding a rotation's waves (the split: 2 CUs x 4; two
            # per CU: half of that)
            per = {6: 8, 7: 4}.get(r["shape"], r["shape"])
            busy += r["ms"] * min(r["jobs"] * per, 1024) / 1024
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


def serve_bench(requests_per_rate: int, tick_cap: int = 0, seed: int = 5, tuned: bool = False):
    """Serving: every request brings a fresh client key, generated before its
    phase starts (KeyGen is the client's work) and submitted as the
    serialized PK blob the client uploads, which the server deserializes,
    uploads and converts to the NTT domain inside the request's latency.
    Queries have 16- or 32-bit signed coordinates (50/50), 1..256 boxes
    (log-uniform) and 32-bit payloads.  A burst measures the saturated rate,
    then Poisson arrivals at 0.25/0.5/0.75/0.95 of it.  tick_cap > 0 caps the
    blind rotations of a server tick (-1: sized from the timed table); p50
    is also given for requests of at most 16 boxes and for larger ones.
    Every result is checked against the plaintext predicate."""
    import math
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    rng = np.random.default_rng(seed)
    if not tuned:
        # launch shapes are per device, not per key: tune once with one key
        lp.autotune(lp.DeviceKey(lp.keygen(None, 5999)[1]), buckets=TUNE_BUCKETS, br_steps=64)

    def make_requests(base, count):
        reqs = []
        for i in range(base, base + count):
            l = 16 if rng.random() < 0.5 else 32
            nb = int(min(256, max(1, math.floor(math.exp(rng.uniform(0, math.log(257)))))))
            q = W.random_query(10000 + i, l, nb, 32, region=W.KOREA if i % 2 else W.ZERO_STRADDLE,
                               force_inside=bool(rng.random() < 0.8))
            sk, ck = lp.keygen(None, 5000 + i)   # a fresh client key per request
            blob = ck.serialize()
            del ck
            xb, yb, bb, pb = q.plain_bits()
            ct = sk.encrypt_bits(np.concatenate([xb, yb, bb, pb]), seed=20000 + i)
            reqs.append((q, sk, blob, _query_parts(ct, q.l, q.n_boxes)))
        return reqs

    def run(reqs, arrivals):
        srv = lp.Server(200 << 30, max_tick_rotations="auto" if tick_cap < 0 else tick_cap)
        t0 = time.perf_counter()
        tickets = []
        for (q, sk, blob, parts), at in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit_blob(blob, q.l, q.n_boxes, q.m, True, *parts))
        lats, ok = [], True
        for (q, sk, blob, parts), t in zip(reqs, tickets):
            st, out, lat = srv.poll(t)
            ok &= st == 0
            if st == 0:
                d, _ = sk.decrypt_bits(out)
                ok &= W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True)
                lats.append(lat)
        wall = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        n_br = sum(lp.bbox_counts(q.l, q.n_boxes, q.m)[0] for q, _, _, _ in reqs)
        small = [x for x, (q, _, _, _) in zip(lats, reqs) if q.n_boxes <= 16]
        large = [x for x, (q, _, _, _) in zip(lats, reqs) if q.n_boxes > 16]
        p50 = lambda v: round(float(np.percentile(v, 50)) * 1e3, 1) if v else None
        return {"queries_per_s": round(len(reqs) / wall, 3), "bootstraps_per_s": round(n_br / wall, 1),
                "p50_ms": p50(lats), "p99_ms": round(float(np.percentile(lats, 99)) * 1e3, 1) if lats else None,
                "p99_samples": len(lats), "p50_ms_upto16_boxes": p50(small), "p50_ms_over16_boxes": p50(large),
                "requests": len(reqs), "ticks": stats["ticks"], "widest_tick": stats["widest_tick"],
                "correct": bool(ok)}

    t_start = time.perf_counter()
    burst = make_requests(0, requests_per_rate)
    sat = run(burst, [0.0] * len(burst))
    del burst
    print(f"serve: burst done, {sat['queries_per_s']} queries/s", file=sys.stderr, flush=True)
    res = {"metric": "serving: p50/p99 latency and queries/s under Poisson arrivals on 1 MI355X",
           "workload": "requests with a fresh client key each (serialized PK uploaded per request), 16- or 32-bit "
                       "signed coordinates, 1..256 boxes log-uniform, 32-bit payloads",
           "requests_per_rate": requests_per_rate, "keys": "fresh per request", "tick_cap": tick_cap,
           "saturated": sat, "rates": []}
    for k, f in enumerate((0.25, 0.5, 0.75, 0.95)):
        reqs = make_requests(1000 * (k + 1), requests_per_rate)
        lam = f * sat["queries_per_s"]
        arr = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
        r = run(reqs, list(arr))
        del reqs
        print(f"serve: rate {f} done, p50 {r['p50_ms']} ms", file=sys.stderr, flush=True)
        r["offered_fraction"] = f
        r["offered_queries_per_s"] = round(lam, 3)
        res["rates"].append(r)
    res["correct"] = bool(sat["correct"] and all(r["correct"] for r in res["rates"]))
    res["seconds"] = round(time.perf_counter() - t_start, 1)
    return res


def clients_bench(n_clients: int, steps: int, warmup: int, seed: int = 4, tuned: bool = False):
    """Many clients at once, each with its own keys: the first half use 32-bit
    floor(deg * 1e6) signed coordinates, the second half 16-bit 9.7 ones; box
    counts uniform in 1..64; 32-bit payloads; the Korea-like region, the
    zero-straddling one for odd clients.  All queries run as one fused program:
    level L of every query is one blind-rotation and one key-switch launch,
    each replayed from its hipGraph.  The program is compiled and its graphs
    captured before timing (lp_eval_bbox_prepare); with warmup = 0 a quarter
    second of batched gates brings the clocks up instead of a whole untimed
    batch.  Every result is checked against the plaintext predicate."""
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    if not tuned:
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
        items.append((L, N, q.m, True, *[lp.to_device(a) for a in _query_parts(ct, L, N)]))
        sks.append(sk)
        qs.append(q)
        br, ks, _ = lp.bbox_counts(L, N, q.m)
        n_br += br
        n_ks += ks
        if (c + 1) % 32 == 0:
            print(f"clients: {c + 1} keys and queries on the device", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    lp.eval_bbox_prepare(keys, items)
    prep = time.perf_counter() - t1
    setup = time.perf_counter() - t0
    outs = [torch.empty((q.m, keys[0].params.n + 1), dtype=torch.int32, device="cuda") for q in qs]
    for _ in range(warmup):
        outs = lp.eval_bbox_batch(keys, items, outs)
    if warmup == 0:
        a = items[0][6][:min(4096, items[0][6].shape[0])]   # the first client's bound ciphertexts
        t_w = time.perf_counter()
        while time.perf_counter() - t_w < 0.25:
            lp.bootstrap_batch(keys[0], "NAND", a, a)
            torch.cuda.synchronize()
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
    return {"metric": "fused queries of many clients with their own keys on 1 MI355X",
            "workload": f"{n_clients} clients with their own keys; half 32-bit, half 16-bit signed coordinates; "
                        "1..64 boxes uniform; 32-bit payloads; fused per depth level from hipGraphs",
            "clients": n_clients, "bootstraps": n_br, "keyswitches": n_ks,
            "levels": max(lp.bbox_counts(q.l, q.n_boxes, q.m)[2] for q in qs),
            "device_key_gb": round(sum(k.bytes for k in keys) / 1e9, 2),
            "seconds_per_batch": round(wall, 3), "bootstraps_per_s": round(n_br / wall, 1),
            "queries_per_s": round(n_clients / wall, 3), "steps": steps, "warmup": warmup,
            "setup_s": round(setup, 1), "prepare_s": round(prep, 2), "correct_vs_predicate": bool(ok)}


FIG4A_S = {8: 3.256, 16: 6.139, 24: 8.764, 32: 11.670}  # seconds, Fig. 4a
TABLE2_S = {"lambda128": {13: 4.88, 16: 5.67}, "lambda80": {13: 4.36, 16: 5.12}}  # seconds, Table 2


def shape_rows(shapes, reps: int = 3, seed: int = 6, tuned: bool = False):
    """One query at a time per shape (kind, parameter set, l, N, m, paper
    seconds or None), each with its set's own key, timed over reps after one
    untimed run, checked against the plaintext predicate.  kind "table2" takes
    the nine city boxes and services printed in Table 1 and a point in Seoul;
    the other kinds take synthetic tilings."""
    import torch
    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    torch.cuda.set_device(0)
    keys = {}
    for name, params in (("lambda128", None), ("lambda80", lp.params_lambda80())):
        sk, ck = lp.keygen(params, seed)
        keys[name] = (sk, lp.DeviceKey(ck))
    if not tuned:
        lp.autotune(keys["lambda128"][1], buckets=TUNE_BUCKETS, br_steps=64)
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
        parts = [lp.to_device(a) for a in _query_parts(ct, l, N)]
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
        if kind == "table2":
            row["result"] = W.from_bits(d)
        if paper_s is not None:
            row["paper_cpu_s"] = paper_s
        rows.append(row)
        print(f"shapes: {kind} {ps} l={l} N={N}: {row['ms_per_query']} ms", file=sys.stderr, flush=True)
    return rows


TABLE2_SHAPES = [("table2", ps, l, 9, 9, TABLE2_S[ps][l]) for ps in ("lambda128", "lambda80") for l in (13, 16)]


def sweep_bench(reps: int = 3, seed: int = 6):
    """The paper's experiment shapes on the GPU, 8- to 32-bit queries over the
    Korea-like region (a continent-sized one at 8 bits), one query at a time:
    Fig. 4a (N = 10 boxes, m = 9, l = 8/16/24/32), Table 2 (the nine city boxes
    and services printed in Table 1, N = m = 9, at l = 13 and 16, under both
    the lambda 128 and the lambda 80 parameter sets, for a point in Seoul),
    Fig. 4b (l = 16, N = 10, m = 1 to 64; the paper prints no values for it)
    and a sweep over N at l = 16, m = 9.  The paper's CPU times (6-core Ryzen
    5 3500X, TFHE 1.1) are listed beside the Fig. 4a and Table 2 shapes as
    context, not as a target."""
    shapes = [("fig4a", "lambda128", l, 10, 9, FIG4A_S[l]) for l in (8, 16, 24, 32)]
    shapes += TABLE2_SHAPES
    shapes += [("fig4b", "lambda128", 16, 10, m, None) for m in (1, 16, 32, 64)]
    shapes += [("boxes", "lambda128", 16, N, 9, None) for N in (1, 4, 16, 28)]
    rows = shape_rows(shapes, reps, seed)
    print(json.dumps({"metric": "paper experiment shapes: bbox query latency on 1 MI355X", "rows": rows}), flush=True)


def mfma_bench(sizes=(1, 32, 128, 1024, 4096, 16384), seed: int = 7):
    """The int8 matrix-core external product against the NTT path, per
    blind-rotation step, at equal batch sizes.  MFMA: digits, key limbs, the
    Toeplitz products and the sum of the partials for one step's key rows
    (lp_debug_external_product_mfma), averaged over repeated calls.  NTT: the
    whole CMux step inside the blind-rotation kernel the library launches at
    that size (digits, transforms, products, inverse, accumulator update),
    from the difference of rotations cut to 630 and to 126 steps over 504.
    Every MFMA output is checked against the oracle's external product on a
    sample of rows."""
    import torch
    import oracle as O
    import paper_2407_19871_amd as lp

    torch.cuda.set_device(0)
    okeys = O.keygen(seed)
    octx = O.Ctx(okeys)
    dk = lp.DeviceKey(lp.CloudKey.from_arrays(lp.params_default(), okeys.bsk, okeys.ksk))
    P = okeys.params
    step = 11
    key = lp.to_device(np.ascontiguousarray(okeys.bsk.reshape(P.n, 2 * P.l, 2, P.N)[step]))
    rng = np.random.default_rng(seed)
    rows = []
    for B in sizes:
        d_host = rng.integers(0, 2**32, size=(B, 2 * P.N), dtype=np.uint64).astype(np.uint32)
        d = lp.to_device(d_host)
        out = lp.debug_external_product_mfma(key, d)
        torch.cuda.synchronize()
        samp = np.unique(np.concatenate([[0, B - 1], rng.choice(B, min(B, 8), replace=False)]))
        got = lp.to_host(out)[samp]
        ok = all(np.array_equal(got[k], octx.external_product(step, d_host[b])) for k, b in enumerate(samp))
        reps = max(3, min(200, 20000 // B))
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            lp.debug_external_product_mfma(key, d, out=out)
        ev1.record()
        torch.cuda.synchronize()
        mfma_us = ev0.elapsed_time(ev1) * 1e3 / reps
        ct = lp.to_device(O.encrypt_bits(okeys, rng.integers(0, 2, B).astype(np.uint8), seed=seed + B))
        times = {}
        for st in (126, 630):
            lp.debug_blind_rotate(dk, ct, st)
            t0 = time.perf_counter()
            lp.debug_blind_rotate(dk, ct, st)
            times[st] = time.perf_counter() - t0
        ntt_us = (times[630] - times[126]) / 504 * 1e6
        waves = lp.tune_pick(B)["br_waves"]
        rows.append({"batch": B, "mfma_us_per_step": round(mfma_us, 2), "ntt_us_per_step": round(ntt_us, 2),
                     "ntt_kernel": SHAPE_KERNEL.get(waves, str(waves)), "mfma_over_ntt": round(mfma_us / ntt_us, 3),
                     "mfma_equal_to_oracle": bool(ok)})
        print(f"mfma: batch {B}: {mfma_us:.1f} us/step against {ntt_us:.1f} (NTT)", file=sys.stderr, flush=True)
    return {"metric": "CMux external product per blind-rotation step: int8 MFMA against the NTT path on 1 MI355X",
            "rows": rows}


def small_query(lp, torch, reps: int = 5):
    """The 8-bit unsigned coordinates vs one box query with an 8-bit payload
    (107 bootstraps in 12 levels), with its own key.  Returns the row and the
    run's inputs and output for the oracle baseline."""
    from oracle import plain
    from paper_2407_19871_amd import workloads as W
    seed = 1
    q = W.random_query_u8(seed, force_inside=True)
    sk, ck = lp.keygen(None, seed)
    dk = lp.DeviceKey(ck)
    xb, yb, bb, pb = q.plain_bits()
    bits = np.concatenate([xb, yb, bb, pb])
    ct = sk.encrypt_bits(bits, seed=seed)
    l, N, m = q.l, q.n_boxes, q.m
    parts = [lp.to_device(a) for a in _query_parts(ct, l, N)]
    out = lp.eval_bbox_query(dk, l, N, m, False, *parts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lp.eval_bbox_query(dk, l, N, m, False, *parts, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res = lp.to_host(out)
    d, _ = sk.decrypt_bits(res)
    n_br, _, levels = lp.bbox_counts(l, N, m)
    row = {"workload": "8-bit unsigned point vs 1 encrypted box, 8-bit payload", "bootstraps": n_br,
           "levels": levels, "ms_per_query": round(dt * 1e3, 2), "bootstraps_per_s": round(n_br / dt, 1),
           "correct_vs_predicate": bool(W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m,
                                                                        False))}
    return row, ("bbox8x1", seed, q, bits, ct, False, res)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true",
                    help="skip the batched-gate microbenchmark and the 8-bit one-box query")
    ap.add_argument("--no-clients", action="store_true", help="skip the 256-client fused batch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-table2", action="store_true", help="skip the Table 2 shapes")
    ap.add_argument("--quick", action="store_true",
                    help="the headline query, its roofline and the oracle only (implies the four --no-* above)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests per arrival rate of the serving run in the default line")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run device copies of this many bytes (traffic calibration)")
    ap.add_argument("--serve", type=int, default=0,
                    help="serving benchmark alone with this many requests per arrival rate (separate JSON line)")
    ap.add_argument("--tick-cap", type=int, default=0,
                    help="with --serve: blind rotations per server tick at most (0 = whole levels, "
                         "-1 = sized from the timed launch-shape table)")
    ap.add_argument("--sweep", action="store_true",
                    help="the paper's Fig. 4a / Table 2 query shapes and a box-count sweep (separate JSON line)")
    ap.add_argument("--clients", type=int, default=0,
                    help="fused queries of this many clients alone (separate JSON line)")
    ap.add_argument("--mfma", action="store_true",
                    help="the int8 matrix-core external product against the NTT path per step (separate JSON line)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing them on this device first")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the gate-bootstrap path here runs on a single MI355X "
              f"and has no multi-GPU mode (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.quick:
        args.no_micro = args.no_clients = args.no_serve = args.no_table2 = True

    if args.serve:
        print(json.dumps(serve_bench(args.serve, args.tick_cap)), flush=True)
        return
    if args.clients:
        print(json.dumps(clients_bench(args.clients, args.steps, args.warmup)), flush=True)
        return
    if args.sweep:
        sweep_bench()
        return
    if args.mfma:
        print(json.dumps(mfma_bench()), flush=True)
        return

    import torch

    import paper_2407_19871_amd as lp
    from oracle import plain
    from paper_2407_19871_amd import workloads as W

    t_main = time.perf_counter()
    torch.cuda.set_device(0)
    seed = 2
    q = W.random_query(seed, 16, 16, 32, force_inside=True)
    sk, ck = lp.keygen(None, seed)
    xb, yb, bb, pb = q.plain_bits()
    bits = np.concatenate([xb, yb, bb, pb])
    cts = sk.encrypt_bits(bits, seed=seed)
    l, N, m = q.l, q.n_boxes, q.m
    d_x, d_y, d_b, d_p = [lp.to_device(a) for a in _query_parts(cts, l, N)]
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
    prices = op_prices(lp)
    alg = prices["lane_cycles_per_bootstrap"]
    print(f"bench: op prices measured, {alg / 1e9:.3f} G lane-cycles per bootstrap", file=sys.stderr, flush=True)
    out = torch.empty((m, 631), dtype=torch.int32, device="cuda")

    def step():
        lp.eval_bbox_query(dk, l, N, m, True, d_x, d_y, d_b, d_p, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gpu_out = lp.to_host(out)
    d, _ = sk.decrypt_bits(gpu_out)
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
        return alg * jobs / (ms / 1e3) / 1e12 if ms else 0.0

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
        "op_unit": (f"32-bit VALU lane-cycles, {alg / 1e9:.3f}e9 per bootstrap: the method's field operations per "
                    "CMux step, each priced at its own rate measured in this run"),
        "op_prices": prices,
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
        # measured: rocprofv3 VALU busy cycles over the chip's SIMD cycles in the
        # query's rotation launches (from the committed profile, when taken on
        # these kernel sources)
        "valu_busy_frac_rocprof": valu.get("query_valu_busy_frac") if valu else None,
        # time-weighted share of the 1024 SIMDs holding a rotation wave (narrow
        # levels leave most of the chip idle)
        "busy_simd_frac": round(busy_simd, 4) if busy_simd is not None else None,
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
    oracle_runs = [("bbox16x16", seed, q, bits, cts, True, gpu_out)]
    tuned = not args.no_autotune
    if not args.no_micro:
        res["microbench"] = microbench(lp, torch, sk, dk)
        res["microbench"]["frac"] = {b: round(alg * v / (VALU_PEAK_TOPS * 1e12), 4)
                                     for b, v in res["microbench"]["batched_nand_bootstraps_per_s"].items()}
        big = (valu or {}).get("launches", {}).get("1x16384")
        res["microbench"]["valu_busy_frac_rocprof_16384"] = big.get("valu_busy_frac") if big else None
        res["small_query"], run1 = small_query(lp, torch)
        oracle_runs.append(run1)
    if args.copy_probe:
        src = torch.empty(args.copy_probe // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = args.copy_probe
    if not args.no_table2:
        rows = shape_rows(TABLE2_SHAPES, reps=3, tuned=tuned)
        res["table2"] = {"workload": "Table 2 shapes: the nine Table 1 city boxes and services, N = m = 9, a point "
                                     "in Seoul, l = 13 and 16, lambda 128 and lambda 80 sets; paper seconds "
                                     "(6-core CPU) are context", "rows": rows}
    if not args.no_clients:
        res["config4"] = clients_bench(256, 1, 0, tuned=tuned)
        print(f"bench: 256 clients done, {res['config4']['bootstraps_per_s']} bootstraps/s", file=sys.stderr,
              flush=True)
    if not args.no_serve:
        res["config5"] = serve_bench(args.serve_requests, 0, tuned=tuned)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(oracle_runs)
    res["run_seconds"] = round(time.perf_counter() - t_main, 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
