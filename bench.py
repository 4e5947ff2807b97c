#!/usr/bin/env python3
"""Throughput of the gfx950 decimal multiplier.

Default workload: one exact product of two random 10^7-digit integers
(uniform digits, nonzero leading digit, seeds 2001/2002) held as base-10^19
uint64 limbs in HBM.  A step is one whole product -- digit-group split, the
forward NTTs of both operands modulo both primes, pointwise product, inverse
NTTs, CRT, carry and regrouping -- enqueued through the C ABI (dmul_ex) on
the context stream.  W untimed steps, then exactly K timed steps bracketed by
torch.cuda.synchronize(); the product is checked bit for bit against the CPU
oracle afterwards.

Printed: one JSON line with the metric (decimal digits multiplied per
second), the ALU roofline of the dominant kernel (per-kernel HIP-event
durations on the launch stream), the algorithmic HBM rate of the NTT phases,
the CPU oracle timed on this host (one thread, and every core), and the two
further workloads of the metric (skipped with --no-batched/--no-serving):
4096 batched products against one launch set per product, with p50/p99
completion latency of both, and a 100k-request Poisson serving stream with
p50/p99 latency and digits/s; each with its own parity check.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: one 32-bit VALU operation per lane
# per clock (the fp32 vector rate of 157.3 TFLOP/s counts an FMA as two
# flops and packed fp32 as two lanes).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# Word-level operation counts of the field arithmetic (32-bit VALU ops),
# from the formulas the kernels implement: a Montgomery product is six
# 32x32->64 multiply-adds (the middle partial products chained through the
# 64-bit addend, operands below 2^63) plus ten moves, subtractions with
# borrow, selects and adds (the reduction's borrow and the conditional +p);
# a modular add or subtract is a 64-bit add/sub (2), compare (1), 64-bit
# correction (2), select (2).
OPS_MODMUL = 16
OPS_MODADD = 7
OPS_DIF = 2 * OPS_MODADD + OPS_MODMUL              # x+y, (x-y mod p)*w
OPS_DIT = OPS_MODMUL + 2 * OPS_MODADD              # u = y*w, x+u, x-u
OPS_BF1 = 2 * OPS_MODADD                           # factor 1: x+y, x-y
# radix-3 butterfly of a row of 3M points, per triple: b+c, a+(b+c), a halving
# (5), a-(b+c)/2, b-c, kappa*(b-c), m+v, m-v, and the two twiddle products
OPS_R3 = 6 * OPS_MODADD + 5 + 3 * OPS_MODMUL
OPS_SPLIT = 24      # two multiply-high divisions by powers of ten per group
OPS_CRT = 120       # CRT modmul, 64x64 product, four 2-by-1 divisions
OPS_CARRY = 12      # per position: carry map, scan step, digit


def phase_work(N: int, logR: int, logC: int, factor: int, arrays_fwd: int, NP: int, na: int,
               nb: int) -> dict:
    """Algorithmic VALU operations and HBM bytes of each kernel phase of a
    length-N transform laid out as 2^logR rows of factor * 2^logC points."""
    half = N // 2
    fwd_stage = lambda logl: half * (OPS_BF1 + (logl - 1) * OPS_DIF)
    inv_stage = lambda logl: half * (OPS_BF1 + (logl - 1) * OPS_DIT)
    r3 = (N // 3) * OPS_R3 if factor == 3 else 0
    w = {}
    w["fwd_cols"] = (arrays_fwd * (fwd_stage(logR) + N * (2 * OPS_MODMUL + OPS_SPLIT)),
                     2 * 8 * (na + nb) + arrays_fwd * 8 * N)
    w["fwd_rows"] = (arrays_fwd * (fwd_stage(logC) + r3), arrays_fwd * 16 * N)
    w["inv_rows"] = (2 * (N * OPS_MODMUL + inv_stage(logC) + r3), 2 * 24 * N)
    w["inv_cols"] = (2 * (2 * N * OPS_MODMUL + inv_stage(logR)), 2 * 16 * N)
    # fwd_rows, pointwise and inv_rows in one pass: reads the A column-pass
    # arrays, writes the two product arrays
    w["rows"] = (w["fwd_rows"][0] + w["inv_rows"][0], arrays_fwd * 8 * N + 2 * 8 * N)
    w["rec_crt"] = (NP * OPS_CRT, 24 * NP)
    w["rec_apply"] = (NP * OPS_CARRY, 8 * NP + 8 * (na + nb))
    return w


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("field.hpp", "internal.hpp", "ntt_dev.hpp", "rec_dev.hpp", "ntt.hip", "carry.hip",
              "small.hip"):
        with open(os.path.join(ROOT, "paper_2011_11524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, per_launch_units: str):
    """HBM traffic measured by rocprofv3 counters for `kernel`, if the stored
    measurement was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    ent = data.get("kernels", {}).get(kernel)
    if not ent:
        return None
    return ent.get("bytes_per_launch")


# SIMDs of the MI355X (256 CUs x 4) and the clock the VALU peak assumes; a
# wave64 VALU instruction occupies its SIMD for 4 cycles (one quad-cycle).
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


def counters_for(kernel: str):
    """rocprofv3 SQ counters of `kernel` in the C2 product
    (profiles/c2_10m_counters.json), if they were taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "c2_10m_counters.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    return data.get("kernels", {}).get(kernel)


def valu_measured(kernel: str, live_s: float):
    """VALU issue of `kernel` from its counters: the fraction of SIMD cycles
    that issued a VALU instruction (SQ_ACTIVE_INST_VALU quad-cycles x 4 over
    1024 SIMDs x 2.4 GHz x the counted dispatch's duration), and the lane
    instructions per second at this run's live duration."""
    c = counters_for(kernel)
    if not c or "SQ_ACTIVE_INST_VALU" not in c:
        return None
    dur = c["ns_valu"] * 1e-9
    return {"valu_busy": round(c["SQ_ACTIVE_INST_VALU"] * 4 / (SIMDS * CLOCK_HZ * dur), 4),
            "valu_insts_per_launch": c["SQ_INSTS_VALU"],
            "lane_instr_tops": round(c["SQ_INSTS_VALU"] * 64 / live_s / 1e12, 3),
            "lds_bank_conflict_per_lds_cycle": round(c["SQ_LDS_BANK_CONFLICT"] / max(1.0, c["SQ_ACTIVE_INST_LDS"]), 3),
            "source": "profiles/c2_10m_counters.json"}


# rocprofv3 kernel names of the C2 product's phases (prefix match), and the
# calibration copy bench.py --copy-probe-mib appends
PROFILE_KERNELS = {"fwd_cols": "void dmi::k_fwd_cols<", "rows": "void dmi::k_rows_fused<",
                   "inv_cols": "void dmi::k_inv_cols<", "rec_crt": "void dmi::k_rec_crt<",
                   "rec_apply": "void dmi::k_rec_apply<", "copy": "__amd_rocclr_copyBuffer"}


def _counter_dispatches(path: str) -> dict:
    """rocprofv3 counter_collection.csv -> {dispatch: {name, ns, counter: value}}."""
    import csv
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            e = out.setdefault(int(r["Dispatch_Id"]), {
                "name": r["Kernel_Name"], "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def ingest_profiles(prof_dir: str, copy_mib: int, out_dir: str = "") -> None:
    """Reads the counter passes of one rocprofv3 session (the subdirectories
    pmc_valu, pmc_mix, pmc_fetch, pmc_write of prof_dir, each holding
    c2_counter_collection.csv) and writes c2_10m_counters.json and
    hbm_traffic.json into out_dir (default profiles/), tagged with the kernel
    sources' hash: per
    phase the median of each counter over its dispatches, the duration of
    the counted dispatches, VALU busy, and HBM bytes (FETCH_SIZE and
    WRITE_SIZE scaled by what they read for the calibration copy of
    copy_mib MiB)."""
    passes = {}
    for pas in ("valu", "mix", "fetch", "write"):
        path = os.path.join(prof_dir, "pmc_" + pas, "c2_counter_collection.csv")
        if os.path.exists(path):
            passes[pas] = _counter_dispatches(path)
    kernels, names = {}, {}
    for phase, prefix in PROFILE_KERNELS.items():
        ent = {}
        for pas, disp in passes.items():
            mine = [e for e in disp.values() if e["name"].startswith(prefix)]
            if phase == "copy":   # the calibration copy is the largest copy
                mine = sorted(mine, key=lambda e: e.get("FETCH_SIZE", 0) + e.get("WRITE_SIZE", 0)
                              + e["ns"])[-1:]
            if not mine:
                continue
            names[phase] = mine[0]["name"]
            for key in mine[0]:
                if key not in ("name", "ns"):
                    ent[key] = _median([e[key] for e in mine])
            ent["ns_" + pas] = _median([e["ns"] for e in mine])
            ent["dispatches"] = len(mine)
        if ent:
            kernels[phase] = ent
    copy = kernels.pop("copy", {})
    copy_kib = copy_mib * 1024.0
    fetch_scale = copy_kib / copy["FETCH_SIZE"] if copy.get("FETCH_SIZE") else None
    write_scale = copy_kib / copy["WRITE_SIZE"] if copy.get("WRITE_SIZE") else None
    for phase, c in kernels.items():
        if "SQ_ACTIVE_INST_VALU" in c and "ns_valu" in c:
            c["valu_busy"] = c["SQ_ACTIVE_INST_VALU"] * 4 / (SIMDS * CLOCK_HZ * c["ns_valu"] * 1e-9)
            c["valu_insts_per_wave"] = c["SQ_INSTS_VALU"] / max(1.0, c.get("SQ_WAVES", 1.0))
        if "SQ_LDS_BANK_CONFLICT" in c:
            c["lds_bank_conflict_per_lds_active"] = c["SQ_LDS_BANK_CONFLICT"] / max(1.0, c["SQ_ACTIVE_INST_LDS"])
        if fetch_scale and write_scale and "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            c["hbm_bytes"] = 1024.0 * (c["FETCH_SIZE"] * fetch_scale + c["WRITE_SIZE"] * write_scale)
    src = kernel_source_hash()
    workload = "10^7 x 10^7 digits, N = 3*2^19"
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    with open(os.path.join(out_dir, "c2_10m_counters.json"), "w") as f:
        json.dump({"source_hash": src, "workload": workload, "kernel_names": names,
                   "kernels": kernels, "copy": copy, "fetch_scale": fetch_scale,
                   "write_scale": write_scale}, f, indent=1, sort_keys=True)
        f.write("\n")
    if fetch_scale and write_scale:
        traffic = {k: {"fetch_kib_raw": c["FETCH_SIZE"], "write_kib_raw": c["WRITE_SIZE"],
                       "bytes_per_launch": c["hbm_bytes"]}
                   for k, c in kernels.items() if "hbm_bytes" in c}
        with open(os.path.join(out_dir, "hbm_traffic.json"), "w") as f:
            json.dump({"source_hash": src, "fetch_scale": fetch_scale, "write_scale": write_scale,
                       "workload": workload, "kernels": traffic,
                       "summary": "profiles/c2_10m_hbm_counters.md"}, f, indent=1)
            f.write("\n")
    for phase, c in kernels.items():
        print(phase, {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sorted(c.items())})


def cpu_baseline(a, b, budget_s: float, max_products: int):
    import oracle
    times = []
    out = None
    while len(times) < max_products and sum(times) < budget_s:
        t0 = time.perf_counter()
        out = oracle.mul_ntt(a, b)
        times.append(time.perf_counter() - t0)
    return out, times


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def _oracle_rates(jobs, budget_s: float):
    """The oracle on a list of (label, a, b, digits) jobs: single-thread in
    order until budget_s is spent, then the same products spread over every
    host core (the oracle's C code runs outside the interpreter lock).
    Returns ({label: result}, single-thread stats, all-cores stats)."""
    import concurrent.futures
    import oracle
    got, t1, d1 = {}, 0.0, 0
    for lab, a, b, d in jobs:
        if t1 >= budget_s:
            break
        t0 = time.perf_counter()
        got[lab] = oracle.mul_ntt(a, b)
        t1 += time.perf_counter() - t0
        d1 += d
    done = [j for j in jobs if j[0] in got]
    threads = max(1, min(16, len(os.sched_getaffinity(0)), len(done)))
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        par = list(ex.map(lambda j: oracle.mul_ntt(j[1], j[2]), done))
    tp = time.perf_counter() - t0
    import numpy as np
    same = all(np.array_equal(x, got[j[0]]) for x, j in zip(par, done))
    single = {"products": len(done), "digits": d1, "seconds": t1, "cores": 1,
              "digits_per_s": d1 / t1 if t1 > 0 else None}
    allc = {"products": len(done), "digits": d1, "seconds": tp, "cores": threads,
            "digits_per_s": d1 / tp if tp > 0 else None, "same_as_single_thread": bool(same)}
    return got, single, allc


def run_batched(dm, torch, steps: int, warmup: int, count: int, oracle_budget_s: float = 6.0):
    """The batched workload: `count` products, operand lengths log-uniform in
    [10^3, 10^6] digits with an aspect ratio uniform in [1, 4], uniform
    digits; one dmul_batch (one launch per phase and size class, classes
    concurrent on side streams) against one dmul_ex per product.

    Throughput from K timed repetitions of each mode.  Completion latency of
    every product -- all `count` requested at once, each complete when its
    result is -- from one more repetition of the plain and the eager
    batched modes with completion events (dmul_ctx_timing), which keep the
    batch's concurrent schedule.  Every mode writes its own outputs; each is
    compared with the plain results, and a seeded sample with the oracle."""
    import numpy as np
    import synth
    da, db = synth.batched_lengths(count)
    pool = synth.OperandPool(10 ** 6, seed=4006, pool_limbs=4 * synth.limbs_for_digits(10 ** 6))
    host, pairs, digits = [], [], 0
    for x, y in zip(da, db):
        a = pool.take(int(x))
        b = pool.take(int(y))
        host.append((a, b))
        pairs.append((dm.to_device(a), dm.to_device(b)))
        digits += int(x) + int(y)
    lens = [dm.plan(len(a), len(b)).N for a, b in host]
    new_outs = lambda: [torch.empty(len(a) + len(b), dtype=torch.uint64, device="cuda") for a, b in host]
    outs = {m: new_outs() for m in ("per_product", "batched", "batched_graph", "latency_per_product",
                                    "latency_batched", "batched_untuned", "batched_queue")}
    ctx = dm.Context(0, stream=torch.cuda.Stream())
    gctx = dm.Context(0, stream=torch.cuda.Stream())
    statuses = []

    def one_by_one(o):
        def f():
            for (ta, tb), z in zip(pairs, o):
                ctx.mul_async(ta, tb, z)
            ctx.sync()
        return f

    def batched(c, pb, graph):
        def f():
            st = c.run_prepared(pb, graph=graph)
            c.sync()
            statuses.append(list(st))
        return f

    prepared = {m: ctx.prepare_batch(pairs, outs[m]) for m in ("batched", "latency_batched")}
    prepared["batched_graph"] = gctx.prepare_batch(pairs, outs["batched_graph"])
    modes = (("per_product", one_by_one(outs["per_product"])),
             ("batched", batched(ctx, prepared["batched"], False)),
             ("batched_graph", batched(gctx, prepared["batched_graph"], True)))
    res = {"products": count, "digits": digits,
           "size_classes": {int(k): int(v) for k, v in zip(*np.unique(lens, return_counts=True))}}
    for name, fn in modes:
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms_per_batch": dt * 1e3, "digits_per_s": digits / dt}
    # completion latency in the timed schedules (concurrent class streams for
    # the batch, one stream for one launch set per product)
    ctx.timing(True)
    one_by_one(outs["latency_per_product"])()
    lat_pp = ctx.timing_read()
    batched(ctx, prepared["latency_batched"], False)()
    lat_b = ctx.timing_read()
    ctx.timing(False)
    for name, lat in (("per_product", lat_pp), ("batched", lat_b)):
        ok = len(lat) == count and min(lat) >= 0
        res[name]["p50_ms"] = _pct(lat, 50) if ok else None
        res[name]["p99_ms"] = _pct(lat, 99) if ok else None
        res[name]["max_ms"] = max(lat) if ok else None
    # the same eager batch on a context without the tuned size-class table
    old_tt = os.environ.get("DMUL_TUNE_TABLE")
    os.environ["DMUL_TUNE_TABLE"] = ""
    uctx = dm.Context(0, stream=torch.cuda.Stream())
    if old_tt is None:
        del os.environ["DMUL_TUNE_TABLE"]
    else:
        os.environ["DMUL_TUNE_TABLE"] = old_tt
    upb = uctx.prepare_batch(pairs, outs["batched_untuned"])
    ufn = batched(uctx, upb, False)
    for _ in range(warmup):
        ufn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ufn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res["batched_untuned"] = {"ms_per_batch": dt * 1e3, "digits_per_s": digits / dt,
                              "table": "none (default row loop 1, default kernel-path rule, 8 side streams)"}
    res["tuned_table_speedup"] = res["batched_untuned"]["ms_per_batch"] / res["batched"]["ms_per_batch"]
    uctx.close()
    # the same eager batch with the whole-product classes in persistent
    # queue launches (one per tier of lengths) instead of one per length
    qctx = dm.Context(0, stream=torch.cuda.Stream())
    qctx.tune_queue(True)
    qfn = batched(qctx, qctx.prepare_batch(pairs, outs["batched_queue"]), False)
    for _ in range(warmup):
        qfn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        qfn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res["batched_queue"] = {"ms_per_batch": dt * 1e3, "digits_per_s": digits / dt,
                            "whole_product_launches": "persistent, one queue per tier of lengths"}
    res["queue_vs_per_length"] = res["batched"]["ms_per_batch"] / res["batched_queue"]["ms_per_batch"]
    qctx.close()
    res["latency_mode"] = ("completion events on the launch streams: eager batch with its classes "
                           "on concurrent side streams, and one launch set per product on one stream")
    res["speedup"] = res["per_product"]["ms_per_batch"] / res["batched"]["ms_per_batch"]
    res["speedup_graph"] = res["per_product"]["ms_per_batch"] / res["batched_graph"]["ms_per_batch"]
    # parity: every mode equals the plain results; a seeded sample equals the oracle
    ref = outs["per_product"]
    mode_same = {m: all(torch.equal(x, y) for x, y in zip(ref, o)) for m, o in outs.items()
                 if m != "per_product"}
    status_ok = all(all(v == 0 for v in st) for st in statuses)
    rng = np.random.default_rng(4007)
    sample = [int(i) for i in rng.choice(count, size=min(64, count), replace=False)]
    jobs = [(i, host[i][0], host[i][1], int(da[i]) + int(db[i])) for i in sample]
    want, single, allc = _oracle_rates(jobs, oracle_budget_s)
    oracle_ok = all(np.array_equal(ref[i].cpu().numpy(), w) for i, w in want.items())
    res["parity"] = "bit-exact" if (all(mode_same.values()) and oracle_ok and status_ok and want) \
        else "MISMATCH"
    res["parity_detail"] = {"modes_equal_plain": mode_same, "statuses_ok": status_ok,
                            "oracle_sample_products": len(want), "oracle_sample_equal": oracle_ok}
    # the oracle on the checked sample (context, not a target)
    res["cpu_oracle_sample"] = single
    res["cpu_oracle_sample_all_cores"] = allc
    ctx.close()
    gctx.close()
    return res


def batched_only(dm, torch, steps: int, warmup: int, count: int) -> int:
    """The eager batch alone, submitted `steps` times after `warmup` (for a
    kernel trace of the batched workload); prints one JSON line."""
    import synth
    da, db = synth.batched_lengths(count)
    pool = synth.OperandPool(10 ** 6, seed=4006, pool_limbs=4 * synth.limbs_for_digits(10 ** 6))
    pairs, outs, digits = [], [], 0
    for x, y in zip(da, db):
        a, b = pool.take(int(x)), pool.take(int(y))
        pairs.append((dm.to_device(a), dm.to_device(b)))
        outs.append(torch.empty(len(a) + len(b), dtype=torch.uint64, device="cuda"))
        digits += int(x) + int(y)
    ctx = dm.Context(0, stream=torch.cuda.Stream())
    pb = ctx.prepare_batch(pairs, outs)
    for _ in range(warmup):
        ctx.run_prepared(pb)
        ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run_prepared(pb)
        ctx.sync()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ctx.close()
    print(json.dumps({"workload": f"{count} batched products (eager)", "ms_per_batch": dt * 1e3,
                      "digits_per_s": digits / dt, "steps": steps}), flush=True)
    return 0


def run_serving(dm, torch, count: int, seed: int = 5005, oracle_budget_s: float = 6.0):
    """The serving workload: `count` requests, each operand length
    round(10^U(2, 7)) digits, Poisson arrivals at 70% of the device's service
    rate (measured on a calibration draw served back to back), operands
    resident in HBM as slices of one random pool; continuous batching over
    two engines.  A seeded sample of requests is re-run alone and compared."""
    import numpy as np
    import synth
    from paper_2011_11524_amd import serve
    pool_limbs = 1 << 21
    pool_h = synth.pack_digits(np.random.default_rng(seed + 10).integers(0, 10, size=pool_limbs * 19,
                                                                          dtype=np.uint8))
    pool = dm.to_device(pool_h)
    budget = 8 << 30
    srv = serve.Server(pool, engines=2, budget_bytes=budget, max_batch=2048)
    try:
        ncal = min(2000, count)
        la, lb = synth.serving_lengths(ncal, seed=seed + 1)
        cal = serve.make_requests(la, lb, np.zeros(ncal), pool_limbs, seed=seed + 2)
        srv.run(cal, realtime=False)                       # warm-up: tables, workspaces
        st_cal, _ = srv.run(cal, realtime=False)
        service = st_cal.wall_s / ncal                     # seconds per request, back to back
        rate = 0.7 / service
        la, lb = synth.serving_lengths(count, seed=seed)
        arr = synth.poisson_arrivals(count, rate, seed=seed + 3)
        reqs = serve.make_requests(la, lb, arr, pool_limbs, seed=seed + 4)
        rng = np.random.default_rng(seed + 5)
        check = set(int(i) for i in rng.choice(count, size=min(200, count), replace=False))
        stats, _ = srv.run(reqs, realtime=True)
        # alone vs in the mix, on a sample: serve the sample again as part of
        # a mix (all at once) and alone, and compare
        sample = [reqs[i] for i in sorted(check)]
        _, mixed = srv.run([serve.Request(k, r.a_off, r.na, r.b_off, r.nb, 0.0)
                            for k, r in enumerate(sample)], keep_outputs=True, realtime=False)
    finally:
        srv.close()
    ctx = dm.Context(0)
    same = len(mixed) == len(sample)
    for k, r in enumerate(sample):
        alone = ctx.mul(pool[r.a_off: r.a_off + r.na].contiguous(), pool[r.b_off: r.b_off + r.nb].contiguous())
        same = same and torch.equal(alone, mixed[k])
    ctx.close()
    # the oracle on a seeded part of the sample (as many as oracle_budget_s allows)
    jobs = [(k, pool_h[r.a_off: r.a_off + r.na], pool_h[r.b_off: r.b_off + r.nb], r.digits())
            for k, r in enumerate(sample)]
    want, single, allc = _oracle_rates(jobs, oracle_budget_s)
    oracle_ok = bool(want) and all(np.array_equal(mixed[k].cpu().numpy(), w) for k, w in want.items())
    out = stats.summary()
    out.update({"service_us_per_request": service * 1e6, "arrival_rate_per_s": rate,
                "target_load": 0.7, "alone_vs_mix_sample": len(sample),
                "alone_vs_mix": "identical" if same else "DIFFERENT",
                "oracle_sample_products": len(want), "oracle_sample": "equal" if oracle_ok else "MISMATCH",
                "parity": "bit-exact" if (same and oracle_ok and not stats.failed) else "MISMATCH",
                "cpu_oracle_sample": single, "cpu_oracle_sample_all_cores": allc,
                "digits_counted": "requested decimal digits of both operands"})
    return out


def run_serving_hot(dm, torch, count: int, hot_frac: float, seed: int = 5105, min_len: int = 1 << 19):
    """Serving with operands that come back: the serving length mix, but a
    fraction `hot_frac` of the requests multiply one of 32 hot operands by a
    partner of 80..100% of its length (a resident operand reused with
    similar-sized partners, so its plan repeats).  The same requests are
    served back to back without and with the spectrum cache (cached
    transforms of returning operands); a sample of results is compared
    between the two runs."""
    import numpy as np
    import synth
    from paper_2011_11524_amd import serve
    pool_limbs = 1 << 21
    pool_h = synth.pack_digits(np.random.default_rng(seed + 10).integers(0, 10, size=pool_limbs * 19,
                                                                          dtype=np.uint8))
    pool = dm.to_device(pool_h)
    la, lb = synth.serving_lengths(count, seed=seed)
    reqs = serve.make_requests(la, lb, np.zeros(count), pool_limbs, seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    hot = [reqs[int(i)] for i in rng.choice(count, size=32, replace=False)]
    for i, r in enumerate(reqs):
        if rng.random() < hot_frac:
            h = hot[int(rng.integers(0, len(hot)))]
            nb = max(1, int(h.na * rng.uniform(0.8, 1.0)))
            b_off = int(rng.integers(0, pool_limbs - nb + 1))
            reqs[i] = serve.Request(r.rid, h.a_off, h.na, b_off, nb, 0.0)
    sample = [int(i) for i in rng.choice(count, size=min(100, count), replace=False)]
    res = {}
    for name, cache in (("no_cache", 0), ("spectrum_cache", 4 << 30)):
        srv = serve.Server(pool, engines=2, budget_bytes=8 << 30, max_batch=2048,
                           spectrum_cache_bytes=cache, spectrum_min_len=min_len)
        try:
            srv.run(reqs[: min(500, count)], realtime=False)          # warm-up
            st, _ = srv.run(reqs, realtime=False)
            _, outs = srv.run([reqs[i] for i in sample], keep_outputs=True, realtime=False)
        finally:
            srv.close()
        s = st.summary()
        res[name] = {"wall_s": s["wall_s"], "digits_per_s": s["digits_per_s"],
                     "spectrum_hits": s["spectrum_hits"], "spectra_made": s["spectra_made"],
                     "_outs": outs}
    same = all(torch.equal(res["no_cache"]["_outs"][k], res["spectrum_cache"]["_outs"][k])
               for k in res["no_cache"]["_outs"])
    for v in res.values():
        v.pop("_outs")
    res.update({"requests": count, "hot_fraction": hot_frac, "hot_operands": len(hot),
                "spectrum_min_len": min_len,
                "speedup": res["no_cache"]["wall_s"] / res["spectrum_cache"]["wall_s"],
                "cached_vs_plain": "identical" if same else "DIFFERENT"})
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--digits", type=int, default=10 ** 7, help="digits of each operand")
    ap.add_argument("--digits-b", type=int, default=0,
                    help="digits of the second operand (default: --digits); e.g. the unbalanced "
                         "4*10^7 x 2*10^7 product")
    ap.add_argument("--force-k", type=int, default=0, help="digit-group size to force (13..18)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time at most")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-product batched workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="only submit the 4096-product batch (eager) --steps times, for kernel traces")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-serving", action="store_true", help="skip the 100k-request serving workload")
    ap.add_argument("--requests", type=int, default=100_000)
    ap.add_argument("--serving-hot", type=float, default=0.0,
                    help="also serve a mix where this fraction of requests reuses 32 hot operands, "
                         "without and with the spectrum cache")
    ap.add_argument("--pow2", action="store_true",
                    help="power-of-two transform length even where 3*2^e is shorter")
    ap.add_argument("--ingest-profiles", default="",
                    help="write profiles/c2_10m_counters.json and profiles/hbm_traffic.json from the "
                         "rocprofv3 counter passes under this directory (pmc_valu, pmc_mix, pmc_fetch, "
                         "pmc_write), taken with --copy-probe-mib (its size is this run's "
                         "--copy-probe-mib, default 256); no GPU is used")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent products shard across GPUs without communication; "
              "see the design notes)", file=sys.stderr)
        return 2
    if args.ingest_profiles:
        ingest_profiles(args.ingest_profiles, args.copy_probe_mib or 256)
        return 0

    import numpy as np
    import torch

    import paper_2011_11524_amd as dm
    import synth

    if not os.path.exists(dm.LIB_PATH):
        from paper_2011_11524_amd import build as libbuild
        libbuild.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.batched_only:
        return batched_only(dm, torch, args.steps, args.warmup, args.batch_count)

    D = args.digits
    DB = args.digits_b or D
    a = synth.random_operand(D, 2001)
    b = synth.random_operand(DB, 2002)
    fk = args.force_k
    pl = dm.plan(len(a), len(b), force_k=fk, pow2=args.pow2)
    ta, tb = dm.to_device(a), dm.to_device(b)
    out = torch.empty(len(a) + len(b), dtype=torch.uint64, device="cuda")
    ctx = dm.Context(0)

    for _ in range(args.warmup):
        ctx.mul_async(ta, tb, out, force_k=fk, pow2=args.pow2)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.mul_async(ta, tb, out, force_k=fk, pow2=args.pow2)
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = (D + DB) / (elapsed / args.steps)
    print(f"[bench] {args.steps} products of {D}x{DB} digits: {ms_per_step:.3f} ms each", flush=True)

    # per-kernel durations (events on the context stream), a separate pass
    ctx.profile(True)
    for _ in range(args.steps):
        ctx.mul_async(ta, tb, out, force_k=fk, pow2=args.pow2)
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    # host-inclusive rate (reported beside the value, never as it): the
    # operands start in pinned host memory, and every step copies them in,
    # multiplies, and copies the product back, all on the context's stream
    ha = torch.from_numpy(a.view(np.int64)).pin_memory()
    hb = torch.from_numpy(b.view(np.int64)).pin_memory()
    hout = torch.empty(len(a) + len(b), dtype=torch.int64).pin_memory()
    steps_h = max(3, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps_h):
        ta.view(torch.int64).copy_(ha, non_blocking=True)
        tb.view(torch.int64).copy_(hb, non_blocking=True)
        ctx.mul_async(ta, tb, out, force_k=fk, pow2=args.pow2)
        hout.copy_(out.view(torch.int64), non_blocking=True)
    ctx.sync()
    torch.cuda.synchronize()
    el_h = (time.perf_counter() - t0) / steps_h
    host_inclusive = {"ms_per_product": round(el_h * 1e3, 4), "digits_per_s": (D + DB) / el_h,
                      "bytes_over_pcie": 8 * 2 * (len(a) + len(b)),
                      "result_matches_device_copy": bool(np.array_equal(hout.numpy().view(np.uint64),
                                                                        out.cpu().numpy()))}
    NP = pl.groups_a + pl.groups_b
    work = phase_work(pl.N, pl.log2_rows, pl.log2_cols, pl.factor, 4, NP, len(a), len(b))
    phases = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_s = ms / cnt / 1e3
        ops, byt = work.get(name, (0, 0))
        phases[name] = {"avg_us": avg_s * 1e6, "launches": cnt,
                        "valu_tops": ops / avg_s / 1e12 if ops else 0.0,
                        "hbm_gbs": byt / avg_s / 1e9 if byt else 0.0}
    dominant = max(phases, key=lambda k: phases[k]["avg_us"])
    d = phases[dominant]
    ops_dom, bytes_dom = work[dominant]
    roofline = {"bound": "alu", "kernel": dominant,
                "achieved": round(d["valu_tops"], 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(d["valu_tops"] / VALU_PEAK_TOPS, 4),
                "ops_per_launch": ops_dom, "bytes_per_launch": bytes_dom,
                "traffic": traffic_for(dominant, "bytes"),
                # measured beside the op model: VALU issue from the kernel's counters
                "measured": valu_measured(dominant, d["avg_us"] * 1e-6)}
    ntt = [k for k in ("fwd_cols", "fwd_rows", "rows", "inv_rows", "inv_cols") if k in phases]
    ntt_s = sum(phases[k]["avg_us"] for k in ntt) / 1e6
    ntt_bytes = sum(work[k][1] for k in ntt)
    # the survey's plain two-pass byte model: 176 N (2 primes x (2 forward x
    # 24N + inverse 40N)), without this build's fused row pass
    plain_bytes = 176 * pl.N
    hbm = {"ntt_phases_gbs": round(ntt_bytes / ntt_s / 1e9, 1), "peak": HBM_PEAK_GBS,
           "frac": round(ntt_bytes / ntt_s / 1e9 / HBM_PEAK_GBS, 4), "ntt_bytes": ntt_bytes,
           "ntt_us": round(ntt_s * 1e6, 2),
           "bytes_model": "this build's passes (fused rows): 16(na+nb) + 8AN + 8AN + 16N + 32N",
           "plain_176N": {"bytes": plain_bytes, "gbs": round(plain_bytes / ntt_s / 1e9, 1),
                          "frac": round(plain_bytes / ntt_s / 1e9 / HBM_PEAK_GBS, 4)}}

    got = out.cpu().numpy()
    result = {
        "metric": ("decimal digits multiplied/sec (10^7x10^7)" if D == DB == 10 ** 7
                   else f"decimal digits multiplied/sec ({D}x{DB})"),
        "value": value,
        "unit": "digits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": (f"exact product of two random {D}-digit integers (base-10^19 limbs)"
                                if DB == D else
                                f"exact product of random {D}- and {DB}-digit integers (base-10^19 limbs)"),
                   "digits_a": D, "digits_b": DB, "limbs_a": len(a), "limbs_b": len(b),
                   "k": pl.k, "N": pl.N, "layout": f"{1 << pl.log2_rows}x{pl.factor << pl.log2_cols}",
                   "seeds": [2001, 2002]},
        "roofline": roofline,
        "hbm": hbm,
        "host_inclusive": host_inclusive,
        "phases": {k: {kk: round(vv, 3) if isinstance(vv, float) else vv for kk, vv in v.items()}
                   for k, v in phases.items()},
    }

    if not args.no_batched:
        print(f"[bench] batched workload: {args.batch_count} products", flush=True)
        result["batched"] = run_batched(dm, torch, max(2, args.steps // 5), 1, args.batch_count)
        print(f"[bench] batched: {json.dumps(result['batched'])}", flush=True)
    if not args.no_serving:
        print(f"[bench] serving workload: {args.requests} requests", flush=True)
        result["serving"] = run_serving(dm, torch, args.requests)
        print(f"[bench] serving: {json.dumps(result['serving'])}", flush=True)
    if args.serving_hot > 0:
        result["serving_hot"] = run_serving_hot(dm, torch, min(args.requests, 4000), args.serving_hot)
        print(f"[bench] serving_hot: {json.dumps(result['serving_hot'])}", flush=True)

    if not args.no_cpu_baseline:
        print("[bench] oracle on the host cores", flush=True)
        want, times = cpu_baseline(a, b, args.cpu_budget, 3)
        cores = 1
        result["cpu_baseline"] = {"value": (D + DB) / (sum(times) / len(times)), "unit": "digits/s",
                                  "cores": cores, "kind": "oracle",
                                  "sample": f"{len(times)} full {D}x{DB}-digit products by the "
                                            "oracle's plain two-prime NTT, single thread",
                                  "host_cores_available": len(os.sched_getaffinity(0))}
        # the same product on every host core at once, one product per thread
        import concurrent.futures
        import oracle
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        t0 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
            par = list(ex.map(lambda _: oracle.mul_ntt(a, b), range(threads)))
        tp = time.perf_counter() - t0
        result["cpu_baseline_all_cores"] = {
            "value": threads * (D + DB) / tp, "unit": "digits/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} full {D}x{DB}-digit products by the oracle, one per thread, at once",
            "same_as_single_thread": bool(all(np.array_equal(x, want) for x in par))}
        result["parity"] = "bit-exact" if np.array_equal(got, want) else "MISMATCH"
        if not np.array_equal(got, want):
            print("[bench] MISMATCH against the oracle", file=sys.stderr, flush=True)

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    ctx.close()
    print(json.dumps(result), flush=True)
    ok = all(r.get("parity", "bit-exact") == "bit-exact"
             for r in (result, result.get("batched", {}), result.get("serving", {})))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
