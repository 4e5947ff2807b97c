"""Size-class autotuner for batched products.

For every transform length N (2^L or 3 * 2^(L-2), the size classes of the
planner) with 2^min <= N <= 2^max, build a batch of products whose plans
have that length (operands of random digits), time the batch with each
candidate launch configuration, and keep the fastest:
  * the kernel path: for N <= 4096 the whole-product kernel (one workgroup
    per product) or the pass kernels (column, row and recovery passes over
    the whole device); longer lengths always take the passes;
  * on the pass kernels, the number of row groups each workgroup of the row
    pass loops over (1 = one group per workgroup, more = fewer,
    longer-lived workgroups).
Then the number of side streams over which a batch's classes run
concurrently is timed on the batched workload (4096 products, operands of
10^3..10^6 digits), and the persistent whole-product launches (one queue per
tier of lengths) against one launch per length, on that workload plus a
batch of 4096 short products (1..1200 limbs).  The table goes to
dmul_tune.txt beside the library (read by every new context): lines
"N row_iters path", "streams S" and "queue Q".

    python -m paper_2011_11524_amd.tune [--min 7] [--max 21] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

CANDIDATES = (1, 2, 4, 8)
STREAMS = (2, 4, 8, 12, 16)
SMALL_MAX_N = 4096


def size_classes(lo_log: int, hi_log: int) -> list:
    """Transform lengths 2^L and 3 * 2^e within [2^lo_log, 2^hi_log], sorted."""
    out = {1 << L for L in range(lo_log, hi_log + 1)}
    out |= {3 << e for e in range(4, hi_log) if (1 << lo_log) <= (3 << e) <= (1 << hi_log)}
    return sorted(out)


def limbs_for_class(N: int) -> int:
    """Operand limbs of the longest balanced product whose transform length
    is at most N (the planner's length grows with the operands)."""
    import paper_2011_11524_amd as dm
    lo, hi = 1, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        try:
            ok = dm.plan(mid, mid).N <= N
        except dm.DmulError:
            ok = False
        lo, hi = (mid, hi) if ok else (lo, mid - 1)
    return lo


def time_batch(ctx, pairs, outs, reps: int) -> float:
    """Seconds per submission of the batch, marshalled once (so the timing
    is the device work and the library's enqueue, not Python's)."""
    import torch
    pb = ctx.prepare_batch(pairs, outs)
    ctx.run_prepared(pb)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.run_prepared(pb)
        ctx.sync()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def main(argv=None) -> int:
    import torch

    import paper_2011_11524_amd as dm
    ap = argparse.ArgumentParser(description="size-class autotuner")
    ap.add_argument("--min", type=int, default=7)
    ap.add_argument("--max", type=int, default=21)
    ap.add_argument("--work", type=float, default=2 ** 24, help="transform points per timed batch")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(dm.LIB_PATH), "dmul_tune.txt"))
    args = ap.parse_args(argv)
    rng = np.random.default_rng(6006)
    os.environ["DMUL_TUNE_TABLE"] = ""        # the tuner's context starts from the defaults
    ctx = dm.Context(0)
    ctx.tune_queue(False)             # one launch per length while the classes are tuned
    rows = []
    for N in size_classes(args.min, args.max):
        nl = limbs_for_class(N)
        if dm.plan(nl, nl).N != N:
            continue
        count = int(max(1, min(4096, args.work // N)))
        pairs, outs = [], []
        for _ in range(count):
            a = rng.integers(0, 10 ** 19, size=nl, dtype=np.uint64)
            b = rng.integers(0, 10 ** 19, size=nl, dtype=np.uint64)
            pairs.append((dm.to_device(a), dm.to_device(b)))
            outs.append(torch.empty(2 * nl, dtype=torch.uint64, device="cuda"))
        times = {}
        if N <= SMALL_MAX_N:
            ctx.tune_path(N, 1)
            times[("whole", 0)] = time_batch(ctx, pairs, outs, args.reps)
        ctx.tune_path(N, 2)
        for it in CANDIDATES:
            ctx.tune(N, it)
            times[("passes", it)] = time_batch(ctx, pairs, outs, args.reps)
        best = min(times, key=times.get)
        ctx.tune(N, 0)
        ctx.tune_path(N, 0)
        rows.append((N, best, times))
        print(f"N={N:8d} products={count:5d} " +
              " ".join(f"{p}{'' if p == 'whole' else k}={v * 1e3:.3f}ms" for (p, k), v in times.items()) +
              f" -> {best}", flush=True)
        del pairs, outs
    # side streams, on the batched workload with the tuned classes
    for N, best, _ in rows:
        ctx.tune_path(N, 1 if best[0] == "whole" else 2)
        if best[0] == "passes":
            ctx.tune(N, best[1])
    import synth
    da, db = synth.batched_lengths(4096)
    pool = synth.OperandPool(10 ** 6, seed=4006, pool_limbs=4 * synth.limbs_for_digits(10 ** 6))
    pairs, outs = [], []
    for x, y in zip(da, db):
        a, b = pool.take(int(x)), pool.take(int(y))
        pairs.append((dm.to_device(a), dm.to_device(b)))
        outs.append(torch.empty(len(a) + len(b), dtype=torch.uint64, device="cuda"))
    ctx.tune_queue(False)
    stimes = {}
    for sn in STREAMS:
        ctx.tune_streams(sn)
        stimes[sn] = time_batch(ctx, pairs, outs, args.reps)
    streams = min(stimes, key=stimes.get)
    print("streams: " + " ".join(f"{k}={v * 1e3:.3f}ms" for k, v in stimes.items()) + f" -> {streams}",
          flush=True)
    ctx.tune_streams(streams)
    rng = np.random.default_rng(4007)
    spairs, souts = [], []
    for _ in range(4096):
        a, b = pool.take(int(rng.integers(1, 1200))), pool.take(int(rng.integers(1, 1200)))
        spairs.append((dm.to_device(a), dm.to_device(b)))
        souts.append(torch.empty(len(a) + len(b), dtype=torch.uint64, device="cuda"))
    qtimes = {}
    for q in (0, 1):
        ctx.tune_queue(bool(q))
        qtimes[q] = (time_batch(ctx, pairs, outs, args.reps), time_batch(ctx, spairs, souts, args.reps))
    queue = min(qtimes, key=lambda q: sum(qtimes[q]))
    print("queue: " + " ".join(f"{k}={v[0] * 1e3:.3f}+{v[1] * 1e3:.3f}ms" for k, v in qtimes.items()) +
          f" -> {queue}", flush=True)
    ctx.close()
    with open(args.out, "w") as f:
        f.write("# size-class table written by paper_2011_11524_amd/tune.py: "
                "N row_iters path (1 whole-product kernel, 2 pass kernels); streams S; queue Q\n")
        for N, best, times in rows:
            f.write(f"{N} {max(1, best[1])} {1 if best[0] == 'whole' else 2}\n")
        f.write(f"streams {streams}\n")
        f.write(f"queue {queue}\n")
    print(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
