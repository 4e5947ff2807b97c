"""Size-class autotuner for batched products.

For every transform length N (2^L or 3 * 2^(L-2), the size classes of the
planner) with 2^min <= N <= 2^max, build a batch of products whose plans
have that length (operands of random digits), time the batch with each
candidate launch parameter, and write the fastest choice per class to
dmul_tune.txt beside the library (read by every new context): lines
"N row_iters".  The tuned parameter is the number of row groups each
workgroup of the row pass loops over (1 = one group per workgroup, more =
fewer, longer-lived workgroups); batches without cached spectra run the
fused row pass, so that is the kernel the timings select for.

    python -m paper_2011_11524_amd.tune [--min 7] [--max 21] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

CANDIDATES = (1, 2, 4, 8)


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
    import torch
    ctx.batch_async(pairs, outs)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.batch_async(pairs, outs)
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
    ctx = dm.Context(0)
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
        best = None
        times = {}
        for it in CANDIDATES:
            ctx.tune(N, it)
            t = time_batch(ctx, pairs, outs, args.reps)
            times[it] = t
            if best is None or t < times[best]:
                best = it
        ctx.tune(N, 0)
        rows.append((N, best, times))
        print(f"N={N:8d} products={count:5d} " +
              " ".join(f"iters{k}={v * 1e3:.3f}ms" for k, v in times.items()) + f" -> {best}", flush=True)
    ctx.close()
    with open(args.out, "w") as f:
        f.write("# size-class table written by paper_2011_11524_amd/tune.py: N row_iters\n")
        for N, best, times in rows:
            f.write(f"{N} {best}\n")
    print(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
