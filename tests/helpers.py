"""Conversions between base-10^19 limb arrays and Python integers, used by
tests to compare against CPython's own integer multiply (an independent
library routine) and to build closed-form cases."""
from __future__ import annotations

import functools

import numpy as np

BASE = 10 ** 19


@functools.lru_cache(maxsize=None)
def _pow_base(e: int) -> int:
    return BASE ** e


def limbs_to_int(limbs) -> int:
    vals = [int(v) for v in np.asarray(limbs, dtype=np.uint64)]

    def rec(lo: int, hi: int) -> int:
        if hi - lo <= 32:
            acc = 0
            for v in reversed(vals[lo:hi]):
                acc = acc * BASE + v
            return acc
        mid = (lo + hi) // 2
        return rec(lo, mid) + rec(mid, hi) * _pow_base(mid - lo)

    return rec(0, len(vals)) if vals else 0


def int_to_limbs(x: int, n: int) -> np.ndarray:
    assert x >= 0
    out = np.zeros(n, dtype=np.uint64)

    def rec(v: int, lo: int, cnt: int):
        if cnt <= 32:
            for i in range(cnt):
                v, r = divmod(v, BASE)
                out[lo + i] = r
            assert v == 0 or lo + cnt == n, "value does not fit"
            return
        half = cnt // 2
        q, r = divmod(v, _pow_base(half))
        rec(r, lo, half)
        rec(q, lo + half, cnt - half)

    rec(x, 0, n)
    return out
