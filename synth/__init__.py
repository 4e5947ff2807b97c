"""Seeded synthetic operands for the decimal multiplier.

This module is shared by the CPU oracle's tests and the GPU path's tests and
benchmark.  It holds no part of the multiplication method: it only draws
decimal digits and packs them into the I/O format, little-endian base-10^19
``uint64`` limbs (limb i holds decimal digits [19i, 19i+19) counted from the
least-significant end).

Digit recipe (the paper fixes only "numbers of n decimal digits", Section 10):
every digit is uniform in 0..9, the most significant digit is redrawn
uniformly from 1..9, all from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math

import numpy as np

LIMB_DIGITS = 19
LIMB_BASE = 10 ** 19
_POW10 = np.array([10 ** t for t in range(LIMB_DIGITS)], dtype=np.uint64)


def limbs_for_digits(d: int) -> int:
    """Number of base-10^19 limbs that hold d decimal digits."""
    return (d + LIMB_DIGITS - 1) // LIMB_DIGITS


def pack_digits(digits_le: np.ndarray) -> np.ndarray:
    """Pack little-endian decimal digits (uint8, least significant first)
    into base-10^19 limbs."""
    d = np.asarray(digits_le, dtype=np.uint8)
    nl = limbs_for_digits(len(d))
    buf = np.zeros(nl * LIMB_DIGITS, dtype=np.uint64)
    buf[: len(d)] = d
    buf = buf.reshape(nl, LIMB_DIGITS)
    out = np.zeros(nl, dtype=np.uint64)
    for t in range(LIMB_DIGITS):
        out += buf[:, t] * _POW10[t]
    return out


def random_digits(d: int, rng: np.random.Generator) -> np.ndarray:
    """d uniform decimal digits, least significant first, top digit 1..9."""
    if d <= 0:
        return np.zeros(0, dtype=np.uint8)
    dig = rng.integers(0, 10, size=d, dtype=np.uint8)
    dig[-1] = rng.integers(1, 10, dtype=np.uint8)
    return dig


def random_operand(d: int, seed: int) -> np.ndarray:
    """A d-digit random integer as base-10^19 limbs (seed-fixed)."""
    return pack_digits(random_digits(d, np.random.default_rng(seed)))


def random_operand_rng(d: int, rng: np.random.Generator) -> np.ndarray:
    return pack_digits(random_digits(d, rng))


def all_nines(d: int) -> np.ndarray:
    """10^d - 1 as base-10^19 limbs."""
    return pack_digits(np.full(d, 9, dtype=np.uint8))


def repeated_limbs(value: int, nlimbs: int) -> np.ndarray:
    """nlimbs copies of one limb value (e.g. 10^19 - 1 for an all-9s operand
    that fills every limb)."""
    return np.full(nlimbs, value, dtype=np.uint64)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def batched_lengths(count: int = 4096, seed: int = 4004, lo_exp: float = 3.0,
                    hi_exp: float = 6.0, max_ratio: float = 4.0):
    """Operand digit lengths for the batched workload.

    L1 = round(10^U(lo_exp, hi_exp)); r ~ U(1, max_ratio); L2 = max(1, round(L1/r));
    a fair coin picks which operand is the longer one."""
    rng = np.random.default_rng(seed)
    l1 = np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)
    r = rng.uniform(1.0, max_ratio, size=count)
    l2 = np.maximum(1, np.rint(l1 / r)).astype(np.int64)
    swap = rng.integers(0, 2, size=count).astype(bool)
    da = np.where(swap, l2, l1)
    db = np.where(swap, l1, l2)
    return da, db


def serving_lengths(count: int = 100_000, seed: int = 5005, lo_exp: float = 2.0,
                    hi_exp: float = 7.0):
    """Operand digit lengths for the serving workload: each operand length is
    independently round(10^U(lo_exp, hi_exp))."""
    rng = np.random.default_rng(seed)
    da = np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)
    db = np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)
    return np.maximum(da, 1), np.maximum(db, 1)


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5006) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


class OperandPool:
    """A seeded pool of random digits from which operands are cut.

    Serving draws 10^5 operands of up to 10^7 digits each; generating fresh
    random digits for all of them would take tens of gigabytes, so each
    operand is an (offset, length) slice of one random pool of limbs.  The
    top limb of a slice is re-drawn so the operand has exactly the requested
    number of significant digits."""

    def __init__(self, max_digits: int, seed: int = 5007, pool_limbs: int | None = None):
        rng = np.random.default_rng(seed)
        self.max_limbs = limbs_for_digits(max_digits)
        n = pool_limbs or 2 * self.max_limbs
        digits = rng.integers(0, 10, size=n * LIMB_DIGITS, dtype=np.uint8)
        self.limbs = pack_digits(digits)
        self.rng = np.random.default_rng(seed + 1)

    def take(self, d: int) -> np.ndarray:
        nl = limbs_for_digits(d)
        off = int(self.rng.integers(0, len(self.limbs) - nl + 1))
        x = self.limbs[off: off + nl].copy()
        top_digits = d - (nl - 1) * LIMB_DIGITS
        lo = 10 ** (top_digits - 1)
        x[-1] = self.rng.integers(lo, 10 * lo, dtype=np.uint64)
        return x


def digits_of(limbs: np.ndarray) -> int:
    """Number of significant decimal digits of a limb array (0 for zero)."""
    nz = np.flatnonzero(limbs)
    if len(nz) == 0:
        return 0
    top = int(nz[-1])
    return top * LIMB_DIGITS + len(str(int(limbs[top])))


def log_uniform(lo: float, hi: float, size: int, rng: np.random.Generator) -> np.ndarray:
    return np.rint(10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=size))
