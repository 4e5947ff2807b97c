"""The allocation-free entry point dmul_ex_noalloc (C ABI, through ctypes):
its products equal those of dmul_ex, the entry point whose workspace the
library allocates, bit for bit, on calls in a row that reuse the static
scratch with a smaller product after a larger one; a length beyond the
static maximum is refused with DMUL_ENOMEM and a bad limb is reported."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2011_11524_amd as dm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L = dm.lib()
    ctx = dm.Context(0)
    yield dm, torch, L, ctx
    ctx.close()


def _call(L, ctx, fn, a, b, out):
    return getattr(L, fn)(ctx._h, ctypes.c_void_p(a.data_ptr()), a.numel(),
                          ctypes.c_void_p(b.data_ptr()), b.numel(), ctypes.c_void_p(out.data_ptr()), 0)


def _both(dm, torch, L, ctx, a, b):
    want = torch.empty(a.numel() + b.numel(), dtype=torch.uint64, device="cuda")
    got = torch.full_like(want, 7)
    assert _call(L, ctx, "dmul_ex", a, b, want) == 0
    assert L.dmul_sync(ctx._h) == 0
    assert _call(L, ctx, "dmul_ex_noalloc", a, b, got) == 0
    assert L.dmul_sync(ctx._h) == 0
    return got, want


def test_noalloc_matches_dmul_ex_twice(env):
    """Two calls in a row, the second smaller: the 10^7 x 10^7-digit product
    (N = 3 * 2^19, the five-launch path), then a 3 * 10^5 x 2 * 10^5-digit
    one, then a 2 * 10^4 x 1.5 * 10^4-digit one (the one-workgroup kernel),
    each equal to dmul_ex's; the last also to the oracle."""
    dm, torch, L, ctx = env
    cases = [(10 ** 7, 10 ** 7, 2001), (300_000, 200_000, 13), (20_000, 15_000, 11)]
    for da, db, seed in cases:
        _note(f"noalloc {da}x{db} digits")
        a = synth.random_operand(da, seed)
        b = synth.random_operand(db, seed + 1)
        got, want = _both(dm, torch, L, ctx, dm.to_device(a), dm.to_device(b))
        assert torch.equal(got, want), f"{da}x{db}: dmul_ex_noalloc differs from dmul_ex"
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.mul_ntt(a, b))


def test_noalloc_square_and_limits(env):
    dm, torch, L, ctx = env
    _note("noalloc square, 2^21 edge, over-limit refusal, bad limb")
    a = dm.to_device(synth.random_operand(2_000_000, 21))
    got, want = _both(dm, torch, L, ctx, a, a)
    assert torch.equal(got, want)
    # the longest static length, N = 2^21 (forced power of two)
    x = dm.to_device(synth.random_operand(9_000_000, 22))
    y = dm.to_device(synth.random_operand(8_000_000, 23))
    pl = dm.plan(x.numel(), y.numel(), pow2=True)
    assert pl.N == 1 << 21
    w1 = torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda")
    w2 = torch.empty_like(w1)
    flags = dm.flags_for(0, True)
    assert L.dmul_ex(ctx._h, ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(y.data_ptr()),
                     y.numel(), ctypes.c_void_p(w1.data_ptr()), flags) == 0
    assert L.dmul_ex_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()), x.numel(),
                             ctypes.c_void_p(y.data_ptr()), y.numel(), ctypes.c_void_p(w2.data_ptr()),
                             flags) == 0
    assert L.dmul_sync(ctx._h) == 0
    assert torch.equal(w1, w2)
    # beyond the static maximum: refused before anything is enqueued
    big = dm.to_device(synth.random_operand(16_000_000, 24))
    assert dm.plan(big.numel(), big.numel()).N > 1 << 21
    out = torch.empty(2 * big.numel(), dtype=torch.uint64, device="cuda")
    assert _call(L, ctx, "dmul_ex_noalloc", big, big, out) == dm.DMUL_ENOMEM
    assert L.dmul_sync(ctx._h) == 0
    # a limb >= 10^19 is reported by the next sync, and the next call is fine
    bad = dm.to_device(np.array([5, 10 ** 19 + 1, 3], np.uint64))
    good = dm.to_device(np.array([1, 2], np.uint64))
    o = torch.empty(5, dtype=torch.uint64, device="cuda")
    assert _call(L, ctx, "dmul_ex_noalloc", bad, good, o) == 0
    assert L.dmul_sync(ctx._h) == dm.DMUL_EDIGIT
    got, want = _both(dm, torch, L, ctx, good, good)
    assert torch.equal(got, want)
