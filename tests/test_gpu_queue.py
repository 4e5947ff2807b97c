"""The persistent whole-product launches of a batch (dmul_ctx_tune_queue(1)):
products of mixed transform lengths, grouped in three tiers by register and
LDS need, taken by a grid of resident workgroups from a queue in device
memory.  Every result equals the
same batch with one launch per length (tolerance 0), the product alone, and
a sample the oracle; graph replays, per-product status and scratch poisoning
hold as on the per-length path."""
import os
import random
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _rand_limbs(rng, n):
    return np.array([rng.randrange(10 ** 19) for _ in range(n)], dtype=np.uint64)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2011_11524_amd as dm
    assert torch.cuda.is_available()
    return dm, torch


def _mixed(rng):
    """Operand sizes whose transform lengths cover the three tiers (sub-
    transforms of <= 2^8, 2^9..2^10 and 2^11..2^12 points, with and without
    the factor 3), several products per length with uneven shapes, and a
    square."""
    shapes = []
    for na in (1, 3, 9, 20, 41, 70, 110, 160, 230, 330, 480, 640, 950, 1400):
        for f in (1.0, 0.55, 0.2):
            nb = max(1, int(na * f))
            shapes.append((na, nb))
            shapes.append((nb, na))
    rng.shuffle(shapes)
    return shapes


def _tier(pl):
    logm = pl.log2_n
    return 0 if logm <= 8 else (1 if logm <= 10 and not (pl.factor == 3 and logm == 10) else 2)


def test_queue_matches_per_length_single_and_oracle(env):
    dm, torch = env
    _note("queued batch of mixed lengths vs per-length launches")
    rng = random.Random(9191)
    shapes = _mixed(rng)
    host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in shapes]
    host.append((host[5][0], host[5][0]))                       # a square
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    dev[-1] = (dev[5][0], dev[5][0])
    tiers = {_tier(dm.plan(len(a), len(b))) for a, b in host}
    assert tiers == {0, 1, 2}, tiers
    ctx = dm.Context(0, stream=torch.cuda.Stream())
    try:
        ctx.tune_queue(True)
        q_outs, q_st = ctx.batch(dev)
        ctx.tune_queue(False)
        p_outs, p_st = ctx.batch(dev)
        assert q_st == [0] * len(dev) and p_st == [0] * len(dev)
        for i, (qo, po) in enumerate(zip(q_outs, p_outs)):
            assert torch.equal(qo, po), f"product {i} differs between the queue and per-length launches"
        ctx.tune_queue(True)
        for i, (da, db) in enumerate(dev):
            assert torch.equal(ctx.mul(da, db), q_outs[i]), f"product {i} differs from the product alone"
    finally:
        ctx.close()
    for i in range(0, len(host), 7):
        a, b = host[i]
        np.testing.assert_array_equal(dm.to_host(q_outs[i]), oracle.mul_ntt(a, b))


def test_queue_graph_replays(env):
    """A queued batch captured in a graph: every replay (queue heads reset by
    the captured fill) equals the eager result, with other work between."""
    dm, torch = env
    _note("queued batch, graph replays")
    rng = random.Random(9292)
    shapes = _mixed(rng)[:30]
    host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in shapes]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    ctx = dm.Context(0, stream=torch.cuda.Stream())
    ctx.tune_queue(True)
    try:
        eager, st = ctx.batch(dev)
        assert st == [0] * len(dev)
        outs = [torch.zeros_like(o) for o in eager]
        for rep in range(4):
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            _, st = ctx.batch(dev, graph=True, outs=outs)
            assert st == [0] * len(dev)
            for i, (o, e) in enumerate(zip(outs, eager)):
                assert torch.equal(o, e), f"replay {rep}, product {i}"
            x = dm.to_device(_rand_limbs(rng, 300))
            np.testing.assert_array_equal(dm.to_host(ctx.mul(x, x)), oracle.mul_ntt(dm.to_host(x), dm.to_host(x)))
    finally:
        ctx.close()
    for i in (0, 11, 29):
        np.testing.assert_array_equal(dm.to_host(eager[i]), oracle.mul_ntt(*host[i]))


def test_queue_status_and_two_batches(env):
    """A bad limb in one queued product is reported for that product only,
    two queued batches before one sync keep their own statuses, and the
    queue heads serve the second batch afresh."""
    dm, torch = env
    _note("queued batches: bad limb, two batches before one sync")
    rng = random.Random(9393)
    shapes = _mixed(rng)[:24]
    host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in shapes]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    bad_h = host[7][0].copy()
    bad_h[len(bad_h) // 2] = np.uint64(10 ** 19 + 11)
    first = list(dev)
    first[7] = (dm.to_device(bad_h), dev[7][1])
    second = dev[::-1]
    ctx = dm.Context(0, stream=torch.cuda.Stream())
    ctx.tune_queue(True)
    try:
        outs1 = [torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda") for x, y in first]
        outs2 = [torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda") for x, y in second]
        st1 = ctx.batch_async(first, outs1)
        st2 = ctx.batch_async(second, outs2)
        ctx.sync()
        assert [int(s) for s in st1] == [dm.DMUL_EDIGIT if i == 7 else 0 for i in range(len(first))]
        assert [int(s) for s in st2] == [0] * len(second)
        for i, (a, b) in enumerate(host):
            want = oracle.mul_ntt(a, b)
            if i != 7:
                np.testing.assert_array_equal(dm.to_host(outs1[i]), want)
            np.testing.assert_array_equal(dm.to_host(outs2[len(host) - 1 - i]), want)
    finally:
        ctx.close()


def test_queue_poisoned_scratch(env):
    """The queued batch on a context whose workspaces and map words (the
    queue heads among them) are poisoned before every batch."""
    dm, torch = env
    _note("queued batch, poisoned scratch")
    old = os.environ.get("DMUL_POISON")
    os.environ["DMUL_POISON"] = "1"
    try:
        ctx = dm.Context(0, stream=torch.cuda.Stream())
    finally:
        if old is None:
            del os.environ["DMUL_POISON"]
        else:
            os.environ["DMUL_POISON"] = old
    ctx.tune_queue(True)
    rng = random.Random(9494)
    shapes = _mixed(rng)[:40]
    host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in shapes]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    try:
        for _ in range(2):
            outs, st = ctx.batch(dev)
            assert st == [0] * len(dev)
            for (a, b), o in zip(host, outs):
                np.testing.assert_array_equal(dm.to_host(o), oracle.mul_ntt(a, b))
    finally:
        ctx.close()
