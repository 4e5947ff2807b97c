"""Products on contexts whose scratch is poisoned (DMUL_POISON: every
workspace and carry-map word is filled with 0xff by a fill kernel before
each product or batch), so no kernel can pass by reading what the previous
product left behind.  Every kernel family, against the oracle."""
import os
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
def poisoned():
    import torch
    import paper_2011_11524_amd as dm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    old = os.environ.get("DMUL_POISON")
    os.environ["DMUL_POISON"] = "1"
    try:
        ctx = dm.Context(0, stream=torch.cuda.Stream())
    finally:
        if old is None:
            del os.environ["DMUL_POISON"]
        else:
            os.environ["DMUL_POISON"] = old
    yield dm, torch, ctx
    ctx.close()


# (digits a, digits b, pow2): the one-workgroup kernel, 2^e and 3*2^e pass
# layouts (8- and 16-point rounds, 1024-thread column tiles), the scan
# launch of the recovery (more than 2048 recovery blocks)
CASES = [(3_000, 2_000, False), (10_000, 8_000, False), (120_000, 100_000, False),
         (120_000, 100_000, True), (1_500_000, 900_000, False), (3_000_000, 2_500_000, True),
         (10_000_000, 10_000_000, False), (25_000_000, 20_000_000, False)]


@pytest.mark.parametrize("da,db,pow2", CASES)
def test_poisoned_products_vs_oracle(poisoned, da, db, pow2):
    dm, torch, ctx = poisoned
    _note(f"poisoned scratch {da}x{db} pow2={pow2}")
    a = synth.random_operand(da, 61 + da % 97)
    b = synth.random_operand(db, 62 + db % 89)
    ta, tb = dm.to_device(a), dm.to_device(b)
    got = dm.to_host(ctx.mul(ta, tb, pow2=pow2))
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    sq = dm.to_host(ctx.mul(ta, ta, pow2=pow2))
    np.testing.assert_array_equal(sq, oracle.mul_ntt(a, a))


def test_poisoned_batch_and_noalloc_vs_oracle(poisoned):
    dm, torch, ctx = poisoned
    _note("poisoned scratch: mixed batch (eager and graph) and dmul_ex_noalloc")
    rng = np.random.default_rng(606)
    lens = [(int(x), int(y)) for x, y in zip(10 ** rng.uniform(2, 5.5, 24), 10 ** rng.uniform(2, 5.5, 24))]
    host = [(synth.random_operand(x, 900 + i), synth.random_operand(y, 950 + i)) for i, (x, y) in enumerate(lens)]
    want = [oracle.mul_ntt(a, b) for a, b in host]
    pairs = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    for graph in (False, True, True):
        outs, st = ctx.batch(pairs, graph=graph)
        assert st == [0] * len(pairs)
        for o, w in zip(outs, want):
            np.testing.assert_array_equal(dm.to_host(o), w)
    for (ta, tb), w in list(zip(pairs, want))[:6]:
        out = torch.empty(ta.numel() + tb.numel(), dtype=torch.uint64, device="cuda")
        ctx.mul_noalloc_async(ta, tb, out)
        ctx.sync()
        np.testing.assert_array_equal(dm.to_host(out), w)
