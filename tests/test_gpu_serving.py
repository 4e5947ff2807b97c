"""Serving: every result of the continuous-batching loop equals the same
request multiplied alone (bit-exact, tolerance 0), and a sample equals the
CPU oracle.  Batches overlap on the device (two engines in flight)."""
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
    from paper_2011_11524_amd import serve
    assert torch.cuda.is_available()
    pool_h = synth.pack_digits(np.random.default_rng(77).integers(0, 10, size=60_000 * 19, dtype=np.uint8))
    pool = dm.to_device(pool_h)
    return dm, serve, torch, pool_h, pool


@pytest.mark.parametrize("realtime", [False, True])
def test_served_results_equal_alone(env, realtime):
    dm, serve, torch, pool_h, pool = env
    _note(f"serving realtime={realtime}")
    n = 400
    la, lb = synth.serving_lengths(n, seed=91, lo_exp=2.0, hi_exp=5.3)
    arrivals = synth.poisson_arrivals(n, rate_per_s=20000.0, seed=92) if realtime else np.zeros(n)
    reqs = serve.make_requests(la, lb, arrivals, len(pool_h), seed=93)
    srv = serve.Server(pool, engines=2, budget_bytes=64 << 20, max_batch=64)
    try:
        stats, results = srv.run(reqs, keep_outputs=True, realtime=realtime)
    finally:
        srv.close()
    assert stats.completed == n and len(results) == n
    s = stats.summary()
    assert s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]
    if not realtime:
        assert stats.max_overlap >= 2, "two engines should have batches in flight together"
    ctx = dm.Context(0)
    try:
        for r in reqs:
            a = pool[r.a_off: r.a_off + r.na]
            b = pool[r.b_off: r.b_off + r.nb]
            alone = ctx.mul(a.contiguous(), b.contiguous())
            assert torch.equal(alone, results[r.rid]), f"request {r.rid} differs alone vs in the mix"
    finally:
        ctx.close()
    rng = np.random.default_rng(94)
    for i in rng.choice(n, size=8, replace=False):
        r = reqs[i]
        want = oracle.mul_ntt(pool_h[r.a_off: r.a_off + r.na], pool_h[r.b_off: r.b_off + r.nb])
        np.testing.assert_array_equal(results[r.rid].cpu().numpy(), want)


def test_admission_respects_budget(env):
    dm, serve, torch, pool_h, pool = env
    _note("serving budget")
    n = 120
    la, lb = synth.serving_lengths(n, seed=95, lo_exp=3.0, hi_exp=5.0)
    reqs = serve.make_requests(la, lb, np.zeros(n), len(pool_h), seed=96)
    budget = 2 << 20
    srv = serve.Server(pool, engines=2, budget_bytes=budget, max_batch=1000)
    try:
        stats, _ = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    assert stats.completed == n
    biggest = max(serve.Server.footprint(r.na, r.nb) for r in reqs)
    assert stats.max_inflight_bytes <= 2 * max(budget, biggest)
    assert stats.batches > 2
