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
    assert stats.completed == n and not stats.failed
    assert all(serve.Server.footprint(r.na, r.nb) <= budget for r in reqs)
    # every batch fits one engine's budget; two engines hold at most two batches
    assert 0 < stats.max_batch_bytes <= budget
    assert stats.max_inflight_bytes <= 2 * budget
    assert stats.batches > 2


def _alone(dm, torch, pool, r):
    a = pool[r.a_off: r.a_off + r.na].contiguous()
    b = pool[r.b_off: r.b_off + r.nb].contiguous()
    return dm.mul(a, b)


def test_oversized_request_refused_alone(env):
    """A request whose footprint alone exceeds the budget is refused with
    DMUL_ENOMEM; the requests around it are served and equal their products
    alone."""
    dm, serve, torch, pool_h, pool = env
    _note("serving: oversized request")
    budget = 1 << 20
    reqs = [serve.Request(0, 10, 300, 900, 250, 0.0),
            serve.Request(1, 5000, 20000, 100, 20000, 0.0),     # ~2.5 MB workspace
            serve.Request(2, 77, 40, 3000, 600, 0.0)]
    assert serve.Server.footprint(20000, 20000) > budget
    srv = serve.Server(pool, engines=2, budget_bytes=budget, max_batch=16)
    try:
        stats, res = srv.run(reqs, keep_outputs=True, realtime=False)
    finally:
        srv.close()
    assert stats.failed == {1: dm.DMUL_ENOMEM}
    assert sorted(res) == [0, 2] and stats.completed == 3
    for r in (reqs[0], reqs[2]):
        assert torch.equal(res[r.rid], _alone(dm, torch, pool, r))


def test_bad_limb_request_isolated(env):
    """A request with a limb >= 10^19 fails with DMUL_EDIGIT; the rest of its
    batch and the loop go on."""
    dm, serve, torch, pool_h, pool = env
    _note("serving: bad limb in one request")
    bad_h = pool_h.copy()
    bad_h[20000] = np.uint64(10 ** 19 + 3)
    bad = dm.to_device(bad_h)
    reqs = [serve.Request(i, 100 * i, 50 + 7 * i, 30000 + 11 * i, 90, 0.0) for i in range(12)]
    reqs[5] = serve.Request(5, 19990, 40, 100, 30, 0.0)           # reads limb 20000
    srv = serve.Server(bad, engines=2, budget_bytes=64 << 20, max_batch=64)
    try:
        stats, res = srv.run(reqs, keep_outputs=True, realtime=False)
    finally:
        srv.close()
    assert stats.failed == {5: dm.DMUL_EDIGIT}
    assert stats.completed == 12 and len(res) == 11
    for r in reqs:
        if r.rid != 5:
            assert torch.equal(res[r.rid], _alone(dm, torch, bad, r))


def test_refused_batch_retried_alone(env):
    """When the library refuses a batch's workspace (its context budget
    holds one product of these, the engine admits several), every request of
    the batch is run again alone and served correctly."""
    dm, serve, torch, pool_h, pool = env
    _note("serving: batch refused by the library budget, requests retried alone")
    n, na, nb = 10, 700, 650
    ws = dm.workspace_bytes(na, nb)
    reqs = [serve.Request(i, 1000 * i, na, 40000 - 500 * i, nb, 0.0) for i in range(n)]
    srv = serve.Server(pool, engines=2, budget_bytes=8 * ws, max_batch=64, ctx_budget_bytes=ws)
    try:
        stats, res = srv.run(reqs, keep_outputs=True, realtime=False)
    finally:
        srv.close()
    assert not stats.failed and stats.completed == n
    assert stats.retried >= 2
    for r in reqs:
        assert torch.equal(res[r.rid], _alone(dm, torch, pool, r))
    r = reqs[3]
    want = oracle.mul_ntt(pool_h[r.a_off: r.a_off + r.na], pool_h[r.b_off: r.b_off + r.nb])
    np.testing.assert_array_equal(res[r.rid].cpu().numpy(), want)


def test_digits_counted_as_requested(env):
    dm, serve, torch, pool_h, pool = env
    _note("serving: digit accounting")
    reqs = serve.make_requests([100, 1000], [20, 57], np.zeros(2), len(pool_h), seed=3)
    srv = serve.Server(pool, engines=1, budget_bytes=64 << 20)
    try:
        stats, _ = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    assert stats.digits == 100 + 20 + 1000 + 57


def test_spectrum_cache_reuses_hot_operands(env):
    """Requests that come back to a few hot operands (and squares of them):
    the server caches their transforms and later products skip those
    passes; every result still equals the product alone, and a sample the
    oracle."""
    dm, serve, torch, pool_h, pool = env
    _note("serving with a spectrum cache")
    rng = np.random.default_rng(95)
    npool = len(pool_h)
    hot = []
    for _ in range(6):
        n = int(rng.integers(300, 3000))
        hot.append((int(rng.integers(0, npool - n)), n))
    reqs = []
    for i in range(240):
        u = rng.random()
        if u < 0.1:
            a_off, na = hot[int(rng.integers(0, len(hot)))]
            b_off, nb = a_off, na                       # a square of a hot operand
        else:
            nb = int(rng.integers(50, 3000))
            b_off = int(rng.integers(0, npool - nb))
            if u < 0.7:
                a_off, na = hot[int(rng.integers(0, len(hot)))]
            else:
                na = int(rng.integers(50, 3000))
                a_off = int(rng.integers(0, npool - na))
        reqs.append(serve.Request(i, a_off, na, b_off, nb, 0.0))
    srv = serve.Server(pool, engines=2, budget_bytes=32 << 20, max_batch=32,
                       spectrum_cache_bytes=256 << 20, spectrum_min_len=0)
    try:
        stats, res = srv.run(reqs, keep_outputs=True, realtime=False)
        torch.cuda.synchronize()
    finally:
        srv.close()
    s = stats.summary()
    assert s["requests"] == len(reqs)
    assert s["spectra_made"] > 0 and s["spectrum_hits"] > 0, s
    for r in reqs:
        a = pool[r.a_off: r.a_off + r.na]
        b = pool[r.b_off: r.b_off + r.nb]
        alone = dm.mul(a, b)
        assert torch.equal(res[r.rid], alone), f"request {r.rid} differs from the product alone"
    for r in reqs[::40]:
        a = pool_h[r.a_off: r.a_off + r.na]
        b = pool_h[r.b_off: r.b_off + r.nb]
        np.testing.assert_array_equal(dm.to_host(res[r.rid]), oracle.mul_ntt(a, b))
