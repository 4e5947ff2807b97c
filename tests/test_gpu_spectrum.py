"""Cached forward transforms (dmul_spectrum_*, dmul_ex_spectrum,
dmul_batch_ex) against the CPU oracle, bit for bit.

A spectrum is the forward transform of one operand modulo both primes for
one plan (k, N); a product that takes an operand from its spectrum skips
that operand's forward passes.  Every result here is compared with oracle
O2 on the same operands, and with the plain path where both exist.
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    import torch
    import paper_2011_11524_amd as dm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dm.lib()
    return dm


@pytest.fixture(scope="module")
def ctx(dm):
    c = dm.Context(0)
    yield c
    c.close()


def _note(msg):
    print(f"[case] {msg}", flush=True)


def _limbs(rng, n):
    return rng.integers(0, 10 ** 19, size=n, dtype=np.uint64)


def _partners_same_plan(dm, na, nb, count, rng):
    """count partner lengths whose plan with na equals plan(na, nb)."""
    want = dm.plan(na, nb)
    out = [nb]
    tries = 0
    while len(out) < count and tries < 10000:
        tries += 1
        m = int(rng.integers(max(1, nb // 2), nb + nb // 2 + 2))
        p = dm.plan(na, m)
        if p.k == want.k and p.N == want.N:
            out.append(m)
    return out


# (na, nb): lengths 3*2^e and 2^e, square and 2n x n layouts.  Products
# with spectra always run the pass kernels, also at lengths where plain
# products take the one-workgroup kernel (the first pair).
SIZES = [(300, 200), (2000, 1500), (5264, 5264), (20000, 7000), (60000, 60000)]


@pytest.mark.parametrize("na,nb", SIZES)
def test_spectrum_reuse_across_partners(dm, ctx, na, nb):
    rng = np.random.default_rng(na + 7 * nb)
    a = _limbs(rng, na)
    da = dm.to_device(a)
    pl = dm.plan(na, nb)
    _note(f"spectrum {na} limbs for partners of {nb} (N={pl.N}, k={pl.k})")
    sa = ctx.spectrum(da, nb)
    assert dm.spectrum_bytes(na, nb) == 16 * pl.N
    for m in _partners_same_plan(dm, na, nb, 4, rng):
        b = _limbs(rng, m)
        got = dm.to_host(ctx.mul_spectrum(sa, dm.to_device(b)))
        np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    # the spectrum is read, never written: a second use gives the same product
    b = _limbs(rng, nb)
    first = dm.to_host(ctx.mul_spectrum(sa, dm.to_device(b)))
    again = dm.to_host(ctx.mul_spectrum(sa, dm.to_device(b)))
    np.testing.assert_array_equal(first, again)
    np.testing.assert_array_equal(first, dm.to_host(ctx.mul(da, dm.to_device(b))))
    sa.close()


@pytest.mark.parametrize("na,nb", SIZES)
def test_spectrum_times_spectrum_and_square(dm, ctx, na, nb):
    rng = np.random.default_rng(3 * na + nb)
    a = _limbs(rng, na)
    b = _limbs(rng, nb)
    da, db = dm.to_device(a), dm.to_device(b)
    _note(f"spectrum x spectrum {na}x{nb}")
    sa = ctx.spectrum(da, nb)
    sb = ctx.spectrum(db, na)
    got = dm.to_host(ctx.mul_spectrum(sa, sb=sb))
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    sq = ctx.spectrum(da, na)
    got2 = dm.to_host(ctx.mul_spectrum(sq, sb=sq))
    np.testing.assert_array_equal(got2, oracle.mul_ntt(a, a))
    for s in (sa, sb, sq):
        s.close()


def test_spectrum_plan_mismatch_and_bad_limb(dm, ctx):
    _note("spectrum errors")
    rng = np.random.default_rng(77)
    a = _limbs(rng, 1000)
    sa = ctx.spectrum(dm.to_device(a), 1000)
    # a partner so long that the plan's length differs
    with pytest.raises(dm.DmulError) as e:
        ctx.mul_spectrum(sa, dm.to_device(_limbs(rng, 100000)))
    assert e.value.code == dm.DMUL_EINVAL
    # forcing another k changes the plan as well
    with pytest.raises(dm.DmulError) as e:
        ctx.mul_spectrum(sa, dm.to_device(_limbs(rng, 1000)), force_k=14)
    assert e.value.code == dm.DMUL_EINVAL
    sa.close()
    # a limb >= 10^19 in the operand is reported at the next sync
    bad = a.copy()
    bad[17] = np.uint64(10 ** 19)
    sbad = ctx.spectrum(dm.to_device(bad), 1000)
    with pytest.raises(dm.DmulError) as e:
        ctx.sync()
    assert e.value.code == dm.DMUL_EDIGIT
    sbad.close()
    # and the context is fine afterwards
    b = _limbs(rng, 900)
    got = dm.to_host(ctx.mul(dm.to_device(a), dm.to_device(b)))
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))


def test_batch_with_spectra(dm, ctx):
    """One batch mixing plain products, products with a cached operand on
    either side, spectrum x spectrum and squares, across several lengths
    (including the one-workgroup range for the plain ones)."""
    rng = np.random.default_rng(4242)
    pairs, want, keep = [], [], []
    for na, nb in [(5, 9), (700, 300), (2000, 1500), (5264, 5264), (20000, 7000)]:
        a, b = _limbs(rng, na), _limbs(rng, nb)
        da, db = dm.to_device(a), dm.to_device(b)
        w = oracle.mul_ntt(a, b)
        pairs.append((da, db))
        want.append(w)
        if dm.plan(na, nb).N > 4096:
            sa, sb = ctx.spectrum(da, nb), ctx.spectrum(db, na)
            sq = ctx.spectrum(da, na)
            keep += [sa, sb, sq]
            pairs += [(sa, db), (da, sb), (sa, sb), (sq, sq)]
            want += [w, w, w, oracle.mul_ntt(a, a)]
    _note(f"batch with spectra, {len(pairs)} products")
    outs, st = ctx.batch(pairs)
    assert st == [0] * len(pairs)
    for o, w in zip(outs, want):
        np.testing.assert_array_equal(dm.to_host(o), w)
    for s in keep:
        s.close()


def test_spectrum_in_caller_memory(dm, ctx):
    """Transforms held in a buffer the caller allocated (a torch tensor):
    same products; a buffer too small is refused."""
    import torch
    rng = np.random.default_rng(515)
    na, nb = 3000, 2500
    a, b = _limbs(rng, na), _limbs(rng, nb)
    da, db = dm.to_device(a), dm.to_device(b)
    _note("spectrum in caller memory")
    words = dm.spectrum_bytes(na, nb) // 8
    mem = torch.empty(words, dtype=torch.uint64, device="cuda")
    sa = ctx.spectrum(da, nb, mem=mem)
    got = dm.to_host(ctx.mul_spectrum(sa, db))
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    sa.close()
    small = torch.empty(words - 1, dtype=torch.uint64, device="cuda")
    with pytest.raises(dm.DmulError) as e:
        ctx.spectrum(da, nb, mem=small)
    assert e.value.code == dm.DMUL_EINVAL


def test_graph_batch_with_a_failing_product(dm):
    """A graph batch in which one product cannot be planned (its spectrum was
    made for another partner length): every submission reports that
    product's DMUL_EINVAL and computes the others, so no replay hides it."""
    import torch
    _note("graph batch with a failing product")
    s = torch.cuda.Stream()
    ctx = dm.Context(0, stream=s)
    try:
        rng = np.random.default_rng(606)
        a, b = _limbs(rng, 3000), _limbs(rng, 2500)
        c, e = _limbs(rng, 40000), _limbs(rng, 100)
        da, db, dc, de = (dm.to_device(x) for x in (a, b, c, e))
        sa = ctx.spectrum(da, 2500)                      # for partners of 2500 limbs
        pairs = [(da, db), (sa, dc), (dc, de), (sa, db)]  # the second needs another N
        want = [oracle.mul_ntt(a, b), None, oracle.mul_ntt(c, e), oracle.mul_ntt(a, b)]
        outs = [torch.zeros(n, dtype=torch.uint64, device="cuda") for n in (5500, 43000, 40100, 5500)]
        for rep in range(3):
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            _, st = ctx.batch(pairs, graph=True, outs=outs)
            assert st == [0, dm.DMUL_EINVAL, 0, 0], (rep, st)
            for o, w in zip(outs, want):
                if w is not None:
                    np.testing.assert_array_equal(dm.to_host(o), w)
        sa.close()
    finally:
        ctx.close()
