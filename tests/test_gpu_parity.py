"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every product is compared limb by limb -- integer work, so the bar is
bit-exact -- against oracle O2 (the plain two-prime NTT), and on small
sizes also against oracle O1 (schoolbook) and CPython's integer multiply.
"""
import random
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import int_to_limbs, limbs_to_int

pytestmark = pytest.mark.gpu

P1 = 9223371564408373249
P2 = 9223371938070528001


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
    sys.stdout.flush()


def _rand_limbs(rng, n):
    return np.array([rng.randrange(10 ** 19) for _ in range(n)], dtype=np.uint64)


def _gpu_mul(dm, ctx, a, b, force_k=0, pow2=False):
    da = dm.to_device(a)
    db = da if b is a else dm.to_device(b)
    return dm.to_host(ctx.mul(da, db, force_k=force_k, pow2=pow2))


_ORACLE_CACHE = {}


def _oracle_mul(key, a, b, force_k=0):
    """oracle.mul_ntt, memoised per test case so both length families share it."""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE.clear()
        _ORACLE_CACHE[key] = oracle.mul_ntt(a, b, force_k=force_k)
    return _ORACLE_CACHE[key]


SMALL = [(1, 1), (1, 2), (2, 1), (3, 5), (7, 7), (17, 31), (64, 3), (80, 80), (81, 81), (100, 1),
         (1, 100), (255, 257), (1000, 1000), (1000, 37), (2049, 2047), (4000, 300), (5264, 5264)]


@pytest.mark.parametrize("pow2", [False, True])
@pytest.mark.parametrize("na,nb", SMALL)
def test_random_products_match_oracle(dm, ctx, na, nb, pow2):
    _note(f"random {na}x{nb} pow2={pow2}")
    rng = random.Random(na * 7919 + nb)
    a = _rand_limbs(rng, na)
    b = _rand_limbs(rng, nb)
    got = _gpu_mul(dm, ctx, a, b, pow2=pow2)
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    if na * nb <= 10 ** 6:
        np.testing.assert_array_equal(got, oracle.schoolbook(a, b))
        assert limbs_to_int(got) == limbs_to_int(a) * limbs_to_int(b)


@pytest.mark.parametrize("k", [13, 14, 15, 16, 17, 18])
def test_forced_digit_group_sizes(dm, ctx, k):
    rng = random.Random(k)
    for na, nb in [(1, 1), (5, 9), (80, 33), (300, 1200)]:
        if oracle.choose_k(na, nb, k) == 0:
            continue
        _note(f"force_k={k} {na}x{nb}")
        a = _rand_limbs(rng, na)
        b = _rand_limbs(rng, nb)
        got = _gpu_mul(dm, ctx, a, b, force_k=k)
        np.testing.assert_array_equal(got, oracle.mul_ntt(a, b, force_k=k))


def _groups(x_limbs, k, count):
    X = limbs_to_int(x_limbs)
    B = 10 ** k
    out = []
    for _ in range(count):
        X, r = divmod(X, B)
        out.append(r)
    return out


@pytest.mark.parametrize("pow2", [False, True])
@pytest.mark.parametrize("na,nb", [(1, 1), (3, 4), (40, 40), (100, 60), (400, 333), (37, 500)])
def test_convolution_residues(dm, ctx, na, nb, pow2):
    """The transform step alone: the device residues equal the cyclic
    convolution of the digit groups mod each prime.  The expected values
    come from the oracle's pinned radix-2 transform (convolution theorem) at
    the power-of-two length L >= n + m; with N >= n + m no coefficient
    wraps, so the length-N cyclic convolution is that result padded with
    zeros (for N = 3*2^e as well)."""
    _note(f"residues {na}x{nb} pow2={pow2}")
    rng = random.Random(na + 1000 * nb)
    a = _rand_limbs(rng, na)
    b = _rand_limbs(rng, nb)
    pl = dm.plan(na, nb, pow2=pow2)
    N = pl.N
    n, m = pl.groups_a, pl.groups_b
    L = 1
    while L < n + m:
        L *= 2
    x = _groups(a, pl.k, n) + [0] * (L - n)
    y = _groups(b, pl.k, m) + [0] * (L - m)
    r1, r2 = ctx.residues(dm.to_device(a), dm.to_device(b), pow2=pow2)
    for p, got in ((P1, dm.to_host(r1)), (P2, dm.to_host(r2))):
        g = oracle.generator(p)
        xi = pow(g, (p - 1) // L, p)
        fx = oracle.transform(x, p, xi)
        fy = oracle.transform(y, p, xi)
        prod = [int(u) * int(v) % p for u, v in zip(fx, fy)]
        back = oracle.transform(prod, p, pow(xi, p - 2, p))
        linv = pow(L, p - 2, p)
        want = [int(v) * linv % p for v in back][: n + m] + [0] * (N - (n + m))
        np.testing.assert_array_equal(got, np.array(want, dtype=np.uint64))


def _sizes_with_length(dm, N, seed):
    """Unequal operand sizes (na, nb) whose plan picks transform length N."""
    rng = random.Random(seed)
    for _ in range(200):
        frac = rng.uniform(0.70, 0.98)           # of the longest length N admits
        ratio = rng.uniform(0.2, 0.8)
        need = int(N * frac)
        ga = max(1, int(need * ratio))
        gb = max(1, need - ga)
        na = max(1, ga * 15 // 19)
        nb = max(1, gb * 15 // 19)
        if dm.plan(na, nb).N == N:
            return na, nb
    raise AssertionError(f"no sizes found for N={N}")


@pytest.mark.parametrize("e", list(range(4, 20)))
def test_radix3_lengths_vs_oracle(dm, ctx, e):
    """Every row layout of the transform lengths 3*2^e (rows of 3*2^logC
    points, logC = 2..10) against the oracle, and against the power-of-two
    path on the same operands."""
    N = 3 << e
    na, nb = _sizes_with_length(dm, N, e)
    pl = dm.plan(na, nb)
    assert pl.factor == 3 and pl.log2_n == e
    _note(f"radix-3 N=3*2^{e} ({pl.log2_rows}x3*2^{pl.log2_cols}) {na}x{nb}")
    rng = np.random.default_rng(7000 + e)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
    got = _gpu_mul(dm, ctx, a, b)
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))
    np.testing.assert_array_equal(_gpu_mul(dm, ctx, a, b, pow2=True), got)
    # a squared from one buffer: one operand transformed, the row pass's
    # squaring branch, at the length a*a plans to
    sq = _gpu_mul(dm, ctx, a, a)
    np.testing.assert_array_equal(sq, oracle.mul_ntt(a, a))


def _small_classes():
    """Transform lengths of the one-workgroup kernel: 2^2..2^12 and 3*2^4..3*2^10."""
    return sorted([1 << e for e in range(2, 13)] + [3 << e for e in range(4, 11)])


def _sizes_at_most(dm, N, seed):
    """Operand sizes (na, nb) whose plan picks length N, drawn near the top
    of the class (so that the longest products of the class are covered)."""
    rng = random.Random(seed)
    for _ in range(400):
        na = rng.randint(1, max(1, N * 13 // 19))
        nb = rng.randint(1, max(1, N * 13 // 19))
        try:
            if dm.plan(na, nb).N == N:
                return na, nb
        except dm.DmulError:
            pass
    for na in range(1, N):
        if dm.plan(na, na).N == N:
            return na, na
    raise AssertionError(f"no sizes for N={N}")


def test_whole_product_kernel_every_class(dm, ctx):
    """Every transform length of the one-workgroup kernel (N <= 4096):
    single products (that kernel up to N = 256, the passes beyond), and
    one batch with 8 products of every length (4 products, 4 squares), where
    every length takes the kernel; all against the oracle."""
    rng = np.random.default_rng(9100)
    pairs, want = [], []
    for N in _small_classes():
        for rep in range(4):
            na, nb = _sizes_at_most(dm, N, N + 1000 * rep)
            a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
            b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
            w = oracle.mul_ntt(a, b)
            w2 = oracle.mul_ntt(a, a)
            if rep == 0:
                _note(f"whole-product N={N} {na}x{nb}")
                np.testing.assert_array_equal(_gpu_mul(dm, ctx, a, b), w)
                np.testing.assert_array_equal(_gpu_mul(dm, ctx, a, a), w2)
            da, db = dm.to_device(a), dm.to_device(b)
            pairs += [(da, db), (da, da)]
            want += [w, w2]
    _note(f"whole-product batch of {len(pairs)}")
    outs, st = ctx.batch(pairs)
    assert st == [0] * len(pairs)
    for o, w in zip(outs, want):
        np.testing.assert_array_equal(dm.to_host(o), w)


def _mod_pm(limbs):
    """(X mod 10^19 - 1, X mod 10^19 + 1) of a limb array: since 10^19 is
    1 resp. -1 modulo these, the (alternating) limb sums decide them."""
    x = np.asarray(limbs, dtype=np.uint64)

    def total(v):
        return int(np.sum(v & np.uint64(0xFFFFFFFF))) + (int(np.sum(v >> np.uint64(32))) << 32)

    M1, M2 = 10 ** 19 - 1, 10 ** 19 + 1
    return total(x) % M1, (total(x[0::2]) - total(x[1::2])) % M2


@pytest.mark.parametrize("e", [20, 22, 23])
def test_radix3_long_rows_vs_oracle(dm, ctx, e):
    """The longest layouts of 3*2^e (2^10..2^12 rows of 3*2^10..3*2^11 points,
    the column kernels of 2^11 and 2^12 points) limb by limb against the
    oracle (whose power-of-two transform of up to 2^25 points takes tens of
    seconds on the host), plus the product's residues modulo 10^19 - 1 and
    10^19 + 1 and equality with the power-of-two path."""
    N = 3 << e
    na, nb = _sizes_with_length(dm, N, 100 + e)
    pl = dm.plan(na, nb)
    assert pl.factor == 3 and pl.log2_n == e
    _note(f"radix-3 N=3*2^{e} ({pl.log2_rows}x3*2^{pl.log2_cols}) {na}x{nb} vs oracle")
    rng = np.random.default_rng(8000 + e)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
    got = _gpu_mul(dm, ctx, a, b)
    assert int(got.max()) < 10 ** 19
    (a1, a2), (b1, b2), (z1, z2) = _mod_pm(a), _mod_pm(b), _mod_pm(got)
    assert z1 == a1 * b1 % (10 ** 19 - 1)
    assert z2 == a2 * b2 % (10 ** 19 + 1)
    np.testing.assert_array_equal(_gpu_mul(dm, ctx, a, b, pow2=True), got)
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))


def test_power_of_two_2_24_vs_oracle(dm, ctx):
    """N = 2^24 (4096 x 4096, the 2^12-point column and row kernels), chosen
    by the planner because 3*2^22 is too short: limb by limb against the
    oracle."""
    na, nb = 7_000_000, 5_600_000
    pl = dm.plan(na, nb)
    assert (pl.N, pl.factor, pl.log2_rows, pl.log2_cols) == (1 << 24, 1, 12, 12)
    _note(f"N=2^24 {na}x{nb} limbs, k={pl.k} vs oracle")
    rng = np.random.default_rng(2424)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
    got = _gpu_mul(dm, ctx, a, b)
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))


@pytest.mark.parametrize("n", [1, 2, 50, 81, 777, 5264])
def test_squaring_same_buffer(dm, ctx, n):
    _note(f"square {n}")
    rng = random.Random(n)
    a = _rand_limbs(rng, n)
    da = dm.to_device(a)
    got = dm.to_host(ctx.mul(da, da))
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, a))


@pytest.mark.parametrize("nl", [1, 2, 79, 80, 81, 7611, 7612, 716383])
def test_all_nines_limbs_bound_edges(dm, ctx, nl):
    """Operands of all 10^19-1 limbs, at the edges of the bound: the last
    size with k = 18 (80 limbs), k = 17 (7611) and k = 16 (716,383 limbs,
    13.6M digits, largest coefficient within 1e-6 of p1*p2)."""
    _note(f"nines-limbs {nl}")
    a = synth.repeated_limbs(10 ** 19 - 1, nl)
    got = _gpu_mul(dm, ctx, a, a.copy())
    np.testing.assert_array_equal(got, _nines_square_limbs(19 * nl, 2 * nl))
    assert dm.plan(nl, nl).k == oracle.choose_k(nl, nl)


def _nines_square_limbs(d, nlimbs):
    dig = np.zeros(19 * nlimbs, dtype=np.uint8)
    dig[0] = 1
    dig[d] = 8
    dig[d + 1:2 * d] = 9
    return synth.pack_digits(dig)


@pytest.mark.parametrize("d", [1530, 100_000])
def test_all_nines_closed_form(dm, ctx, d):
    _note(f"nines-closed {d}")
    a = synth.all_nines(d)
    got = _gpu_mul(dm, ctx, a, a.copy())
    np.testing.assert_array_equal(got, _nines_square_limbs(d, 2 * len(a)))


def test_c1_100k_digits_vs_schoolbook(dm, ctx):
    _note("C1 100k x 100k")
    a = synth.random_operand(100_000, 1001)
    b = synth.random_operand(100_000, 1002)
    got = _gpu_mul(dm, ctx, a, b)
    np.testing.assert_array_equal(got, oracle.schoolbook(a, b))


@pytest.mark.parametrize("pow2", [False, True])
def test_c2_10m_digits_vs_oracle(dm, ctx, pow2):
    _note(f"C2 10^7 x 10^7 random pow2={pow2}")
    a = synth.random_operand(10 ** 7, 2001)
    b = synth.random_operand(10 ** 7, 2002)
    assert dm.plan(len(a), len(b), pow2=pow2).N == (1 << 21 if pow2 else 3 << 19)
    got = _gpu_mul(dm, ctx, a, b, pow2=pow2)
    np.testing.assert_array_equal(got, _oracle_mul("c2", a, b))


def test_c2_all_nines_closed_form(dm, ctx):
    _note("C2 10^7 all nines")
    d = 10 ** 7
    a = synth.all_nines(d)
    got = _gpu_mul(dm, ctx, a, a.copy())
    np.testing.assert_array_equal(got, _nines_square_limbs(d, 2 * len(a)))


@pytest.mark.parametrize("force_k,pow2", [(0, False), (14, False), (14, True)])
def test_c3_unbalanced_vs_oracle(dm, ctx, force_k, pow2):
    """C3 at its default k (N = 2^22, square layout), and at k = 14 both as
    3*2^21 (2048 rows of 3*1024) and as the 2n x n power-of-two layout
    2^23 = 2048 x 4096."""
    _note(f"C3 4e7 x 2e7 force_k={force_k} pow2={pow2}")
    a = synth.random_operand(4 * 10 ** 7, 3001)
    b = synth.random_operand(2 * 10 ** 7, 3002)
    got = _gpu_mul(dm, ctx, a, b, force_k=force_k, pow2=pow2)
    np.testing.assert_array_equal(got, _oracle_mul(("c3", force_k), a, b, force_k=force_k))


def test_errors_and_empty(dm, ctx):
    import torch
    _note("errors")
    a = dm.to_device(np.array([10 ** 19, 5], dtype=np.uint64))
    b = dm.to_device(np.array([7], dtype=np.uint64))
    with pytest.raises(dm.DmulError) as e:
        ctx.mul(a, b)
    assert e.value.code == dm.DMUL_EDIGIT
    # the error is cleared: the next product succeeds
    ok = ctx.mul(dm.to_device(np.array([3], np.uint64)), b)
    assert dm.to_host(ok).tolist() == [21, 0]
    # overlap of out with an input
    buf = torch.zeros(8, dtype=torch.uint64, device="cuda")
    with pytest.raises(dm.DmulError) as e:
        ctx.mul_async(buf[:2], buf[2:4], buf[1:5])
    assert e.value.code == dm.DMUL_EINVAL
    # empty operand: zeros
    z = dm.mul(torch.zeros(0, dtype=torch.uint64, device="cuda"), dm.to_device(np.array([9, 9], np.uint64)))
    assert dm.to_host(z).tolist() == [0, 0]
    # forced k beyond the bound
    with pytest.raises(dm.DmulError) as e:
        ctx.mul(dm.to_device(np.ones(81, np.uint64)), dm.to_device(np.ones(81, np.uint64)), force_k=18)
    assert e.value.code == dm.DMUL_ERANGE


def test_default_context_and_host_entry(dm):
    _note("dmul() and dmul_host()")
    rng = random.Random(99)
    a = _rand_limbs(rng, 333)
    b = _rand_limbs(rng, 444)
    want = oracle.mul_ntt(a, b)
    np.testing.assert_array_equal(dm.to_host(dm.mul(dm.to_device(a), dm.to_device(b))), want)
    np.testing.assert_array_equal(dm.mul_host(a, b), want)
    np.testing.assert_array_equal(dm.mul_host(a, b, force_k=15), want)


def test_device_selection(dm):
    """Context calls leave the thread's current device alone; a context on a
    device that does not exist is refused (DMUL_EDEVICE) and nothing else
    is disturbed."""
    import torch
    _note("device selection")
    before = torch.cuda.current_device()
    with pytest.raises(dm.DmulError) as e:
        dm.Context(torch.cuda.device_count() + 7)
    assert e.value.code == dm.DMUL_EDEVICE
    assert torch.cuda.current_device() == before
    rng = random.Random(5)
    a, b = _rand_limbs(rng, 2000), _rand_limbs(rng, 1500)
    c = dm.Context(before)
    try:
        got = dm.to_host(c.mul(dm.to_device(a), dm.to_device(b)))
    finally:
        c.close()
    assert torch.cuda.current_device() == before
    np.testing.assert_array_equal(got, oracle.mul_ntt(a, b))


def test_batch_matches_single_and_oracle(dm, ctx):
    _note("batch mixed sizes")
    rng = random.Random(4242)
    sizes = [(1, 1), (5, 3), (80, 81), (700, 20), (20, 700), (1500, 1499), (3, 9000), (64, 64)]
    host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in sizes]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    outs, st = ctx.batch(dev)
    assert st == [0] * len(sizes)
    for (a, b), o, (da, db) in zip(host, outs, dev):
        want = oracle.mul_ntt(a, b)
        np.testing.assert_array_equal(dm.to_host(o), want)
        np.testing.assert_array_equal(dm.to_host(ctx.mul(da, db)), want)


def test_batch_reports_per_product_status(dm, ctx):
    _note("batch with one bad operand")
    good = dm.to_device(np.array([1, 2, 3], np.uint64))
    bad = dm.to_device(np.array([10 ** 19 + 1], np.uint64))
    outs, st = ctx.batch([(good, good), (bad, good), (good, good)])
    assert st[0] == 0 and st[1] == dm.DMUL_EDIGIT and st[2] == 0
    np.testing.assert_array_equal(dm.to_host(outs[2]), oracle.mul_ntt([1, 2, 3], [1, 2, 3]))


def test_two_batches_before_one_sync(dm, ctx):
    """Two batches enqueued before one sync report to their own status
    arrays: the bad limb of the first batch's product 1 is reported there,
    and no product of the second batch is blamed for it."""
    import torch
    _note("two batches, one sync, bad limb in the first")
    rng = random.Random(4343)
    good = [(_rand_limbs(rng, n), _rand_limbs(rng, m)) for n, m in ((3, 4), (90, 70), (600, 500))]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in good]
    bad = dm.to_device(np.array([10 ** 19 + 5, 1], np.uint64))
    first = [dev[0], (bad, dev[1][1]), dev[2]]
    second = [dev[2], dev[1], dev[0]]
    outs1 = [torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda") for x, y in first]
    outs2 = [torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda") for x, y in second]
    st1 = ctx.batch_async(first, outs1)
    st2 = ctx.batch_async(second, outs2)
    ctx.sync()
    assert list(st1) == [0, dm.DMUL_EDIGIT, 0]
    assert list(st2) == [0, 0, 0]
    for i in (0, 2):
        np.testing.assert_array_equal(dm.to_host(outs1[i]), oracle.mul_ntt(*good[i]))
    for (a, b), o in zip([good[2], good[1], good[0]], outs2):
        np.testing.assert_array_equal(dm.to_host(o), oracle.mul_ntt(a, b))
    # the words are cleared by the sync: a clean batch afterwards reports OK
    _, st3 = ctx.batch(second)
    assert st3 == [0, 0, 0]


def test_repeatable(dm, ctx):
    _note("determinism")
    a = synth.random_operand(300_000, 7)
    b = synth.random_operand(250_000, 8)
    da, db = dm.to_device(a), dm.to_device(b)
    first = dm.to_host(ctx.mul(da, db))
    for _ in range(3):
        np.testing.assert_array_equal(dm.to_host(ctx.mul(da, db)), first)
    np.testing.assert_array_equal(first, oracle.mul_ntt(a, b))


def test_batch_graph_replays_match(dm):
    """A batch captured in a HIP graph and replayed several times, with other
    work on the device in between, gives the eager result on every replay."""
    import torch
    _note("batch graph replay")
    s = torch.cuda.Stream()
    ctx = dm.Context(0, stream=s)
    try:
        rng = random.Random(777)
        sizes = [(3, 5), (80, 81), (700, 20), (1500, 1499), (64, 64), (33, 4000)]
        host = [(_rand_limbs(rng, x), _rand_limbs(rng, y)) for x, y in sizes]
        dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
        torch.cuda.synchronize()
        want = [oracle.mul_ntt(a, b) for a, b in host]
        outs = [torch.zeros(a.numel() + b.numel(), dtype=torch.uint64, device="cuda") for a, b in dev]
        for rep in range(4):
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            _, st = ctx.batch(dev, graph=True, outs=outs)
            assert st == [0] * len(sizes)
            for o, w in zip(outs, want):
                np.testing.assert_array_equal(dm.to_host(o), w)
            # eager work in between the replays
            x = dm.to_device(_rand_limbs(rng, 500))
            np.testing.assert_array_equal(dm.to_host(ctx.mul(x, x)), oracle.mul_ntt(dm.to_host(x), dm.to_host(x)))
    finally:
        ctx.close()


def test_concurrent_repeats_every_kernel_family(dm):
    """Products that cover every kernel family (one-workgroup batches,
    column passes with wavefront-owned and workgroup-owned columns, the
    1024-thread forward tile of 2048-row columns, the fused row pass at 8
    and 16 points per thread, both recovery forms) enqueued on two contexts
    with their own streams at once, four times over: every result equals
    the oracle's.  Waves of different workgroups then run out of step, which
    is where a missing barrier shows."""
    import torch
    _note("concurrent repeats")
    rng = np.random.default_rng(8080)
    sizes = [(3000, 2000, False), (60000, 45000, False), (20000, 20000, True),
             (300000, 250000, False), (1300000, 900000, True)]
    cases = []
    for na, nb, pow2 in sizes:
        a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
        b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
        cases.append((dm.to_device(a), dm.to_device(b), pow2, oracle.mul_ntt(a, b)))
    small = []
    for _ in range(16):
        a = rng.integers(0, 10 ** 19, size=int(rng.integers(100, 700)), dtype=np.uint64)
        b = rng.integers(0, 10 ** 19, size=int(rng.integers(100, 700)), dtype=np.uint64)
        small.append((dm.to_device(a), dm.to_device(b), oracle.mul_ntt(a, b)))
    ctxs = [dm.Context(0, stream=torch.cuda.Stream()) for _ in range(2)]
    try:
        for rep in range(4):
            singles, batches = [], []
            for c in ctxs:
                for da, db, pow2, want in cases:
                    o = torch.empty(da.numel() + db.numel(), dtype=torch.uint64, device="cuda")
                    c.mul_async(da, db, o, pow2=pow2)
                    singles.append((o, want))
                outs = [torch.empty(x.numel() + y.numel(), dtype=torch.uint64, device="cuda")
                        for x, y, _ in small]
                st = c.batch_async([(x, y) for x, y, _ in small], outs)
                batches.append((outs, st))
            for c in ctxs:
                c.sync()
            for o, want in singles:
                np.testing.assert_array_equal(dm.to_host(o), want, err_msg=f"rep {rep}")
            for outs, st in batches:
                assert [int(v) for v in st] == [0] * len(small)
                for o, (_, _, want) in zip(outs, small):
                    np.testing.assert_array_equal(dm.to_host(o), want, err_msg=f"rep {rep} batch")
    finally:
        for c in ctxs:
            c.close()


def test_context_budget_enomem(dm):
    """A context's workspace budget: a product needing more gets DMUL_ENOMEM
    (single product) or that status per product (batch); products within it
    still run."""
    _note("workspace budget")
    c = dm.Context(0, budget_bytes=1 << 20)
    try:
        rng = np.random.default_rng(31)
        big_a = rng.integers(0, 10 ** 19, size=30000, dtype=np.uint64)   # N = 2^16: 2 MiB workspace
        big_b = rng.integers(0, 10 ** 19, size=30000, dtype=np.uint64)
        assert dm.workspace_bytes(30000, 30000) > (1 << 20)
        with pytest.raises(dm.DmulError) as e:
            c.mul(dm.to_device(big_a), dm.to_device(big_b))
        assert e.value.code == dm.DMUL_ENOMEM
        a = rng.integers(0, 10 ** 19, size=3000, dtype=np.uint64)
        b = rng.integers(0, 10 ** 19, size=2000, dtype=np.uint64)
        assert dm.workspace_bytes(3000, 2000) <= (1 << 20)
        np.testing.assert_array_equal(dm.to_host(c.mul(dm.to_device(a), dm.to_device(b))),
                                      oracle.mul_ntt(a, b))
        outs, st = c.batch([(dm.to_device(big_a), dm.to_device(big_b))])
        assert st == [dm.DMUL_ENOMEM]
    finally:
        c.close()


def test_largest_power_of_two_length(dm, ctx):
    """The longest transform, N = 2^26 (8192 x 8192, two 3*10^8-digit
    operands at k = 15): the product's residues modulo 10^19 - 1 and
    10^19 + 1, exact at any size, and the digit range.  Not against the
    oracle: its transform of 2^26 points takes more than a minute per prime
    pass on the host, beyond a test's time limit."""
    na = nb = 15_800_000
    pl = dm.plan(na, nb)
    assert (pl.N, pl.factor, pl.log2_rows, pl.log2_cols) == (1 << 26, 1, 13, 13)
    _note(f"N=2^26 {na}x{nb} limbs, k={pl.k}")
    rng = np.random.default_rng(2626)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    b = rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)
    got = _gpu_mul(dm, ctx, a, b)
    assert int(got.max()) < 10 ** 19
    (a1, a2), (b1, b2), (z1, z2) = _mod_pm(a), _mod_pm(b), _mod_pm(got)
    assert z1 == a1 * b1 % (10 ** 19 - 1)
    assert z2 == a2 * b2 % (10 ** 19 + 1)


def _all_nines_product(na, nb):
    """Limbs of (10^(19 na) - 1) * (10^(19 nb) - 1) = 10^(19(na+nb)) -
    10^(19 na) - 10^(19 nb) + 1 for na <= nb: 1, na - 1 zeros, nb - na limbs
    10^19 - 1, one limb 10^19 - 2, na - 1 limbs 10^19 - 1."""
    a, b = min(na, nb), max(na, nb)
    nine = np.uint64(10 ** 19 - 1)
    z = np.full(a + b, nine, dtype=np.uint64)
    z[0] = 1
    z[1:a] = 0
    z[b] = np.uint64(10 ** 19 - 2)
    return z


@pytest.mark.parametrize("e,na", [(27, 30_000_000), (28, 55_000_000)])
def test_longest_two_pass_lengths(dm, ctx, e, na):
    """N = 2^27 (2^13 rows of 2^14 points) and 2^28 (2^14 x 2^14): the
    2^14-point passes read their root tables from global memory and the
    2^14-point rows run unfused.  All-nines operands (the convolution's worst
    case) limb by limb against their closed form, and random operands by
    their residues modulo 10^19 - 1 and 10^19 + 1 (the oracle's transforms of
    2^27 and 2^28 points take minutes per prime on the host)."""
    import torch
    pl = dm.plan(na, na)
    assert (pl.N, pl.factor, pl.log2_rows + pl.log2_cols) == (1 << e, 1, e)
    assert pl.log2_cols == 14 and pl.log2_rows == e - 14
    _note(f"N=2^{e} {na}x{na} limbs, k={pl.k}, all nines")
    nines = torch.full((na,), 10 ** 19 - 1, dtype=torch.uint64, device="cuda")
    got = dm.to_host(ctx.mul(nines, nines))
    np.testing.assert_array_equal(got, _all_nines_product(na, na))
    del nines, got
    _note(f"N=2^{e} {na}x{na - 1234567} limbs, random")
    rng = np.random.default_rng(2700 + e)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    b = rng.integers(0, 10 ** 19, size=na - 1234567, dtype=np.uint64)
    assert dm.plan(len(a), len(b)).N == 1 << e
    z = _gpu_mul(dm, ctx, a, b)
    assert int(z.max()) < 10 ** 19
    (a1, a2), (b1, b2), (z1, z2) = _mod_pm(a), _mod_pm(b), _mod_pm(z)
    assert z1 == a1 * b1 % (10 ** 19 - 1)
    assert z2 == a2 * b2 % (10 ** 19 + 1)


def test_tuned_paths_and_streams(dm):
    """Every kernel path a size-class table may choose (whole-product kernel
    or passes at N <= 4096, any row-loop count) and side-stream counts from
    1 to 16 give the oracle's products."""
    import torch
    _note("tuned kernel paths and side streams")
    c = dm.Context(0, stream=torch.cuda.Stream())
    try:
        rng = np.random.default_rng(5150)
        host = [(rng.integers(0, 10 ** 19, size=int(x), dtype=np.uint64),
                 rng.integers(0, 10 ** 19, size=int(y), dtype=np.uint64))
                for x, y in zip(10 ** rng.uniform(0.5, 3.6, 40), 10 ** rng.uniform(0.5, 3.6, 40))]
        want = [oracle.mul_ntt(a, b) for a, b in host]
        pairs = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
        Ns = sorted({dm.plan(len(a), len(b)).N for a, b in host})
        for path, iters, streams in ((1, 0, 1), (2, 1, 16), (2, 4, 3), (0, 8, 0)):
            for N in Ns:
                c.tune_path(N, path if (path != 1 or N <= 4096) else 2)
                c.tune(N, iters)
            c.tune_streams(streams)
            for graph in (False, True):
                outs, st = c.batch(pairs, graph=graph)
                assert st == [0] * len(pairs)
                for o, w in zip(outs, want):
                    np.testing.assert_array_equal(dm.to_host(o), w)
            np.testing.assert_array_equal(dm.to_host(c.mul(*pairs[5])), want[5])
        with pytest.raises(dm.DmulError):
            c.tune_path(8192, 1)
        with pytest.raises(dm.DmulError):
            c.tune_streams(17)
    finally:
        c.close()


@pytest.mark.parametrize("na,nb,count", [(5264, 5264, 300), (60000, 50000, 40)])
def test_lean_and_default_launches_agree(dm, ctx, na, nb, count):
    """A short product alone launches too few workgroups to fill the CUs,
    so it takes the lean configuration (4 points per thread, narrow tiles,
    512-position recovery blocks); the same length in a large batch takes
    the default one (16 points per thread, wide tiles, 1280-position blocks).
    Both give the same limbs, and a sample of them equals the oracle."""
    pl = dm.plan(na, nb)
    assert pl.N > 4096 and pl.log2_rows <= 9      # pass kernels, lean-eligible lengths
    _note(f"lean vs default launches: {count} products of {na}x{nb} limbs (N = {pl.N})")
    rng = np.random.default_rng(7000 + na)
    host = [(rng.integers(0, 10 ** 19, size=na, dtype=np.uint64),
             rng.integers(0, 10 ** 19, size=nb, dtype=np.uint64)) for _ in range(count)]
    dev = [(dm.to_device(a), dm.to_device(b)) for a, b in host]
    outs, st = ctx.batch(dev)
    assert st == [0] * count
    for (da, db), o in zip(dev, outs):
        np.testing.assert_array_equal(dm.to_host(o), dm.to_host(ctx.mul(da, db)))
    for i in (0, count - 1):
        np.testing.assert_array_equal(dm.to_host(outs[i]), oracle.mul_ntt(*host[i]))
