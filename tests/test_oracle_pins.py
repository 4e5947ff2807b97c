"""Pins for the CPU oracle: each checks the oracle against something other
than itself -- values the paper prints, closed forms, library routines
(sympy, CPython integers) or brute force -- so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails here."""
import json
import os
import random

import numpy as np
import pytest
import sympy

import oracle
import synth
from helpers import int_to_limbs, limbs_to_int

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P1 = 9223371564408373249
P2 = 9223371938070528001


# --------------------------------------------------------------------------
# Section 4.2: the lambda tables (24 printed values).
# --------------------------------------------------------------------------

def test_lambda_table_matches_paper():
    with open(os.path.join(GOLDEN, "lambda_table.json")) as f:
        table = json.load(f)
    for row in table["rows"]:
        got = [oracle.lambda_digits(row["mu_bits"], 2 ** row["M_log2"], ell) for ell in (1, 2, 3, 4)]
        assert got == row["lambda"], row


# --------------------------------------------------------------------------
# Section 4.5: primes of the form c*3*2^n + 1, Miller-Rabin, FindPrimes.
# --------------------------------------------------------------------------

def test_find_primes_64_32_2():
    ps = oracle.find_primes(64, 32, 2)
    assert ps == [P1, P2]
    (p, g) = oracle.primes()
    assert p == [P1, P2]
    for q in ps:
        assert sympy.isprime(q)
        assert q < 2 ** 63
        e = sympy.multiplicity(2, q - 1)
        c3 = (q - 1) >> e
        assert e >= 32 and c3 % 3 == 0 and (c3 // 3) % 2 == 1
        assert (q - 1) % (2 ** 32) == 0


def test_primes_are_the_two_largest_of_their_form():
    # Every c*3*2^n+1 (c odd, 32 <= n <= 62) above p1 and below 2^63, other
    # than p2, must be composite.
    found = []
    for n in range(32, 63):
        step = 3 << n
        c = 1
        # first odd c with c*3*2^n + 1 > p1
        c = max(1, (P1 - 1) // step)
        if c % 2 == 0:
            c -= 1
        while c * step + 1 < 2 ** 63:
            v = c * step + 1
            if v >= P1 and sympy.isprime(v):
                found.append(v)
            c += 2
    assert sorted(set(found)) == [P1, P2]


def test_find_primes_for_n_small_word_bruteforce():
    # w = 24: enumerate the form directly and compare with FindPrimes.
    w, nmin, ell = 24, 4, 3
    pmax = 2 ** (w - 1) - 1
    cands = set()
    for n in range(nmin, w - 1):
        c = 1
        while c * 3 * 2 ** n + 1 <= pmax:
            v = c * 3 * 2 ** n + 1
            if sympy.isprime(v):
                cands.add(v)
            c += 2
    assert oracle.find_primes(w, nmin, ell) == sorted(cands)[-ell:]
    for n in (4, 7, 11):
        got = oracle.find_primes_for_n(n, pmax, 5)
        want = sorted([v for v in cands if (v - 1) % (3 * 2 ** n) == 0
                       and ((v - 1) // (3 * 2 ** n)) % 2 == 1], reverse=True)[:5]
        assert got == want


def test_miller_rabin_against_sympy():
    rng = random.Random(7)
    specials = [0, 1, 2, 3, 4, 561, 1105, 2047, 1373653, 25326001, 3215031751,
                2152302898747, 3474749660383, 341550071728321, 3825123056546413051,
                18446744073709551557, 18446744073709551615, P1, P2, P1 * 0 + 2 ** 61 - 1]
    vals = specials + [rng.getrandbits(64) | 1 for _ in range(3000)] + \
        [rng.getrandbits(32) for _ in range(2000)]
    for v in vals:
        assert oracle.is_prime(v) == sympy.isprime(v), v


def test_generators_are_smallest_primitive_roots():
    _, g = oracle.primes()
    assert g[0] == sympy.primitive_root(P1)
    assert g[1] == sympy.primitive_root(P2)
    assert sympy.n_order(g[0], P1) == P1 - 1
    assert sympy.n_order(g[1], P2) == P2 - 1


# --------------------------------------------------------------------------
# Sections 3.3 and 5: the transform against the DFT definition.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [P1, P2])
@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64])
def test_transform_is_the_dft(p, N):
    g = sympy.primitive_root(p)
    xi = pow(g, (p - 1) // N, p)
    rng = random.Random(N * 31 + p % 1000)
    x = [rng.randrange(p) for _ in range(N)]
    want = [sum(x[i] * pow(xi, i * k, p) for i in range(N)) % p for k in range(N)]
    got = [int(v) for v in oracle.transform(x, p, xi)]
    assert got == want
    # inverse: N^-1 * tau(., xi^-1) restores x (eq. idft)
    back = oracle.transform(got, p, pow(xi, p - 2, p))
    ninv = pow(N, p - 2, p)
    assert [int(v) * ninv % p for v in back] == x


def test_cyclic_convolution_definition_and_theorem():
    rng = random.Random(3)
    for n in (1, 2, 3, 5, 8, 16):
        x = [rng.randrange(1000) for _ in range(n)]
        y = [rng.randrange(1000) for _ in range(n)]
        want = [sum(x[i] * y[(k - i) % n] for i in range(n)) for k in range(n)]
        assert oracle.cyclic_convolution(x, y) == want
        if n & (n - 1) == 0:
            # convolution theorem (eq. conv_theorem) mod each prime
            for p in (P1, P2):
                xi = pow(sympy.primitive_root(p), (p - 1) // n, p)
                fx = oracle.transform(x, p, xi)
                fy = oracle.transform(y, p, xi)
                prod = [int(a) * int(b) % p for a, b in zip(fx, fy)]
                back = oracle.transform(prod, p, pow(xi, p - 2, p))
                ninv = pow(n, p - 2, p)
                assert [int(v) * ninv % p for v in back] == [w % p for w in want]


# --------------------------------------------------------------------------
# Digit-group choice: eq. ci_bound used as the CRT range condition.
# --------------------------------------------------------------------------

def _k_brute(na, nb, force=0):
    for k in range(18, 0, -1):
        if force and k != force:
            continue
        nk = -(-19 * na // k)
        mk = -(-19 * nb // k)
        if (10 ** k - 1) ** 2 * min(nk, mk) < P1 * P2:
            return k
    return 0


def test_choose_k_against_exact_bound():
    rng = random.Random(11)
    sizes = [1, 2, 79, 80, 81, 85, 86, 8000, 8059, 8060, 8061, 805900, 805901,
             10 ** 7, 2 ** 30] + [rng.randrange(1, 10 ** 8) for _ in range(200)]
    for na in sizes:
        nb = rng.choice(sizes)
        assert oracle.choose_k(na, nb) == _k_brute(na, nb), (na, nb)
        for f in (14, 16, 18):
            assert oracle.choose_k(na, nb, f) == _k_brute(na, nb, f)
    # k = 18 holds up to 80 limbs (85 groups of 18 digits) and no further
    assert oracle.choose_k(80, 80) == 18 and oracle.choose_k(81, 81) == 17
    assert oracle.choose_k(80, 10 ** 6) == 18


def test_ratio_of_largest_coefficient_at_k18_edge():
    # The largest coefficient allowed at k = 18 comes within 0.1% of p1*p2:
    # 85 * (10^18 - 1)^2 / (p1 p2).
    r = 85 * (10 ** 18 - 1) ** 2 / (P1 * P2)
    assert 0.999 < r < 1.0
    assert 86 * (10 ** 18 - 1) ** 2 > P1 * P2


# --------------------------------------------------------------------------
# Whole product: O1 and O2 against CPython integers and closed forms.
# --------------------------------------------------------------------------

def _rand_limbs(rng, n):
    return np.array([rng.randrange(10 ** 19) for _ in range(n)], dtype=np.uint64)


@pytest.mark.parametrize("na,nb", [(0, 0), (0, 3), (3, 0), (1, 1), (1, 7), (2, 2), (5, 3),
                                   (17, 31), (64, 64), (80, 80), (81, 200), (300, 17),
                                   (1000, 999)])
def test_products_match_python_int(na, nb):
    rng = random.Random(na * 1000 + nb)
    a = _rand_limbs(rng, na)
    b = _rand_limbs(rng, nb)
    want = int_to_limbs(limbs_to_int(a) * limbs_to_int(b), na + nb)
    np.testing.assert_array_equal(oracle.schoolbook(a, b), want)
    np.testing.assert_array_equal(oracle.mul_ntt(a, b), want)


def test_product_independent_of_k():
    rng = random.Random(5)
    a = _rand_limbs(rng, 40)
    b = _rand_limbs(rng, 23)
    want = int_to_limbs(limbs_to_int(a) * limbs_to_int(b), 63)
    for k in range(1, 19):
        if oracle.choose_k(40, 23, k) == 0:
            with pytest.raises(oracle.OracleError):
                oracle.mul_ntt(a, b, force_k=k)
            continue
        out, info = oracle.mul_ntt(a, b, force_k=k, return_info=True)
        assert info.k == k
        np.testing.assert_array_equal(out, want)


def test_all_nines_limbs_and_bound_edges():
    for nl in (1, 2, 79, 80, 81, 150):
        a = synth.repeated_limbs(10 ** 19 - 1, nl)
        x = limbs_to_int(a)
        assert x == 10 ** (19 * nl) - 1
        want = int_to_limbs(x * x, 2 * nl)
        out, info = oracle.mul_ntt(a, a, return_info=True)
        np.testing.assert_array_equal(out, want)
        assert info.k == (18 if nl <= 80 else 17)
    # forcing k = 18 past the bound is refused
    a = synth.repeated_limbs(10 ** 19 - 1, 81)
    with pytest.raises(oracle.OracleError) as e:
        oracle.mul_ntt(a, a, force_k=18)
    assert e.value.code == oracle.ORACLE_ERANGE


def _closed_nines_product(da, db):
    """Little-endian digits of (10^da - 1)(10^db - 1), da >= db >= 1:
    10^(da+db) - 10^da - 10^db + 1."""
    d = np.zeros(da + db, dtype=np.uint8)
    d[0] = 1
    d[db:da] = 9
    d[da] = 8
    d[da + 1:da + db] = 9
    return d


@pytest.mark.parametrize("da,db", [(1, 1), (5, 5), (19, 19), (40, 7), (1530, 1530), (1520, 1520),
                                   (20000, 20000), (30011, 1777)])
def test_closed_form_nines(da, db):
    a = synth.all_nines(da)
    b = synth.all_nines(db)
    na, nb = len(a), len(b)
    want_digits = _closed_nines_product(da, db)
    want = synth.pack_digits(np.concatenate([want_digits, np.zeros(19 * (na + nb) - len(want_digits), np.uint8)]))
    np.testing.assert_array_equal(oracle.mul_ntt(a, b), want)
    if da * db <= 10 ** 8:
        np.testing.assert_array_equal(oracle.schoolbook(a, b), want)


def test_closed_form_difference_of_squares_and_shift():
    for a_d in (3, 19, 38, 1000, 12345):
        x = synth.pack_digits(np.array([1] + [0] * (a_d - 1) + [1], dtype=np.uint8))  # 10^a + 1
        y = synth.all_nines(a_d)                                                    # 10^a - 1
        out = oracle.mul_ntt(x, y)
        want = synth.pack_digits(np.concatenate([np.full(2 * a_d, 9, np.uint8),
                                                 np.zeros(19 * (len(x) + len(y)) - 2 * a_d, np.uint8)]))
        np.testing.assert_array_equal(out, want)
    rng = random.Random(9)
    a = _rand_limbs(rng, 50)
    for j in (0, 1, 7):
        s = np.zeros(j + 1, dtype=np.uint64)
        s[j] = 1                              # 10^(19 j)
        out = oracle.mul_ntt(a, s)
        want = np.zeros(51 + j, dtype=np.uint64)
        want[j:j + 50] = a
        np.testing.assert_array_equal(out, want)


def test_invalid_limb_and_empty():
    a = np.array([10 ** 19], dtype=np.uint64)
    b = np.array([1], dtype=np.uint64)
    for f in (oracle.mul_ntt, oracle.schoolbook):
        with pytest.raises(oracle.OracleError) as e:
            f(a, b)
        assert e.value.code == oracle.ORACLE_EDIGIT
    out = oracle.mul_ntt(np.zeros(0, np.uint64), np.array([5, 6], np.uint64))
    np.testing.assert_array_equal(out, np.zeros(2, np.uint64))


def _residues(limbs):
    """Z mod (10^19 - 1) (limb sum) and Z mod (10^19 + 1) (alternating sum)."""
    m1, m2 = 10 ** 19 - 1, 10 ** 19 + 1
    v = [int(t) for t in limbs]
    return sum(v) % m1, sum(t if i % 2 == 0 else -t for i, t in enumerate(v)) % m2


@pytest.mark.slow
def test_large_random_product_residues_and_schoolbook():
    # 100,000-digit operands: O2 against O1 bit for bit, and both against
    # the residues mod 10^19 -/+ 1 of the factors.
    a = synth.random_operand(100_000, 1001)
    b = synth.random_operand(100_000, 1002)
    o2, info = oracle.mul_ntt(a, b, return_info=True)
    assert info.k == 17 and info.N == 2 ** 14
    np.testing.assert_array_equal(o2, oracle.schoolbook(a, b))
    ra, rb, rz = _residues(a), _residues(b), _residues(o2)
    assert rz[0] == ra[0] * rb[0] % (10 ** 19 - 1)
    assert rz[1] == ra[1] * rb[1] % (10 ** 19 + 1)
    assert limbs_to_int(o2) == limbs_to_int(a) * limbs_to_int(b)
