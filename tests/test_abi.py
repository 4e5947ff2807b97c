"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/dmul.h declares, and its planning agrees with the
oracle's digit-group rule and the padding rule of Section 3.2."""
import ctypes
import os
import re

import pytest

import oracle
import paper_2011_11524_amd as dm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "dmul.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmul\w*)\s*\(", text)) - {"DMUL_FLAG_FORCE_K"})


def test_header_symbols_exported():
    names = _header_functions()
    assert names, "no functions parsed from the header"
    L = dm.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/dmul.h but not exported"
    assert sorted(dm.EXPORTS) == names


def test_primes_match_oracle():
    assert dm.primes() == oracle.primes()


def test_strerror():
    for c in (0, -1, -2, -3, -4, -5):
        assert dm.strerror(c)
    assert "10^19" in dm.strerror(dm.DMUL_EDIGIT)


def _lengths(need, pow2):
    """Transform lengths the planner may pick for `need` coefficients, in
    increasing order: 2^e (2 <= e <= 28) and, unless pow2, 3*2^e
    (4 <= e <= 23), each with its R x C layout (log2 R, log2 C)."""
    out = []
    for e in range(2, 29):
        out.append((1 << e, 1, e, e // 2))
    if not pow2:
        for e in range(4, 24):
            out.append((3 << e, 3, e, max(e // 2, e - 11)))
    return sorted(o for o in out if o[0] >= need)


SIZES = [(1, 1), (2, 3), (80, 80), (81, 81), (5264, 5264), (526316, 526316), (2105264, 1052632),
         (10**6, 3), (3, 10**6), (12345, 67890), (7, 9), (40, 41), (300, 200)]


@pytest.mark.parametrize("pow2", [False, True])
@pytest.mark.parametrize("na,nb", SIZES)
def test_plan_matches_oracle_rule(na, nb, pow2):
    p = dm.plan(na, nb, pow2=pow2)
    assert p.k == oracle.choose_k(na, nb)
    n = -(-19 * na // p.k)
    m = -(-19 * nb // p.k)
    assert (p.groups_a, p.groups_b) == (n, m)
    N, factor, e, log_r = _lengths(n + m, pow2)[0]
    assert (p.N, p.factor, p.log2_n, p.log2_rows) == (N, factor, e, log_r)
    assert p.log2_rows + p.log2_cols == p.log2_n
    assert p.workspace_bytes == 32 * p.N == (dm.workspace_bytes(na, nb) if not pow2 else 32 * p.N)


def test_plan_forced_k_and_ranges():
    # C3 at k = 14: 4,285,715 coefficients fit 3*2^21 (2048 rows of 3*1024)
    p = dm.plan(2105264, 1052632, force_k=14)
    assert (p.N, p.factor, p.log2_rows, p.log2_cols) == (3 << 21, 3, 10, 11)
    assert dm.plan(2105264, 1052632, force_k=14, pow2=True).log2_n == 23
    assert dm.plan(2105264, 1052632).N == 1 << 22       # 4,000,001 <= 2^22 < 3*2^21
    assert dm.plan(526316, 526316).N == 3 << 19          # C2: 1,250,000 -> 1,572,864
    with pytest.raises(dm.DmulError) as e:
        dm.plan(81, 81, force_k=18)         # 86 groups of 18 digits break the bound
    assert e.value.code == dm.DMUL_ERANGE
    with pytest.raises(dm.DmulError) as e:
        dm.plan(10, 10, force_k=12)         # below the three-part split
    assert e.value.code == dm.DMUL_EINVAL
    with pytest.raises(dm.DmulError) as e:
        dm.plan(2 ** 30, 2 ** 30)           # beyond two LDS passes
    assert e.value.code == dm.DMUL_ERANGE
    # the longest 3*2^e length: 3*2^23 = 2^12 rows of 3*2^11; beyond it 2^25
    na = (3 << 23) * 15 // 19 // 2
    p = dm.plan(na, na)
    assert (p.N, p.log2_rows, p.log2_cols) == (3 << 23, 12, 11)
    assert dm.plan(na + 1000, na + 1000).N == 1 << 25
    assert dm.workspace_bytes(0, 5) == 0


def test_redundant_range_build_exports_and_plans():
    """libdmul_lazy.so: every declared function, its primes (the two largest
    c*3*2^n + 1 below 2^62 with n >= 32, the oracle's FindPrimes(63, 32, 2))
    and the planner's k rule under their product."""
    L = dm.lib("lazy")
    for n in _header_functions():
        assert hasattr(L, n), f"{n} not exported by the redundant-range build"
    p, g = dm.primes("lazy")
    assert p == oracle.find_primes(63, 32, 2)
    assert all(q < 2 ** 62 and q % 2 ** 32 == 1 for q in p)
    assert g == [oracle.generator(p[0]), oracle.generator(p[1])]
    P = p[0] * p[1]
    for na, nb in SIZES:
        k = next(k for k in range(18, 12, -1)
                 if (10 ** k - 1) ** 2 * min(-(-19 * na // k), -(-19 * nb // k)) < P)
        assert dm.plan(na, nb, variant="lazy").k == k


@pytest.mark.parametrize("name,value", [("DMUL_FORCE_K", "12"), ("DMUL_FORCE_K", "19"),
                                        ("DMUL_FORCE_K", "k15"), ("DMUL_FORCE_K", "15 "),
                                        ("DMUL_HBM_BUDGET", "-1"), ("DMUL_HBM_BUDGET", "1e9"),
                                        ("DMUL_HBM_BUDGET", "99999999999999999999999")])
def test_ctx_create_rejects_bad_environment(monkeypatch, name, value):
    """A malformed DMUL_FORCE_K or DMUL_HBM_BUDGET fails context creation
    with DMUL_EINVAL before any device call (so this runs without a GPU)."""
    monkeypatch.setenv(name, value)
    L = dm.lib()
    h = ctypes.c_void_p(1)
    assert L.dmul_ctx_create(ctypes.byref(h), 0, 0) == dm.DMUL_EINVAL
    assert h.value is None
