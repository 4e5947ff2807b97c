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


@pytest.mark.parametrize("na,nb", [(1, 1), (2, 3), (80, 80), (81, 81), (5264, 5264), (526316, 526316),
                                   (2105264, 1052632), (10**6, 3), (3, 10**6), (12345, 67890)])
def test_plan_matches_oracle_rule(na, nb):
    p = dm.plan(na, nb)
    assert p.k == oracle.choose_k(na, nb)
    n = -(-19 * na // p.k)
    m = -(-19 * nb // p.k)
    assert (p.groups_a, p.groups_b) == (n, m)
    assert 2 ** (p.log2_n - 1) < n + m <= 2 ** p.log2_n or (p.log2_n == 2 and n + m <= 4)
    assert p.log2_rows == p.log2_n // 2 and p.log2_rows + p.log2_cols == p.log2_n
    assert p.workspace_bytes == 32 * p.N == dm.workspace_bytes(na, nb)


def test_plan_forced_k_and_ranges():
    assert dm.plan(2105264, 1052632, force_k=14).log2_n == 23
    assert dm.plan(2105264, 1052632).log2_n == 22
    with pytest.raises(dm.DmulError) as e:
        dm.plan(81, 81, force_k=18)         # 86 groups of 18 digits break the bound
    assert e.value.code == dm.DMUL_ERANGE
    with pytest.raises(dm.DmulError) as e:
        dm.plan(10, 10, force_k=12)         # below the three-part split
    assert e.value.code == dm.DMUL_EINVAL
    with pytest.raises(dm.DmulError) as e:
        dm.plan(2 ** 30, 2 ** 30)           # beyond two LDS passes
    assert e.value.code == dm.DMUL_ERANGE
    assert dm.workspace_bytes(0, 5) == 0
