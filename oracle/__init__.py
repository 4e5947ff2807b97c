"""CPU oracle for the exact decimal product -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never links, loads or
calls it, and the two share no code: the only module both sides use is the
seeded operand generator in ``synth``, which holds none of the method's
arithmetic.

Contents
--------
* ``schoolbook(a, b)``      -- O1, the plain definition of the product of two
  base-10^19 integers (Section 3.2), in C.
* ``mul_ntt(a, b, force_k)`` -- O2, the two-prime number-theoretic-transform
  method in its plainest form (Sections 3.2-3.5, 4.2-4.5, 5.1-5.2, 8.2.2),
  in C: naive '%' reduction, the transform of eq. dft by the recursive
  radix-2 split into even- and odd-indexed terms, textbook CRT, sequential
  carry.
* ``is_prime``, ``find_primes``, ``find_primes_for_n``, ``generator``,
  ``transform``, ``choose_k``, ``cyclic_convolution`` -- the pieces the pin
  tests check one by one.
* ``lambda_digits`` -- eq. lambda of Section 4.2 in exact integer arithmetic
  (pure Python; a handful of calls).
* ``sanitize_check.c`` -- a driver that runs every entry point of oracle.c
  under AddressSanitizer and UndefinedBehaviorSanitizer (built by the test
  suite with gcc).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORACLE_OK = 0
ORACLE_EINVAL = -1
ORACLE_EDIGIT = -2
ORACLE_ERANGE = -3
ORACLE_ENOMEM = -4
ORACLE_EINTERNAL = -5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with the host C compiler."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("n", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("N", ctypes.c_uint64), ("p1", ctypes.c_uint64), ("p2", ctypes.c_uint64)]


@dataclass
class NttInfo:
    k: int
    n: int
    m: int
    N: int
    p1: int
    p2: int


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_schoolbook.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u64p]
        lib.oracle_mul_ntt.argtypes = [u64p, ctypes.c_size_t, u64p, ctypes.c_size_t, u64p,
                                       ctypes.c_int, ctypes.POINTER(_Info)]
        lib.oracle_is_prime.argtypes = [ctypes.c_uint64]
        lib.oracle_find_primes_for_n.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u64p]
        lib.oracle_find_primes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p]
        lib.oracle_generator.argtypes = [ctypes.c_uint64]
        lib.oracle_generator.restype = ctypes.c_uint64
        lib.oracle_primes.argtypes = [u64p, u64p]
        lib.oracle_transform.argtypes = [u64p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_choose_k.argtypes = [ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int]
        lib.oracle_cyclic_convolution.argtypes = [u64p, u64p, ctypes.c_size_t, u64p, u64p]
        _lib = lib
    return _lib


def _u64(arr) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(arr, dtype=np.uint64))


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def schoolbook(a, b) -> np.ndarray:
    """O1: exact product, na+nb limbs (base 10^19, little-endian)."""
    a, b = _u64(a), _u64(b)
    out = np.zeros(len(a) + len(b), dtype=np.uint64)
    rc = _load().oracle_schoolbook(_ptr(a), len(a), _ptr(b), len(b), _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


def mul_ntt(a, b, force_k: int = 0, return_info: bool = False):
    """O2: exact product by the two-prime NTT method."""
    a, b = _u64(a), _u64(b)
    out = np.zeros(len(a) + len(b), dtype=np.uint64)
    info = _Info()
    rc = _load().oracle_mul_ntt(_ptr(a), len(a), _ptr(b), len(b), _ptr(out), int(force_k),
                                ctypes.byref(info))
    if rc:
        raise OracleError(rc)
    if return_info:
        return out, NttInfo(info.k, info.n, info.m, info.N, info.p1, info.p2)
    return out


def is_prime(n: int) -> bool:
    return bool(_load().oracle_is_prime(int(n)))


def find_primes_for_n(n: int, p_max: int, count: int) -> list[int]:
    buf = np.zeros(max(count, 1), dtype=np.uint64)
    got = _load().oracle_find_primes_for_n(int(n), int(p_max), int(count), _ptr(buf))
    return [int(v) for v in buf[:got]]


def find_primes(w: int, n_min: int, count: int) -> list[int]:
    buf = np.zeros(max(count, 1), dtype=np.uint64)
    got = _load().oracle_find_primes(int(w), int(n_min), int(count), _ptr(buf))
    if got != count:
        raise OracleError(got)
    return [int(v) for v in buf[:count]]


def generator(p: int) -> int:
    return int(_load().oracle_generator(int(p)))


def primes() -> tuple[list[int], list[int]]:
    """The method's two primes (p1 < p2) and their smallest generators."""
    p = np.zeros(2, dtype=np.uint64)
    g = np.zeros(2, dtype=np.uint64)
    rc = _load().oracle_primes(_ptr(p), _ptr(g))
    if rc:
        raise OracleError(rc)
    return [int(v) for v in p], [int(v) for v in g]


def transform(x, p: int, omega: int) -> np.ndarray:
    """tau(A, omega): A'[k] = sum_i A[i] omega^(ik) mod p (Section 5)."""
    arr = _u64(x).copy()
    rc = _load().oracle_transform(_ptr(arr), len(arr), int(p), int(omega))
    if rc:
        raise OracleError(rc)
    return arr


def choose_k(na: int, nb: int, force_k: int = 0) -> int:
    return int(_load().oracle_choose_k(int(na), int(nb), int(force_k)))


def cyclic_convolution(x, y) -> list[int]:
    """Eq. star over Z by its O(n^2) definition (inputs small enough that
    every sum fits in 128 bits)."""
    x, y = _u64(x), _u64(y)
    n = len(x)
    lo = np.zeros(n, dtype=np.uint64)
    hi = np.zeros(n, dtype=np.uint64)
    _load().oracle_cyclic_convolution(_ptr(x), _ptr(y), n, _ptr(lo), _ptr(hi))
    return [int(h) << 64 | int(l) for l, h in zip(lo, hi)]


def lambda_digits(mu_bits: int, M: int, ell: int) -> int:
    """eq. lambda (Section 4.2): max{n : (10^n - 1)^2 < (mu/2)^ell / M},
    with mu = 2^mu_bits, evaluated exactly as (10^n-1)^2 * M < (mu/2)^ell."""
    bound = (1 << ((mu_bits - 1) * ell))
    n = 0
    while ((10 ** (n + 1) - 1) ** 2) * M < bound:
        n += 1
    return n
