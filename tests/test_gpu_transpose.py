"""The in-place transposition kernels (the scheme of Section 7.6 for square,
n x 2n and 2n x n matrices) against numpy's transpose, and the
natural-order export of a cached forward transform against the oracle's
transform tau(A, omega) of the operand's digit groups (the DFT of eq. dft,
pinned to its O(N^2) definition by the oracle tests)."""
import sys

import numpy as np
import pytest

import oracle
from helpers import limbs_to_int

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2011_11524_amd as dm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = dm.Context(0)
    yield dm, torch, ctx
    ctx.close()


SHAPES = [(32, 32), (32, 64), (64, 32), (128, 128), (256, 512), (512, 256), (1024, 1024),
          (2048, 4096), (4096, 2048), (4096, 8192), (8192, 4096), (8192, 8192)]


@pytest.mark.parametrize("rows,cols", SHAPES)
def test_inplace_transpose_vs_numpy(env, rows, cols):
    dm, torch, ctx = env
    _note(f"in-place transpose {rows}x{cols}")
    rng = np.random.default_rng(rows * 7 + cols)
    host = rng.integers(0, 2 ** 63, size=rows * cols, dtype=np.uint64) | np.uint64(1)
    t = dm.to_device(host)
    got = ctx.transpose(t, rows, cols)
    assert tuple(got.shape) == (cols, rows)
    np.testing.assert_array_equal(got.cpu().numpy(), host.reshape(rows, cols).T)


def test_transpose_rejects_other_shapes(env):
    dm, torch, ctx = env
    t = dm.to_device(np.zeros(64 * 256, np.uint64))
    for rows, cols in ((64, 256), (256, 64), (16, 16), (48, 96), (16384, 1)):
        with pytest.raises(dm.DmulError) as ei:
            ctx.transpose(t, rows, cols)
        assert ei.value.code == dm.DMUL_EINVAL


def _groups(a, k, n, N):
    """The first n base-10^k digit groups of the integer a (limbs), zero
    padded to N: Section 3.2's split, by Python integer arithmetic."""
    x = limbs_to_int(a)
    B = 10 ** k
    out = np.zeros(N, dtype=np.uint64)
    for i in range(n):
        x, out[i] = divmod(x, B)
    assert x == 0
    return out


@pytest.mark.parametrize("logN", [10, 11, 12, 13, 15, 16])
def test_spectrum_export_is_the_dft(env, logN):
    dm, torch, ctx = env
    N = 1 << logN
    na = max(1, (N * 7) // 19 - 3)        # about 0.45 N groups of 16 or 17 digits per operand
    nb = na - 1
    pl = dm.plan(na, nb, pow2=True)
    assert pl.N == N and pl.factor == 1
    _note(f"spectrum export N=2^{logN} ({1 << pl.log2_rows}x{1 << pl.log2_cols}) k={pl.k}")
    rng = np.random.default_rng(1000 + logN)
    a = rng.integers(0, 10 ** 19, size=na, dtype=np.uint64)
    s = ctx.spectrum(dm.to_device(a), nb, pow2=True)
    got = ctx.spectrum_export(s).cpu().numpy()
    s.close()
    x = _groups(a, pl.k, pl.groups_a, N)
    ps, gs = oracle.primes()
    for i in range(2):
        xi = pow(gs[i], (ps[i] - 1) // N, ps[i])
        np.testing.assert_array_equal(got[i], oracle.transform(x % np.uint64(ps[i]), ps[i], xi))


def test_spectrum_export_refusals(env):
    dm, torch, ctx = env
    a = dm.to_device(np.arange(1, 301, dtype=np.uint64))
    s = ctx.spectrum(a, 250)                     # 3 * 2^e layout: no natural-order export
    assert dm.plan(300, 250).factor == 3
    with pytest.raises(dm.DmulError) as ei:
        ctx.spectrum_export(s)
    assert ei.value.code == dm.DMUL_EINVAL
    s.close()
    b = dm.to_device(np.arange(1, 20, dtype=np.uint64))
    s = ctx.spectrum(b, 10, pow2=True)            # N < 2^10
    with pytest.raises(dm.DmulError):
        ctx.spectrum_export(s)
    s.close()
