"""Python binding of libdmul (the gfx950 decimal multiplier).

Argument marshalling only: every step of a product runs in the library's
HIP kernels, reached through the C ABI declared in ``include/dmul.h``.
PyTorch provides device memory (uint64 tensors) and streams.  There is no
CPU fallback: if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

import numpy as np

try:  # torch first, so libdmul binds to the HIP runtime torch already loaded
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
# Two builds of the same sources: the default one (primes below 2^63,
# canonical residues) and the redundant-range one (primes below 2^62,
# butterfly values kept in [0, 2p) / [0, 4p)).  DMUL_LIB=lazy makes the
# second the default of this module.
LIB_PATHS = {"default": os.path.join(_HERE, "libdmul.so"),
             "lazy": os.path.join(_HERE, "libdmul_lazy.so")}
DEFAULT_VARIANT = "lazy" if os.environ.get("DMUL_LIB", "") == "lazy" else "default"
LIB_PATH = LIB_PATHS[DEFAULT_VARIANT]

DMUL_OK = 0
DMUL_EINVAL = -1
DMUL_EDIGIT = -2
DMUL_ERANGE = -3
DMUL_ENOMEM = -4
DMUL_EDEVICE = -5
DMUL_FLAG_GRAPH = 0x100
DMUL_FLAG_POW2 = 0x200

# Every function the header declares (checked by the test suite).
EXPORTS = ("dmul", "dmul_ctx_create", "dmul_ctx_destroy", "dmul_ctx_set_stream", "dmul_ex",
           "dmul_sync", "dmul_batch", "dmul_plan", "dmul_workspace_bytes", "dmul_strerror",
           "dmul_host", "dmul_primes", "dmul_debug_residues", "dmul_version", "dmul_ctx_profile",
           "dmul_ctx_profile_read", "dmul_phase_name", "dmul_ctx_profile_events", "dmul_ctx_tune",
           "dmul_spectrum_create", "dmul_spectrum_destroy", "dmul_spectrum_bytes", "dmul_ex_spectrum",
           "dmul_batch_ex", "dmul_ctx_timing", "dmul_ctx_timing_read", "dmul_ex_noalloc",
           "dmul_spectrum_export", "dmul_debug_transpose", "dmul_ctx_tune_path", "dmul_ctx_tune_streams",
           "dmul_ctx_tune_queue")


class DmulError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = f"{what}: " if what else ""
        super().__init__(f"{msg}{strerror(code)} ({code})")
        self.code = code


class _PlanInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("log2_n", ctypes.c_int32), ("log2_rows", ctypes.c_int32),
                ("log2_cols", ctypes.c_int32), ("groups_a", ctypes.c_uint64),
                ("groups_b", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("transform_len", ctypes.c_uint64), ("factor", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


@dataclass
class Plan:
    """N = factor * 2^log2_n as R x C, R = 2^log2_rows, C = factor * 2^log2_cols."""
    k: int
    log2_n: int
    log2_rows: int
    log2_cols: int
    groups_a: int
    groups_b: int
    workspace_bytes: int
    N: int
    factor: int


_libs = {}


def lib(variant: str | None = None):
    """Load a build of the library ("default": libdmul.so, "lazy":
    libdmul_lazy.so; None: the module's default); raises if it has not been
    built."""
    variant = variant or DEFAULT_VARIANT
    if variant in _libs:
        return _libs[variant]
    path = LIB_PATHS[variant]
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "or python paper_2011_11524_amd/build.py")
    L = ctypes.CDLL(path)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    vp = ctypes.c_void_p
    sz = ctypes.c_size_t
    L.dmul.argtypes = [vp, sz, vp, sz, vp]
    L.dmul_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, sz]
    L.dmul_ctx_destroy.argtypes = [vp]
    L.dmul_ctx_set_stream.argtypes = [vp, vp]
    L.dmul_ex.argtypes = [vp, vp, sz, vp, sz, vp, ctypes.c_uint]
    L.dmul_sync.argtypes = [vp]
    L.dmul_ex_noalloc.argtypes = [vp, vp, sz, vp, sz, vp, ctypes.c_uint]
    L.dmul_batch.argtypes = [vp, sz, ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(vp),
                             ctypes.POINTER(sz), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32),
                             ctypes.c_uint]
    L.dmul_plan.argtypes = [sz, sz, ctypes.c_uint, ctypes.POINTER(_PlanInfo)]
    L.dmul_workspace_bytes.argtypes = [sz, sz]
    L.dmul_workspace_bytes.restype = sz
    L.dmul_strerror.argtypes = [ctypes.c_int]
    L.dmul_strerror.restype = ctypes.c_char_p
    L.dmul_host.argtypes = [ctypes.c_int, u64p, sz, u64p, sz, u64p, ctypes.c_uint]
    L.dmul_primes.argtypes = [u64p, u64p]
    L.dmul_primes.restype = None
    L.dmul_debug_residues.argtypes = [vp, vp, sz, vp, sz, vp, ctypes.c_uint]
    L.dmul_version.restype = ctypes.c_char_p
    L.dmul_ctx_profile.argtypes = [vp, ctypes.c_int]
    L.dmul_ctx_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    L.dmul_ctx_profile_events.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.dmul_ctx_tune.argtypes = [vp, ctypes.c_uint64, ctypes.c_int]
    L.dmul_ctx_tune_path.argtypes = [vp, ctypes.c_uint64, ctypes.c_int]
    L.dmul_ctx_tune_streams.argtypes = [vp, ctypes.c_int]
    L.dmul_ctx_tune_queue.argtypes = [vp, ctypes.c_int]
    L.dmul_ctx_timing.argtypes = [vp, ctypes.c_int]
    L.dmul_ctx_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz]
    L.dmul_ctx_timing_read.restype = ctypes.c_long
    L.dmul_spectrum_create.argtypes = [vp, vp, sz, sz, ctypes.c_uint, vp, sz, ctypes.POINTER(vp)]
    L.dmul_spectrum_destroy.argtypes = [vp]
    L.dmul_spectrum_bytes.argtypes = [sz, sz, ctypes.c_uint]
    L.dmul_spectrum_bytes.restype = sz
    L.dmul_ex_spectrum.argtypes = [vp, vp, vp, sz, vp, vp, ctypes.c_uint]
    L.dmul_batch_ex.argtypes = [vp, sz, ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(vp),
                                ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(vp),
                                ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32), ctypes.c_uint]
    L.dmul_spectrum_export.argtypes = [vp, vp, vp]
    L.dmul_debug_transpose.argtypes = [vp, vp, sz, sz]
    L.dmul_phase_name.argtypes = [ctypes.c_int]
    L.dmul_phase_name.restype = ctypes.c_char_p
    _libs[variant] = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().dmul_strerror(int(code)).decode()
    except RuntimeError:
        return f"dmul status {code}"


def flags_for(force_k: int = 0, pow2: bool = False) -> int:
    return (int(force_k) & 0x1F) | (DMUL_FLAG_POW2 if pow2 else 0)


def primes(variant: str | None = None) -> tuple[list[int], list[int]]:
    p = (ctypes.c_uint64 * 2)()
    g = (ctypes.c_uint64 * 2)()
    lib(variant).dmul_primes(p, g)
    return [int(p[0]), int(p[1])], [int(g[0]), int(g[1])]


def plan(na: int, nb: int, force_k: int = 0, pow2: bool = False, variant: str | None = None) -> Plan:
    info = _PlanInfo()
    rc = lib(variant).dmul_plan(int(na), int(nb), flags_for(force_k, pow2), ctypes.byref(info))
    if rc:
        raise DmulError(rc, "dmul_plan")
    return Plan(info.k, info.log2_n, info.log2_rows, info.log2_cols, info.groups_a,
                info.groups_b, info.workspace_bytes, info.transform_len, info.factor)


def workspace_bytes(na: int, nb: int) -> int:
    return int(lib().dmul_workspace_bytes(int(na), int(nb)))


def spectrum_bytes(na: int, nb: int, force_k: int = 0, pow2: bool = False) -> int:
    return int(lib().dmul_spectrum_bytes(int(na), int(nb), flags_for(force_k, pow2)))


class Spectrum:
    """Cached forward transforms of one operand (dmul_spectrum): made by
    Context.spectrum, used in place of the operand's limbs."""

    def __init__(self, handle, na: int, nb_plan: int, flags: int, owner, mem=None):
        self._h = handle
        self.na = int(na)
        self.nb_plan = int(nb_plan)
        self.flags = int(flags)
        self._lib = owner._lib
        self.mem = mem          # the caller's buffer holding the transforms, if any

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.dmul_spectrum_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_limbs(t, name: str):
    if torch is None or not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.uint64 or t.dim() != 1 or not t.is_contiguous() or t.device.type != "cuda":
        raise TypeError(f"{name} must be a contiguous 1-D torch.uint64 CUDA tensor")


class Context:
    """A dmul context: device tables, workspace, a stream (default: torch's
    current stream on the device at creation time)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream=None, variant: str | None = None):
        self.variant = variant or DEFAULT_VARIANT
        self._lib = lib(self.variant)
        self._pending = []          # batches enqueued since the last sync
        h = ctypes.c_void_p()
        rc = self._lib.dmul_ctx_create(ctypes.byref(h), int(device), int(budget_bytes))
        if rc:
            raise DmulError(rc, "dmul_ctx_create")
        self._h = h
        self.device = int(device)
        self.set_stream(stream if stream is not None else torch.cuda.current_stream(self.device))

    def set_stream(self, stream) -> None:
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        self.stream = stream
        rc = self._lib.dmul_ctx_set_stream(self._h, ctypes.c_void_p(ptr))
        if rc:
            raise DmulError(rc, "dmul_ctx_set_stream")

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.dmul_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- single products ----------------------------------------------------
    def mul_async(self, a, b, out, force_k: int = 0, pow2: bool = False) -> None:
        _check_limbs(a, "a")
        _check_limbs(b, "b")
        _check_limbs(out, "out")
        if out.numel() != a.numel() + b.numel():
            raise ValueError("out must hold len(a) + len(b) limbs")
        rc = self._lib.dmul_ex(self._h, ctypes.c_void_p(a.data_ptr()), a.numel(),
                               ctypes.c_void_p(b.data_ptr()), b.numel(),
                               ctypes.c_void_p(out.data_ptr()), flags_for(force_k, pow2))
        if rc:
            raise DmulError(rc, "dmul_ex")

    def mul_noalloc_async(self, a, b, out, force_k: int = 0, pow2: bool = False) -> None:
        """dmul_ex_noalloc: the product in the library's static scratch (no
        device allocation; transform lengths up to 2^21)."""
        _check_limbs(a, "a")
        _check_limbs(b, "b")
        _check_limbs(out, "out")
        if out.numel() != a.numel() + b.numel():
            raise ValueError("out must hold len(a) + len(b) limbs")
        rc = self._lib.dmul_ex_noalloc(self._h, ctypes.c_void_p(a.data_ptr()), a.numel(),
                                       ctypes.c_void_p(b.data_ptr()), b.numel(),
                                       ctypes.c_void_p(out.data_ptr()), flags_for(force_k, pow2))
        if rc:
            raise DmulError(rc, "dmul_ex_noalloc")

    def sync(self) -> None:
        rc = self._lib.dmul_sync(self._h)
        # the status arrays of the batches this sync completed have been filled
        self._pending = []
        if rc:
            raise DmulError(rc, "dmul_sync")

    def mul(self, a, b, force_k: int = 0, out=None, pow2: bool = False):
        if out is None:
            out = torch.empty(a.numel() + b.numel(), dtype=torch.uint64, device=a.device)
        self.mul_async(a, b, out, force_k, pow2)
        self.sync()
        return out

    # -- cached transforms ---------------------------------------------------
    def spectrum(self, a, nb: int, force_k: int = 0, pow2: bool = False, mem=None) -> "Spectrum":
        """Forward transforms of a for products with partners of nb limbs
        (valid for every partner with the same plan k and N).  mem: an
        optional device tensor (spectrum_bytes(...) bytes at least) that
        holds them; the Spectrum keeps a reference to it."""
        _check_limbs(a, "a")
        h = ctypes.c_void_p()
        flags = flags_for(force_k, pow2)
        mp = ctypes.c_void_p(mem.data_ptr()) if mem is not None else None
        mb = mem.numel() * mem.element_size() if mem is not None else 0
        rc = self._lib.dmul_spectrum_create(self._h, ctypes.c_void_p(a.data_ptr()), a.numel(), int(nb),
                                            flags, mp, mb, ctypes.byref(h))
        if rc:
            raise DmulError(rc, "dmul_spectrum_create")
        return Spectrum(h, a.numel(), nb, flags, self, mem)

    def mul_spectrum_async(self, sa: "Spectrum", b, out, sb: "Spectrum" = None, force_k: int = 0,
                           pow2: bool = False) -> None:
        """out = X * Y with X from its spectrum sa, Y from limbs b or (b None)
        from its spectrum sb."""
        _check_limbs(out, "out")
        if sb is not None:
            nb, bp = sb.na, None
        else:
            _check_limbs(b, "b")
            nb, bp = b.numel(), b.data_ptr()
        if out.numel() != sa.na + nb:
            raise ValueError("out must hold na + nb limbs")
        rc = self._lib.dmul_ex_spectrum(self._h, sa._h, ctypes.c_void_p(bp) if bp else None, nb,
                                        sb._h if sb is not None else None,
                                        ctypes.c_void_p(out.data_ptr()), flags_for(force_k, pow2))
        if rc:
            raise DmulError(rc, "dmul_ex_spectrum")

    def mul_spectrum(self, sa: "Spectrum", b=None, sb: "Spectrum" = None, force_k: int = 0,
                     pow2: bool = False):
        nb = sb.na if sb is not None else b.numel()
        out = torch.empty(sa.na + nb, dtype=torch.uint64, device=f"cuda:{self.device}")
        self.mul_spectrum_async(sa, b, out, sb, force_k, pow2)
        self.sync()
        return out

    def spectrum_export(self, s: "Spectrum"):
        """The spectrum in natural frequency order: a (2, N) uint64 tensor,
        row i the transform modulo prime i (power-of-two plans, N >= 2^10)."""
        N = plan(s.na, s.nb_plan, s.flags & 0x1F, bool(s.flags & DMUL_FLAG_POW2), self.variant).N
        out = torch.empty(2 * N, dtype=torch.uint64, device=f"cuda:{self.device}")
        rc = self._lib.dmul_spectrum_export(self._h, s._h, ctypes.c_void_p(out.data_ptr()))
        if rc:
            raise DmulError(rc, "dmul_spectrum_export")
        self.sync()
        return out.view(2, N)

    def transpose(self, t, rows: int, cols: int):
        """In-place transposition of a rows x cols uint64 CUDA tensor (its
        storage becomes cols x rows); blocking."""
        rc = self._lib.dmul_debug_transpose(self._h, ctypes.c_void_p(t.data_ptr()), int(rows), int(cols))
        if rc:
            raise DmulError(rc, "dmul_debug_transpose")
        self.sync()
        return t.view(cols, rows)

    # -- batches -------------------------------------------------------------
    def prepare_batch(self, pairs: Sequence, outs: Sequence) -> "PreparedBatch":
        """Marshal a batch once, for submitting the same products again
        (run_prepared): the pointer arrays are built here, not per call."""
        return PreparedBatch(pairs, outs)

    def run_prepared(self, pb: "PreparedBatch", force_k: int = 0, graph: bool = False,
                     pow2: bool = False):
        """Enqueue a prepared batch; returns its host status array (filled by
        sync())."""
        flags = flags_for(force_k, pow2) | (DMUL_FLAG_GRAPH if graph else 0)
        if pb.spectra:
            rc = self._lib.dmul_batch_ex(self._h, pb.n, pb.A, pb.NA, pb.SA, pb.B, pb.NB, pb.SB, pb.O,
                                         pb.st, flags)
        else:
            rc = self._lib.dmul_batch(self._h, pb.n, pb.A, pb.NA, pb.B, pb.NB, pb.O, pb.st, flags)
        if rc:
            raise DmulError(rc, "dmul_batch")
        # the library writes pb.st at the next sync: keep it (and the
        # batch's tensors) alive until then
        self._pending.append(pb)
        return pb.st

    def batch_async(self, pairs: Sequence, outs: Sequence, force_k: int = 0, graph: bool = False,
                    pow2: bool = False):
        """Enqueue len(pairs) products (a_i, b_i) -> outs[i]; returns the host
        status array that sync() fills in.  An operand may be a Spectrum of
        this context's device instead of a tensor.  graph=True captures the
        batch in a HIP graph, replayed when the same batch is submitted
        again."""
        pb = PreparedBatch(pairs, outs)
        return self.run_prepared(pb, force_k, graph, pow2)

    def batch(self, pairs: Sequence, force_k: int = 0, graph: bool = False, outs=None,
              pow2: bool = False):
        if outs is None:
            size = lambda x: x.na if isinstance(x, Spectrum) else x.numel()
            outs = [torch.empty(size(a) + size(b), dtype=torch.uint64, device=f"cuda:{self.device}")
                    for a, b in pairs]
        st = self.batch_async(pairs, outs, force_k, graph, pow2)
        self.sync()
        return outs, [int(s) for s in st]

    def tune(self, transform_len: int, row_iters: int) -> None:
        rc = self._lib.dmul_ctx_tune(self._h, int(transform_len), int(row_iters))
        if rc:
            raise DmulError(rc, "dmul_ctx_tune")

    def tune_path(self, transform_len: int, path: int) -> None:
        """0 default rule, 1 whole-product kernel (N <= 4096), 2 pass kernels."""
        rc = self._lib.dmul_ctx_tune_path(self._h, int(transform_len), int(path))
        if rc:
            raise DmulError(rc, "dmul_ctx_tune_path")

    def tune_streams(self, streams: int) -> None:
        rc = self._lib.dmul_ctx_tune_streams(self._h, int(streams))
        if rc:
            raise DmulError(rc, "dmul_ctx_tune_streams")

    def tune_queue(self, on: bool) -> None:
        """Whole-product classes of a batch in persistent launches per tier
        (True, the default) or one launch per transform length (False)."""
        rc = self._lib.dmul_ctx_tune_queue(self._h, 1 if on else 0)
        if rc:
            raise DmulError(rc, "dmul_ctx_tune_queue")

    # -- per-kernel timing ----------------------------------------------------
    def profile(self, enable: bool) -> None:
        rc = self._lib.dmul_ctx_profile(self._h, 1 if enable else 0)
        if rc:
            raise DmulError(rc, "dmul_ctx_profile")

    def profile_read(self) -> dict:
        n = 16
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_uint64 * n)()
        got = self._lib.dmul_ctx_profile_read(self._h, ms, cnt, n)
        if got < 0:
            raise DmulError(got, "dmul_ctx_profile_read")
        return {self._lib.dmul_phase_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(got)}

    def profile_events(self):
        """[(phase name, end ms)] of every kernel of the work completed by the
        last sync, in launch order."""
        n = self._lib.dmul_ctx_profile_events(self._h, None, None, 0)
        if n <= 0:
            return []
        ph = (ctypes.c_int32 * n)()
        t = (ctypes.c_double * n)()
        self._lib.dmul_ctx_profile_events(self._h, ph, t, n)
        return [(self._lib.dmul_phase_name(ph[i]).decode(), float(t[i])) for i in range(n)]

    # -- completion timing ---------------------------------------------------
    def timing(self, enable: bool) -> None:
        """Per-product completion events (batches keep their concurrent
        class streams; graph capture is skipped while on)."""
        rc = self._lib.dmul_ctx_timing(self._h, 1 if enable else 0)
        if rc:
            raise DmulError(rc, "dmul_ctx_timing")

    def timing_read(self) -> list:
        """Completion ms of every product of the work completed by the last
        sync (submission order), after the first of that work's start."""
        n = self._lib.dmul_ctx_timing_read(self._h, None, 0)
        if n < 0:
            raise DmulError(n, "dmul_ctx_timing_read")
        ms = (ctypes.c_double * max(n, 1))()
        self._lib.dmul_ctx_timing_read(self._h, ms, n)
        return [float(ms[i]) for i in range(n)]

    # -- debug view of the convolution ---------------------------------------
    def residues(self, a, b, force_k: int = 0, pow2: bool = False):
        """The cyclic convolution of the digit groups of a and b mod p1 and mod
        p2 (two length-N uint64 tensors)."""
        pl = plan(a.numel(), b.numel(), force_k, pow2)
        res = torch.empty(2 * pl.N, dtype=torch.uint64, device=a.device)
        rc = self._lib.dmul_debug_residues(self._h, ctypes.c_void_p(a.data_ptr()), a.numel(),
                                           ctypes.c_void_p(b.data_ptr()), b.numel(),
                                           ctypes.c_void_p(res.data_ptr()), flags_for(force_k, pow2))
        if rc:
            raise DmulError(rc, "dmul_debug_residues")
        return res[: pl.N], res[pl.N:]


def to_device(limbs, device: int = 0):
    """numpy uint64 limbs -> CUDA uint64 tensor."""
    arr = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint64))
    return torch.from_numpy(arr).to(f"cuda:{device}")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def mul(a, b, force_k: int = 0, pow2: bool = False):
    """Z = X * Y with the device's default context (blocking).  a, b: CUDA
    uint64 tensors; returns a new tensor of len(a) + len(b) limbs."""
    _check_limbs(a, "a")
    _check_limbs(b, "b")
    out = torch.empty(a.numel() + b.numel(), dtype=torch.uint64, device=a.device)
    if force_k or pow2:
        ctx = _default_context(a.device.index or 0)
        return ctx.mul(a, b, force_k, out, pow2)
    with torch.cuda.device(a.device):
        # dmul runs on the null stream: operands made on another current
        # stream must be complete first
        cur = torch.cuda.current_stream()
        if cur.cuda_stream != 0:
            cur.synchronize()
        rc = lib().dmul(ctypes.c_void_p(a.data_ptr() if a.numel() else 0), a.numel(),
                        ctypes.c_void_p(b.data_ptr() if b.numel() else 0), b.numel(),
                        ctypes.c_void_p(out.data_ptr() if out.numel() else 0))
    if rc:
        raise DmulError(rc, "dmul")
    return out


def mul_host(a, b, force_k: int = 0, device: int = 0, pow2: bool = False) -> np.ndarray:
    """Host-array convenience (copies in and out); for tests and tools."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
    out = np.zeros(len(a) + len(b), dtype=np.uint64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    rc = lib().dmul_host(int(device), a.ctypes.data_as(u64p), len(a), b.ctypes.data_as(u64p), len(b),
                         out.ctypes.data_as(u64p), flags_for(force_k, pow2))
    if rc:
        raise DmulError(rc, "dmul_host")
    return out


class PreparedBatch:
    """The marshalled arguments of one batch (host arrays of device
    pointers, sizes, spectra, statuses); keeps its tensors alive."""

    def __init__(self, pairs: Sequence, outs: Sequence):
        n = len(pairs)
        self.n = n
        self.A = (ctypes.c_void_p * n)()
        self.B = (ctypes.c_void_p * n)()
        self.SA = (ctypes.c_void_p * n)()
        self.SB = (ctypes.c_void_p * n)()
        self.O = (ctypes.c_void_p * n)()
        self.NA = (ctypes.c_size_t * n)()
        self.NB = (ctypes.c_size_t * n)()
        self.st = (ctypes.c_int32 * n)()
        self.spectra = False
        self._refs = (list(pairs), list(outs))
        for i, ((a, b), o) in enumerate(zip(pairs, outs)):
            for x, P, S, L in ((a, self.A, self.SA, self.NA), (b, self.B, self.SB, self.NB)):
                if isinstance(x, Spectrum):
                    S[i] = x._h.value
                    L[i] = x.na
                    self.spectra = True
                else:
                    P[i] = x.data_ptr() if x.numel() else 0
                    L[i] = x.numel()
            self.O[i] = o.data_ptr() if o.numel() else 0


_contexts: dict[int, Context] = {}


def _default_context(device: int) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]
