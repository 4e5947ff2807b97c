"""Serving loop: continuous batching of multiplication requests.

Requests arrive over time (each names its two operands as slices of a pool
of limbs resident in HBM).  The loop admits waiting requests in arrival
order while their device footprint -- the product's workspace
(dmul_workspace_bytes) plus its na + nb result limbs -- fits the budget of a
free engine, and launches the admitted set as one dmul_batch on that
engine's stream.  With two or more engines (each a dmul context with its own
HIP stream and workspace), a new batch is formed and launched while earlier
ones still run, so requests that arrive during a batch join the next one
instead of waiting for the device to drain: continuous batching, with the
work of successive batches overlapping on the device.

Each request's latency is the time from its arrival to the host observing
its batch complete (a HIP event on the engine's stream).  The loop is
argument marshalling and bookkeeping only; every product runs in the
library's kernels.

Failures stay with their request.  A request whose footprint alone exceeds
the engine budget is refused at admission (status DMUL_ENOMEM).  Each
engine's library context enforces the same budget.  A batch the library
refuses as a whole (DMUL_ENOMEM from the workspace budget or an allocation,
or an argument error) is split, and each of its requests is run again alone;
a request that fails alone, or whose own product fails (DMUL_EDIGIT for a
limb >= 10^19), is reported with its status and the loop goes on.  Only a
device error (DMUL_EDEVICE) ends the loop.

Transforms can stay resident too: with a spectrum cache, an operand that
comes back (the same pool slice, in a product of the same plan k and N)
gets its forward transforms cached as a dmul spectrum, and later products
with it skip those passes (dmul_batch_ex).  The cache is an LRU bounded in
bytes; a spectrum made on one engine's stream is used on the other only
after an event that orders the two.
"""
from __future__ import annotations

import ctypes
import gc
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

from . import (DMUL_EDEVICE, DMUL_ENOMEM, Context, DmulError, lib, plan, spectrum_bytes, torch,
               workspace_bytes)


@dataclass
class Request:
    rid: int
    a_off: int          # limb offset of operand a in the pool
    na: int             # limbs of a
    b_off: int
    nb: int
    arrival: float      # seconds after the start of the run
    da: int = 0         # requested decimal digits of a and b (0: 19 per limb)
    db: int = 0

    def digits(self) -> int:
        return (self.da or 19 * self.na) + (self.db or 19 * self.nb)


@dataclass
class ServeStats:
    completed: int = 0
    digits: int = 0
    wall_s: float = 0.0
    batches: int = 0
    latencies_s: list = field(default_factory=list)
    max_inflight_bytes: int = 0
    max_overlap: int = 0        # largest number of batches in flight at once
    max_batch_bytes: int = 0    # largest footprint of one batch (at most the engine budget)
    spectrum_hits: int = 0      # operands taken from cached transforms
    spectra_made: int = 0
    failed: dict = field(default_factory=dict)   # rid -> status of requests that failed
    retried: int = 0            # requests run again alone after their batch was refused

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_s, dtype=float) * 1e3
        return {
            "requests": self.completed,
            "batches": self.batches,
            "digits": self.digits,
            "wall_s": self.wall_s,
            "digits_per_s": self.digits / self.wall_s if self.wall_s > 0 else None,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_batch": self.completed / self.batches if self.batches else 0,
            "max_inflight_bytes": self.max_inflight_bytes,
            "max_batch_bytes": self.max_batch_bytes,
            "max_batches_in_flight": self.max_overlap,
            "spectrum_hits": self.spectrum_hits,
            "spectra_made": self.spectra_made,
            "failed": len(self.failed),
            "retried_alone": self.retried,
        }


class _Engine:
    """One dmul context with its own stream; at most one batch in flight."""

    def __init__(self, device: int, budget: int, ctx_budget: int):
        self.stream = torch.cuda.Stream(device=device)
        # the library enforces the workspace budget itself
        self.ctx = Context(device, budget_bytes=ctx_budget, stream=self.stream)
        self.budget = budget
        self.busy = None            # (event, requests, out buffer, bytes) of the batch in flight

    def close(self):
        self.ctx.close()


class Server:
    """Continuous-batching server over a resident operand pool.

    pool: 1-D torch.uint64 CUDA tensor of limbs; requests reference slices.
    engines: number of contexts/streams (>= 2 lets batches overlap).
    budget_bytes: device footprint one engine may hold in flight.
    max_batch: most requests per batch.
    spectrum_cache_bytes: device memory for cached transforms of operands
        that come back (0 = none).
    spectrum_min_len: the shortest transform length worth caching: making a
        spectrum costs host work and two launches of its own, which pays off
        only where a forward transform is long.
    ctx_budget_bytes: the workspace budget of each engine's library context
        (default: budget_bytes).
    """

    def __init__(self, pool, device: int = 0, engines: int = 2, budget_bytes: int = 8 << 30,
                 max_batch: int = 1024, spectrum_cache_bytes: int = 0, spectrum_min_len: int = 1 << 19,
                 ctx_budget_bytes: int | None = None):
        self.pool = pool
        self.device = device
        cb = budget_bytes if ctx_budget_bytes is None else ctx_budget_bytes
        self.engines = [_Engine(device, budget_bytes, cb) for _ in range(max(1, engines))]
        self.max_batch = max_batch
        self._base = pool.data_ptr()
        self.spec_cap = int(spectrum_cache_bytes)
        self.spec_min = int(spectrum_min_len)
        self._spectra = OrderedDict()   # (offset, limbs, k, N) -> [Spectrum, bytes, event, stream]
        self._spec_bytes = 0
        self._seen = {}                 # operand key -> times used
        self._seen_cap = 1 << 20
        self._stats = None
        lib()

    def close(self):
        for e in self.engines:
            e.close()

    @staticmethod
    def footprint(na: int, nb: int) -> int:
        return workspace_bytes(na, nb) + 8 * (na + nb)

    def _operand_spectrum(self, eng: _Engine, off: int, n: int, partner: int, pl):
        """The cached transforms of pool[off: off + n] for plan pl, made now
        (on eng's stream) if this operand has been used before; or None."""
        if not self.spec_cap or pl.N < self.spec_min:
            return None
        key = (off, n, pl.k, pl.N)
        ent = self._spectra.get(key)
        if ent is not None:
            self._spectra.move_to_end(key)
            if ent[3] is not eng.stream:
                eng.stream.wait_event(ent[2])
                ent[0].mem.record_stream(eng.stream)
            self._stats.spectrum_hits += 1
            return ent[0]
        seen = self._seen.get(key, 0)
        if len(self._seen) >= self._seen_cap:   # forget old sightings in a long run
            self._seen.clear()
        self._seen[key] = seen + 1
        nbytes = spectrum_bytes(n, partner)
        if seen == 0 or nbytes > self.spec_cap:
            return None
        while self._spectra and self._spec_bytes + nbytes > self.spec_cap:
            _, old = self._spectra.popitem(last=False)
            self._spec_bytes -= old[1]
        with torch.cuda.stream(eng.stream):      # from torch's caching allocator, no hipMalloc
            mem = torch.empty(nbytes // 8, dtype=torch.uint64, device=f"cuda:{self.device}")
        spec = eng.ctx.spectrum(self.pool[off: off + n], partner, mem=mem)
        ev = torch.cuda.Event()
        ev.record(eng.stream)
        self._spectra[key] = [spec, nbytes, ev, eng.stream]
        self._spec_bytes += nbytes
        self._stats.spectra_made += 1
        return spec

    def _launch(self, eng: _Engine, reqs: list, keep_outputs: bool):
        """Enqueue one batch: output buffer, dmul_batch, completion event."""
        total = sum(r.na + r.nb for r in reqs)
        with torch.cuda.stream(eng.stream):
            out = torch.empty(total, dtype=torch.uint64, device=f"cuda:{self.device}")
        n = len(reqs)
        A = (ctypes.c_void_p * n)()
        B = (ctypes.c_void_p * n)()
        SA = (ctypes.c_void_p * n)()
        SB = (ctypes.c_void_p * n)()
        O = (ctypes.c_void_p * n)()
        NA = (ctypes.c_size_t * n)()
        NB = (ctypes.c_size_t * n)()
        st = (ctypes.c_int32 * n)()
        base, optr, ofs = self._base, out.data_ptr(), 0
        used = []
        for i, r in enumerate(reqs):
            A[i] = base + 8 * r.a_off
            B[i] = base + 8 * r.b_off
            NA[i] = r.na
            NB[i] = r.nb
            O[i] = optr + 8 * ofs
            ofs += r.na + r.nb
            if self.spec_cap:
                pl = plan(r.na, r.nb)
                sa = self._operand_spectrum(eng, r.a_off, r.na, r.nb, pl)
                sb = (sa if (r.b_off, r.nb) == (r.a_off, r.na)
                      else self._operand_spectrum(eng, r.b_off, r.nb, r.na, pl))
                if sa is not None:
                    SA[i] = sa._h.value
                    used.append(sa)
                if sb is not None:
                    SB[i] = sb._h.value
                    used.append(sb)
        if used:
            rc = eng.ctx._lib.dmul_batch_ex(eng.ctx._h, n, A, NA, SA, B, NB, SB, O, st, 0)
        else:
            rc = eng.ctx._lib.dmul_batch(eng.ctx._h, n, A, NA, B, NB, O, st, 0)
        if rc == DMUL_EDEVICE:
            raise DmulError(rc, "dmul_batch")
        if rc:
            # refused as a whole (nothing enqueued): every request is run
            # again alone, or fails with this status if it already was alone
            self._refused(reqs, rc)
            return False
        ev = torch.cuda.Event()
        ev.record(eng.stream)
        nbytes = sum(self.footprint(r.na, r.nb) for r in reqs)
        eng.busy = (ev, reqs, out if keep_outputs else None, nbytes, (A, B, O, NA, NB, st, SA, SB, used))
        return True

    def _refused(self, reqs: list, rc: int):
        """Requests whose batch the library refused (rc): alone again, or
        failed if they were alone."""
        if len(reqs) == 1:
            self._fail(reqs[0], rc)
            return
        for r in reversed(reqs):
            self._alone.appendleft(r)
        self._stats.retried += len(reqs)

    def _fail(self, r: Request, rc: int):
        self._stats.failed[r.rid] = int(rc)
        self._stats.completed += 1

    def _retire(self, eng: _Engine, t0: float, stats: ServeStats, results: dict | None):
        ev, reqs, out, nbytes, keep = eng.busy
        eng.busy = None
        now = time.perf_counter() - t0
        rc = eng.ctx._lib.dmul_sync(eng.ctx._h)      # stream already idle: returns at once
        if rc:
            raise DmulError(rc, "dmul_sync")      # a device error: nothing is trustworthy
        st = keep[5]
        ofs, refused = 0, []
        for i, r in enumerate(reqs):
            if st[i] == DMUL_ENOMEM and len(reqs) > 1:
                refused.append(r)                 # the batch's workspace: run it alone
            elif st[i] != 0:
                self._fail(r, st[i])
            else:
                stats.latencies_s.append(now - r.arrival)
                stats.digits += r.digits()
                stats.completed += 1
                if results is not None and out is not None:
                    results[r.rid] = out[ofs: ofs + r.na + r.nb]
            ofs += r.na + r.nb
        if refused:
            self._refused(refused, DMUL_ENOMEM)

    def run(self, reqs: list, keep_outputs: bool = False, realtime: bool = True) -> tuple[ServeStats, dict]:
        """Serve `reqs` (sorted by arrival).  With realtime, a request is
        admitted only once its arrival time has passed; otherwise all are
        available at once.  Returns the statistics and, with keep_outputs,
        {rid: result tensor}."""
        stats = ServeStats()
        self._stats = stats
        # the cyclic garbage collector, run over the many request objects of
        # a long stream, pauses the loop for tens of milliseconds at a time
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(reqs, stats, keep_outputs, realtime)
        finally:
            if gc_was_on:
                gc.enable()

    def _run(self, reqs: list, stats: ServeStats, keep_outputs: bool, realtime: bool):
        results = {} if keep_outputs else None
        nxt = 0                      # next request not yet admitted
        self._alone = deque()        # requests to run again, each alone
        t0 = time.perf_counter()
        while stats.completed < len(reqs):
            now = time.perf_counter() - t0
            for eng in self.engines:
                if eng.busy is not None and eng.busy[0].query():
                    self._retire(eng, t0, stats, results)
            inflight = sum(1 for e in self.engines if e.busy is not None)
            launched = False
            for eng in self.engines:
                if eng.busy is not None:
                    continue
                if self._alone:
                    batch = [self._alone.popleft()]
                else:
                    if nxt >= len(reqs) or (realtime and reqs[nxt].arrival > now):
                        break
                    batch, used = [], 0
                    while (nxt < len(reqs) and len(batch) < self.max_batch
                           and (not realtime or reqs[nxt].arrival <= now)):
                        r = reqs[nxt]
                        fp = self.footprint(r.na, r.nb)
                        if fp > eng.budget:           # can never fit: refused, not admitted
                            self._fail(r, DMUL_ENOMEM)
                            nxt += 1
                            continue
                        if used + fp > eng.budget:
                            break
                        batch.append(r)
                        used += fp
                        nxt += 1
                    if not batch:
                        continue
                if not self._launch(eng, batch, keep_outputs):
                    continue
                stats.batches += 1
                inflight += 1
                stats.max_overlap = max(stats.max_overlap, inflight)
                stats.max_inflight_bytes = max(
                    stats.max_inflight_bytes, sum(e.busy[3] for e in self.engines if e.busy is not None))
                stats.max_batch_bytes = max(stats.max_batch_bytes, eng.busy[3])
                launched = True
            if not launched:
                if (all(e.busy is None for e in self.engines) and nxt < len(reqs) and realtime
                        and not self._alone):
                    wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(2e-5)
        stats.wall_s = time.perf_counter() - t0
        return stats, (results or {})


def make_requests(lengths_a, lengths_b, arrivals, pool_limbs: int, seed: int = 5008) -> list:
    """Requests whose operands are random slices of a pool of `pool_limbs`
    limbs (digit lengths rounded up to whole limbs)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i, (da, db, t) in enumerate(zip(lengths_a, lengths_b, arrivals)):
        na = max(1, (int(da) + 18) // 19)
        nb = max(1, (int(db) + 18) // 19)
        ao = int(rng.integers(0, pool_limbs - na + 1))
        bo = int(rng.integers(0, pool_limbs - nb + 1))
        reqs.append(Request(i, ao, na, bo, nb, float(t), max(1, int(da)), max(1, int(db))))
    return reqs
