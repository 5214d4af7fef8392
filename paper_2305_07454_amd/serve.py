"""Serving loop over the device-resident stream state.

Chunks of records arrive as a Poisson process.  A chunk is admitted in FIFO
order when the device arena -- a ring of record slots reserved for chunks in
flight, carved at start-up from the device memory free then -- has room for it
(admission by free device memory).  Its columns are
copied host-to-device on a copy stream.  The compute stream runs one push at
a time.  With continuous batching, every chunk that is copied and waiting when
the compute stream frees up joins the next push (chunks that arrive while a
push runs overlap with it on the device).  With the per-chunk policy each push
takes one chunk.  Features go back device-to-host on a third stream.  A chunk's
latency is the time its features are in host memory minus its scheduled
arrival.  The loop (Server) drives the device through an executor (the
copies, the push, event polls), so that it can be exercised with a stand-in.

The host pool is replayed in cycles: cycle c shifts journey ids by c * 2^40,
so every cycle brings new journeys (each with its timestamps in order, which
is the arrival-order precondition) over the same grid cells and time bins.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np
import torch

from . import cvetl

JID_SHIFT = 1 << 40


@dataclasses.dataclass
class Chunk:
    cid: int
    src: int          # first pool record
    n: int
    cycle: int
    arrival: float    # seconds after start
    slot: int = -1    # first ring record
    copy_ev: object = None
    done_ev: object = None
    t_done: float = -1.0


def poisson_trace(rng, rate_fn, duration_s, sizes_lo, sizes_hi):
    """Arrival times of a non-homogeneous Poisson process (thinning) and
    log-uniform chunk sizes."""
    lam_max = max(rate_fn(t) for t in np.linspace(0, duration_s, 1001))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / lam_max)
        if t >= duration_s:
            break
        if rng.random() * lam_max <= rate_fn(t):
            size = int(math.exp(rng.uniform(math.log(sizes_lo), math.log(sizes_hi))))
            out.append((t, size))
    return out


# device bytes per arena record: the record columns (36) and the features (49)
# in the ring, plus the stream state's per-push scratch, which grows with the
# largest push (the arena); measured from the library's size query
_RING_BYTES = 36 + 49


def arena_from_free_hbm(grid, max_journeys, max_groups, fraction=0.5, cap=64_000_000, device="cuda"):
    """Records in the arena: the largest ring (with the stream state sized for
    pushes of the whole ring) that fits `fraction` of the device memory free
    now, at most `cap`."""
    free, _ = torch.cuda.mem_get_info(torch.device(device))
    base = cvetl.stream_state_bytes(grid, max_journeys, max_groups, 0)
    per = (cvetl.stream_state_bytes(grid, max_journeys, max_groups, 1 << 20) - base) / float(1 << 20) + _RING_BYTES
    a = int((fraction * free - base) / per)
    return max(1 << 20, min(cap, a))


class ServeError(RuntimeError):
    """A push (or its copies) failed; `cids` names the chunks of that push."""

    def __init__(self, msg, cids):
        super().__init__(msg)
        self.cids = list(cids)


class DeviceExecutor:
    """The device side of the serving loop: the pinned host pool, the device
    ring of record slots and feature slots, three streams (copies in, compute,
    copies out) and the resident stream state.  The loop (Server) only calls
    the methods below, each of which enqueues work or polls an event."""

    def __init__(self, pool, grid, arena_records, max_journeys, max_groups, device):
        self.dev = torch.device(device)
        self.A = int(arena_records)
        self.pool_n = pool.n
        self.h = {k: torch.from_numpy(np.ascontiguousarray(c)).pin_memory()
                  for (k, _), c in zip(cvetl.RECORD_FIELDS, pool.columns())}
        self.ring = {k: torch.empty(self.A, dtype=dt, device=self.dev) for k, dt in cvetl.RECORD_FIELDS}
        self.fring = {k: torch.empty(self.A, dtype=dt, device=self.dev) for k, dt in cvetl.FEATURE_FIELDS}
        self.hout = {k: torch.empty(self.A, dtype=dt).pin_memory() for k, dt in cvetl.FEATURE_FIELDS}
        self.s_copy = torch.cuda.Stream(self.dev)
        self.s_comp = torch.cuda.Stream(self.dev)
        self.s_back = torch.cuda.Stream(self.dev)
        self.stream = cvetl.Stream(grid, max_journeys, max_groups, self.A, device=self.dev, stream=self.s_comp)
        self.res = cvetl.new_result(self.dev)
        self._comp_ev = None

    def copy_in(self, c):
        with torch.cuda.stream(self.s_copy):
            a, b = c.src, c.src + c.n
            for k, _ in cvetl.RECORD_FIELDS:
                self.ring[k][c.slot:c.slot + c.n].copy_(self.h[k][a:b], non_blocking=True)
            if c.cycle:
                self.ring["journey_id"][c.slot:c.slot + c.n] += c.cycle * JID_SHIFT
            c.copy_ev = torch.cuda.Event()
            c.copy_ev.record(self.s_copy)

    def copy_done(self, c):
        return c.copy_ev.query()

    def compute_free(self):
        return self._comp_ev is None or self._comp_ev.query()

    def launch(self, batch):
        a = batch[0].slot
        n = sum(c.n for c in batch)
        assert a + n <= self.A
        for c in batch:
            self.s_comp.wait_event(c.copy_ev)
        rec = {k: v[a:a + n] for k, v in self.ring.items()}
        feat = {k: v[a:a + n] for k, v in self.fring.items()}
        self.stream.push(rec, feat=feat, res=self.res, stream=self.s_comp)
        ev = torch.cuda.Event()
        ev.record(self.s_comp)
        self.s_back.wait_event(ev)
        with torch.cuda.stream(self.s_back):
            for k in self.fring:
                self.hout[k][a:a + n].copy_(self.fring[k][a:a + n], non_blocking=True)
        done = torch.cuda.Event()
        done.record(self.s_back)
        for c in batch:
            c.done_ev = done
        self._comp_ev = ev

    def done(self, c):
        return c.done_ev.query()

    def features(self, c):
        return {k: v[c.slot:c.slot + c.n].clone() for k, v in self.hout.items()}

    def finish(self):
        torch.cuda.synchronize()

    def flush(self, jcap, gcap):
        with torch.cuda.stream(self.s_comp):
            out = self.stream.flush(jcap, gcap, stream=self.s_comp)
        torch.cuda.synchronize()
        return out


class Server:
    def __init__(self, pool, grid, batching=True, arena_records=None, max_journeys=1 << 21,
                 max_groups=1 << 23, device="cuda", executor=None, clock=time.perf_counter, sleep=time.sleep,
                 idle=None, max_push_records=None):
        """arena_records: records in the device ring; None carves it from the
        free HBM (arena_from_free_hbm).  Chunks are admitted into the ring in
        arrival order while it has room.  executor: the device side (a
        DeviceExecutor by default); clock / sleep / idle: the loop's time
        source, its wait for the next arrival, and what it does in a round
        that made no progress (nothing: it polls again).  max_push_records:
        the most records one push batches (a single larger chunk still goes
        alone); by default a quarter of the ring, so that while one push
        computes, the copies of the one before and of the next have ring
        space of their own."""
        self.grid = grid
        self.batching = batching
        if executor is None:
            if arena_records is None:
                arena_records = arena_from_free_hbm(grid, max_journeys, max_groups, device=device)
            executor = DeviceExecutor(pool, grid, arena_records, max_journeys, max_groups, device)
        self.ex = executor
        self.A = int(executor.A)
        self.max_push = int(max_push_records) if max_push_records else max(1, self.A // 4)
        self.pool_n = pool.n
        self.clock, self.sleep, self.idle = clock, sleep, idle
        self.keep = {}         # cid -> features copied out for checking

    def run(self, trace, keep_first=0, log=None):
        """Serve the trace (list of (arrival_s, size)); returns per-chunk records.
        A chunk larger than the ring can never be admitted: ValueError before
        anything is served.  A failed push raises ServeError naming its chunks;
        the chunks completed before it keep their completion times."""
        chunks, src, cyc = [], 0, 0
        for i, (t, size) in enumerate(trace):
            if size > self.A:
                raise ValueError(f"chunk {i} of {size} records exceeds the arena of {self.A}: never admissible")
            size = min(size, self.pool_n)
            if src + size > self.pool_n:
                src, cyc = 0, cyc + 1
            chunks.append(Chunk(i, src, size, cyc, t))
            src += size
        pending = collections.deque(chunks)
        copying = collections.deque()     # admitted, H2D issued
        inflight = collections.deque()    # admitted, not yet completed (ring order)
        launched = collections.deque()    # chunks launched, awaiting features on host
        t0 = self.clock()
        next_log = 1.0
        while pending or copying or launched:
            now = self.clock() - t0
            progress = False
            # admission (FIFO) by free arena space
            while pending and pending[0].arrival <= now:
                c = pending[0]
                slot = self._reserve_fifo(c.n, inflight)
                if slot < 0:
                    break
                c.slot = slot
                try:
                    self.ex.copy_in(c)
                except Exception as e:
                    raise ServeError(f"copy of chunk {c.cid} failed: {e}", [c.cid]) from e
                pending.popleft()
                copying.append(c)
                inflight.append(c)
                progress = True
            # launch when the compute stream is free
            if copying and self.ex.compute_free():
                ready = []
                nrec = 0
                while copying and self.ex.copy_done(copying[0]):
                    c = copying[0]
                    if ready and (c.slot != ready[-1].slot + ready[-1].n):
                        break          # not contiguous in the ring (wrapped): next push
                    if ready and nrec + c.n > self.max_push:
                        break          # the push is full: the rest goes in the next
                    nrec += c.n
                    ready.append(copying.popleft())
                    if not self.batching:
                        break
                if ready:
                    try:
                        self.ex.launch(ready)
                    except Exception as e:
                        raise ServeError(f"push of chunks {[c.cid for c in ready]} failed: {e}",
                                         [c.cid for c in ready]) from e
                    launched.extend(ready)
                    progress = True
            # completions (FIFO)
            while launched and self.ex.done(launched[0]):
                c = launched.popleft()
                c.t_done = self.clock() - t0
                if c.cid < keep_first:
                    self.keep[c.cid] = self.ex.features(c)
                inflight.popleft()
                progress = True
            if log and now >= next_log:
                log(f"t={now:.1f}s admitted={len(chunks) - len(pending)} done={sum(1 for c in chunks if c.t_done >= 0)}"
                    f" queue={len(pending)}")
                next_log += 1.0
            if not (copying or launched) and pending and pending[0].arrival > now:
                self.sleep(min(0.0005, pending[0].arrival - now))
            elif not progress and self.idle is not None:
                self.idle()
        self.ex.finish()
        return chunks

    def _reserve_fifo(self, n, inflight):
        """First ring record of a contiguous free range of n records after the
        newest chunk in flight (the ring is freed in FIFO order), or -1."""
        if n > self.A:
            raise ValueError(f"chunk of {n} records exceeds the arena of {self.A}")
        if not inflight:
            return 0
        lo = inflight[0].slot
        newest = inflight[-1]
        tail = newest.slot + newest.n
        if newest.slot >= lo:              # occupied [lo, tail): free [tail, A) and [0, lo)
            if tail + n <= self.A:
                return tail
            return 0 if n <= lo else -1
        return tail if tail + n <= lo else -1   # wrapped: free [tail, lo)

    def flush(self, jcap, gcap):
        return self.ex.flush(jcap, gcap)


def latency_stats(chunks, warmup_s=0.0):
    lat = np.array([c.t_done - c.arrival for c in chunks if c.arrival >= warmup_s and c.t_done >= 0])
    recs = sum(c.n for c in chunks if c.arrival >= warmup_s)
    t_first = min((c.arrival for c in chunks if c.arrival >= warmup_s), default=0.0)
    t_last = max((c.t_done for c in chunks), default=1.0)
    return {
        "chunks": int(lat.size),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p95_ms": round(float(np.percentile(lat, 95)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "max_ms": round(float(lat.max()) * 1e3, 3),
        "mrec_per_s": round(recs / max(t_last - t_first, 1e-9) / 1e6, 3),
    }
