"""Host logic of the serving loop, on the CPU: the arrival process, FIFO
admission into the device ring, and the latency statistics."""
import types

import numpy as np

from paper_2305_07454_amd import serve


def _ring(A):
    return types.SimpleNamespace(A=A)


def _chunk(slot, n):
    return serve.Chunk(cid=0, src=0, n=n, cycle=0, arrival=0.0, slot=slot)


def test_poisson_trace_rate_and_sizes():
    rng = np.random.default_rng(1)
    tr = serve.poisson_trace(rng, lambda t: 200.0, 20.0, 10_000, 5_000_000)
    assert 3600 < len(tr) < 4400
    sizes = np.array([s for _, s in tr])
    assert sizes.min() >= 10_000 and sizes.max() <= 5_000_000
    # log-uniform: median near sqrt(lo * hi)
    assert 150_000 < np.median(sizes) < 330_000
    t = np.array([a for a, _ in tr])
    assert np.all(np.diff(t) > 0)


def test_poisson_trace_burst_thinning():
    rng = np.random.default_rng(2)
    tr = serve.poisson_trace(rng, lambda t: 1000.0 if 10 <= t < 20 else 200.0, 30.0, 10, 20)
    t = np.array([a for a, _ in tr])
    mid = ((t >= 10) & (t < 20)).sum()
    side = ((t < 10) | (t >= 20)).sum()
    assert 8500 < mid < 11500 and 3400 < side < 4600


def test_ring_reservation_fifo():
    r = _ring(100)
    res = lambda n, inflight: serve.Server._reserve_fifo(r, n, inflight)  # noqa: E731
    assert res(40, []) == 0
    a = _chunk(0, 40)
    assert res(50, [a]) == 40
    b = _chunk(40, 50)
    assert res(20, [a, b]) == -1           # only 10 left at the end, oldest holds [0, 40)
    assert res(10, [a, b]) == 90
    # oldest done: free [0, 40) again; the tail is too short so it wraps
    assert res(30, [b]) == 0
    c = _chunk(0, 30)
    assert res(10, [b, c]) == 30           # wrapped: free [30, 40)
    assert res(11, [b, c]) == -1
    try:
        res(101, [])
        assert False
    except ValueError:
        pass


def test_latency_stats():
    cs = []
    for i in range(100):
        c = _chunk(0, 1000)
        c.arrival = i * 0.01
        c.t_done = c.arrival + (0.001 if i % 10 else 0.05)
        cs.append(c)
    st = serve.latency_stats(cs, warmup_s=0.0)
    assert st["chunks"] == 100
    assert abs(st["p50_ms"] - 1.0) < 1e-6 and st["max_ms"] == 50.0
    assert st["p99_ms"] > 40.0


# ---------------------------------------------------------------------------
# The loop against a stand-in executor on a virtual clock: forced failures,
# admission that has to wait for ring space, a slow push.
# ---------------------------------------------------------------------------
class _Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 1e-6)

    def tick(self):
        self.t += 1e-5


class _FakeExecutor:
    """Copies take copy_s, a push takes rec_s per record (plus slow_s when
    it holds chunk slow_cid), results land copy_s after the push; the push that
    holds chunk fail_cid raises.  Ring use is checked on every admission."""

    def __init__(self, A, clock, copy_s=1e-3, rec_s=1e-8, fail_cid=None, slow_cid=None, slow_s=0.2):
        self.A, self.clock = A, clock
        self.copy_s, self.rec_s = copy_s, rec_s
        self.fail_cid, self.slow_cid, self.slow_s = fail_cid, slow_cid, slow_s
        self.busy_until = 0.0
        self.live = []        # chunks admitted and not completed
        self.batches = []     # cids per push, in order
        self.admitted_at = {}

    def copy_in(self, c):
        assert 0 <= c.slot and c.slot + c.n <= self.A
        for o in self.live:   # no two chunks in flight share a ring record
            assert c.slot + c.n <= o.slot or o.slot + o.n <= c.slot, (c.cid, o.cid)
        self.live.append(c)
        self.admitted_at[c.cid] = self.clock.now()
        c.copy_ready = self.clock.now() + self.copy_s

    def copy_done(self, c):
        return self.clock.now() >= c.copy_ready

    def compute_free(self):
        return self.clock.now() >= self.busy_until

    def launch(self, batch):
        cids = [c.cid for c in batch]
        if self.fail_cid in cids:
            raise RuntimeError("device push failed")
        dur = sum(c.n for c in batch) * self.rec_s + (self.slow_s if self.slow_cid in cids else 0.0)
        self.busy_until = self.clock.now() + dur
        for c in batch:
            c.done_at = self.busy_until + self.copy_s
        self.batches.append(cids)

    def done(self, c):
        if self.clock.now() >= c.done_at:
            if c in self.live:
                self.live.remove(c)
            return True
        return False

    def features(self, c):
        return {"n": c.n}

    def finish(self):
        pass


def _server(ex, clock, batching=True):
    pool = types.SimpleNamespace(n=10 ** 9)
    return serve.Server(pool, None, batching=batching, executor=ex, clock=clock.now, sleep=clock.sleep,
                        idle=clock.tick)


def test_fake_executor_batches_fifo():
    clock = _Clock()
    ex = _FakeExecutor(10 ** 7, clock, rec_s=2e-8)
    trace = [(i * 0.001, 100_000 + 1000 * (i % 7)) for i in range(200)]
    chunks = _server(ex, clock).run(trace, keep_first=3)
    done = [c.t_done for c in chunks]
    assert all(t >= 0 for t in done)
    assert all(b >= a for a, b in zip(done, done[1:]))                 # FIFO completion
    assert [c for b in ex.batches for c in b] == list(range(200))       # every chunk once, in order
    assert max(len(b) for b in ex.batches) > 1                         # continuous batching joined chunks
    assert all(c.t_done - c.arrival >= 2 * ex.copy_s - 1e-12 for c in chunks)


def test_fake_executor_per_chunk_pushes():
    clock = _Clock()
    ex = _FakeExecutor(10 ** 7, clock, rec_s=2e-8)
    trace = [(i * 0.001, 100_000) for i in range(50)]
    _server(ex, clock, batching=False).run(trace)
    assert ex.batches == [[i] for i in range(50)]


def test_admission_waits_for_ring_space():
    # a ring of 100 records and chunks of 60: a chunk is admitted only once the
    # one before it has completed and freed its records
    clock = _Clock()
    ex = _FakeExecutor(100, clock, rec_s=1e-4)
    trace = [(0.0, 60), (0.0, 60), (0.0, 60)]
    chunks = _server(ex, clock).run(trace)
    for a, b in zip(chunks, chunks[1:]):
        assert ex.admitted_at[b.cid] >= a.t_done - 1e-9
    assert ex.batches == [[0], [1], [2]]


def test_chunk_larger_than_the_ring_is_refused():
    clock = _Clock()
    ex = _FakeExecutor(100, clock)
    try:
        _server(ex, clock).run([(0.0, 50), (0.0, 101)])
        assert False, "a chunk that can never fit must be refused"
    except ValueError as e:
        assert "chunk 1" in str(e)
    assert ex.batches == []                                            # nothing was served


def test_exception_mid_batch_names_its_chunks():
    clock = _Clock()
    ex = _FakeExecutor(10 ** 7, clock, rec_s=1e-7, fail_cid=30)
    trace = [(i * 0.001, 50_000) for i in range(60)]
    srv = _server(ex, clock)
    try:
        srv.run(trace)
        assert False, "the failed push must surface"
    except serve.ServeError as e:
        assert 30 in e.cids
        served = [c for b in ex.batches for c in b]
        assert served == list(range(min(e.cids)))                      # everything before it was pushed
        assert "30" in str(e)


def test_slow_batch_delays_later_chunks_in_order():
    clock = _Clock()
    ex = _FakeExecutor(10 ** 7, clock, rec_s=1e-8, slow_cid=20, slow_s=0.2)
    trace = [(i * 0.002, 40_000) for i in range(100)]
    chunks = _server(ex, clock).run(trace)
    lat = {c.cid: c.t_done - c.arrival for c in chunks}
    assert all(c.t_done >= 0 for c in chunks)
    assert all(b.t_done >= a.t_done for a, b in zip(chunks, chunks[1:]))
    assert lat[20] >= 0.2 and lat[5] < 0.01                            # the slow push and one before it
    # chunks that arrived during the slow push went out together in the next one
    i = next(k for k, b in enumerate(ex.batches) if 20 in b)
    assert len(ex.batches[i + 1]) > 10
    st = serve.latency_stats(chunks)
    assert st["max_ms"] >= 200.0
    assert max(lat[k] for k in range(20)) < 0.01                      # before the slow push: unaffected
    # the backlog drains: the last chunk waits less than the one right after the slow push
    assert lat[99] < lat[21]


def test_push_size_is_capped_under_backlog():
    # a backlog of small chunks: every push stays within the cap (a quarter
    # of the ring by default) and the chunks still complete in FIFO order
    clock = _Clock()
    A = 4_000_000
    ex = _FakeExecutor(A, clock, rec_s=5e-8)
    trace = [(0.0, 150_000) for _ in range(120)]
    srv = _server(ex, clock)
    assert srv.max_push == A // 4
    chunks = srv.run(trace)
    sizes = {c.cid: c.n for c in chunks}
    assert [c for b in ex.batches for c in b] == list(range(120))
    assert all(sum(sizes[c] for c in b) <= A // 4 for b in ex.batches)
    assert max(len(b) for b in ex.batches) == (A // 4) // 150_000
    done = [c.t_done for c in chunks]
    assert all(b >= a for a, b in zip(done, done[1:]))


def test_chunk_above_the_push_cap_goes_alone():
    clock = _Clock()
    ex = _FakeExecutor(4_000_000, clock)
    trace = [(0.0, 100_000), (0.0, 2_000_000), (0.0, 100_000)]
    _server(ex, clock).run(trace)
    assert [1] in ex.batches and all(len(b) == 1 or 1 not in b for b in ex.batches)
