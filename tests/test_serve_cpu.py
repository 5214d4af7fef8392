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
