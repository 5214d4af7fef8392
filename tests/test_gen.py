"""Generator: shapes, ranges, reproducibility and the stated rates (inputs only)."""
import numpy as np

from paper_2305_07454_amd import gen


def _check_box(r):
    assert r.lat_deg.min() >= gen.LAT_LO and r.lat_deg.max() < gen.LAT_HI
    assert r.lon_deg.min() >= gen.LON_LO and r.lon_deg.max() < gen.LON_HI
    assert r.speed_mps.dtype == np.float32 and r.speed_mps.min() >= 0 and r.speed_mps.max() < 40
    assert r.journey_id.dtype == np.int64 and r.journey_id.min() >= 0
    assert r.ts_ms.min() >= gen.T0_MS and r.ts_ms.max() < gen.T0_MS + gen.DAY_MS


def test_c0_shape_and_reproducible():
    a = gen.make_c0(seed=3, n_journeys=50)
    b = gen.make_c0(seed=3, n_journeys=50)
    for x, y in zip(a.columns(), b.columns()):
        assert np.array_equal(x, y)
    _check_box(a)
    u, c = np.unique(a.journey_id, return_counts=True)
    assert len(u) == 50 and c.min() >= 100 and c.max() <= 900
    zero = (a.speed_mps == 0).mean()
    assert 0.02 < zero < 0.09


def test_c1_rates_and_layout():
    r = gen.make_c1(seed=4, n_journeys=200, median=400.0)
    _check_box(r)
    # journeys come as contiguous blocks (per-journey files)
    change = np.count_nonzero(r.journey_id[1:] != r.journey_id[:-1])
    assert change == 199
    # within a block: ~5 % equal consecutive timestamps, ~2 % descending pairs
    same = r.journey_id[1:] == r.journey_id[:-1]
    d = np.diff(r.ts_ms)[same]
    assert 0.03 < (d == 0).mean() < 0.07
    assert 0.01 < (d < 0).mean() < 0.03
    # steps look like the stated walk: ~25 m, far below the box
    step = np.hypot(np.diff(r.lat_deg)[same], np.diff(r.lon_deg)[same])
    assert 1e-4 < np.median(step) < 4e-4


def test_c2_shard_sizes():
    s = gen.c2_shard_sizes()
    assert s.shape == (115,) and int(s.sum()) == 400_000_000
    assert s.max() == 20_000_000 and s.min() >= 10_000
    small = gen.c2_shard_sizes(n_shards=7, total=70_000, lo=1_000, hi=30_000)
    assert int(small.sum()) == 70_000
    shards = gen.make_c2(seed=9, n_shards=4, total=40_000, lo=1_000, hi=20_000)
    assert sum(x.n for x in shards) == 40_000
    for x in shards:
        _check_box(x)
        assert np.all(np.diff(x.ts_ms) >= 0)           # time-interleaved feed order


def test_fold_stays_in_box():
    x = np.array([35.0, 36.0, 40.6, 41.0, 45.2, 36.0 - 9.2])
    y = gen._fold(x, 36.0, 40.6)
    assert np.all(y >= 36.0) and np.all(y < 40.6)
    assert abs(y[0] - 37.0) < 1e-12 and abs(y[3] - 40.2) < 1e-12
