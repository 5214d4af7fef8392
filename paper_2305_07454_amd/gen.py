"""Seeded synthetic connected-vehicle record generator.

This module only draws inputs.  It holds none of the ETL method's arithmetic
(no sorting by journey, no kinematics, no binning, no aggregation), so both the
HIP path and the CPU oracle may take their inputs from it.

The record shape follows the paper's dataset description (Methods, "Connected
Vehicle Dataset", and Table 1): one row per sensor sample with a journey
identifier, a timestamp, latitude, longitude and speed.  The real Missouri DOT
data is not public; these workloads stand in for it:

* box: latitude [36.0, 40.6), longitude [-95.8, -89.1) (Missouri);
* vehicles: random walks, per-axis steps N(0, (2e-4 deg)^2), reflected at the
  box edges (implemented as a fold of the free walk, which equals per-step
  reflection because every step is far smaller than the box);
* time: 1 Hz samples (20 Hz for the heavy journeys of the skewed stream, the
  0.05 s resolution the paper states), inside one day starting at
  2021-05-09T00:00:00Z (the date of the sample rows in Table 1);
* speed: float32 uniform on [0, 40) m/s with 5 % exact zeros (stopped cars);
* journey ids: distinct random non-negative 63-bit integers (stand-ins for
  hashed string ids such as "33456rd").
"""
from __future__ import annotations

import dataclasses
import numpy as np

T0_MS = 1_620_518_400_000          # 2021-05-09T00:00:00Z in ms since the epoch
DAY_MS = 86_400_000
LAT_LO, LAT_HI = 36.0, 40.6
LON_LO, LON_HI = -95.8, -89.1
WALK_SIGMA_DEG = 2e-4
SEED_BASE = 230507454


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """Spatio-temporal binning parameters (Algorithm 2's origin and steps)."""
    lat0_deg: float
    lon0_deg: float
    dlat_deg: float
    dlon_deg: float
    n_lat: int
    n_lon: int
    t0_ms: int
    bin_ms: int
    n_t: int            # <= 0: unbounded number of time bins

    def as_tuple(self):
        return dataclasses.astuple(self)


def grid_for(step_deg: float, bin_ms: int, n_t: int | None = None) -> GridSpec:
    n_lat = int(round((LAT_HI - LAT_LO) / step_deg))
    n_lon = int(round((LON_HI - LON_LO) / step_deg))
    if n_t is None:
        n_t = DAY_MS // bin_ms
    return GridSpec(LAT_LO, LON_LO, step_deg, step_deg, n_lat, n_lon, T0_MS, bin_ms, n_t)


GRIDS = {
    "c0": grid_for(0.01, 15 * 60_000),
    "c1": grid_for(0.005, 5 * 60_000),
    "c2": grid_for(0.001, 60_000),
    "c3": grid_for(0.005, 5 * 60_000, n_t=0),
    "c4": grid_for(0.001, 60_000, n_t=0),
}


@dataclasses.dataclass
class Records:
    """Structure-of-arrays record batch (host numpy arrays)."""
    journey_id: np.ndarray   # int64
    ts_ms: np.ndarray        # int64
    lat_deg: np.ndarray      # float64
    lon_deg: np.ndarray      # float64
    speed_mps: np.ndarray    # float32
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.journey_id.shape[0])

    def take(self, idx) -> "Records":
        return Records(self.journey_id[idx], self.ts_ms[idx], self.lat_deg[idx],
                       self.lon_deg[idx], self.speed_mps[idx], dict(self.meta))

    def columns(self):
        return (self.journey_id, self.ts_ms, self.lat_deg, self.lon_deg, self.speed_mps)


def concat(parts) -> Records:
    parts = list(parts)
    return Records(*(np.concatenate([p.columns()[i] for p in parts]) for i in range(5)))


def rng_for(config_index: int, seed: int | None = None) -> np.random.Generator:
    s = SEED_BASE + config_index if seed is None else seed
    return np.random.default_rng(np.random.SeedSequence(s))


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def _fold(x, lo, hi):
    """Reflect a free walk into [lo, hi)."""
    w = hi - lo
    m = np.mod(x - lo, 2.0 * w)
    y = lo + (w - np.abs(m - w))
    np.clip(y, lo, np.nextafter(hi, lo), out=y)
    return y


def journey_ids(rng, n_journeys: int) -> np.ndarray:
    ids = np.unique(rng.integers(0, 2**63 - 1, size=n_journeys, dtype=np.int64))
    while ids.shape[0] < n_journeys:            # collisions are ~impossible; keep it exact anyway
        extra = rng.integers(0, 2**63 - 1, size=n_journeys - ids.shape[0], dtype=np.int64)
        ids = np.unique(np.concatenate([ids, extra]))
    return rng.permutation(ids)


def speeds(rng, n: int, zero_frac: float = 0.05) -> np.ndarray:
    s = rng.uniform(0.0, 40.0, size=n).astype(np.float32)
    np.minimum(s, np.nextafter(np.float32(40.0), np.float32(0.0)), out=s)
    s[rng.random(n) < zero_frac] = np.float32(0.0)
    return s


def walks(rng, lengths: np.ndarray, period_ms: int = 1000, day_start_ms: int = T0_MS,
          start_ms: np.ndarray | None = None):
    """Per-journey random walks, journeys laid out contiguously in time order.

    Returns (ts, lat, lon, offsets) where offsets[j] is the first row of journey j.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    j = lengths.shape[0]
    n = int(lengths.sum())
    offsets = np.zeros(j + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    heads = offsets[:-1]
    lat_start = rng.uniform(LAT_LO, LAT_HI, size=j)
    lon_start = rng.uniform(LON_LO, LON_HI, size=j)
    if start_ms is None:
        span = (lengths - 1) * period_ms
        slack = np.maximum(DAY_MS - span, 1) // 1000          # whole seconds of slack in the day
        start_ms = day_start_ms + 1000 * (rng.random(j) * slack).astype(np.int64)
    pos = np.arange(n, dtype=np.int64) - np.repeat(heads, lengths)
    ts = np.repeat(np.asarray(start_ms, dtype=np.int64), lengths) + period_ms * pos
    out = []
    for start, lo, hi in ((lat_start, LAT_LO, LAT_HI), (lon_start, LON_LO, LON_HI)):
        d = rng.normal(0.0, WALK_SIGMA_DEG, size=n)
        d[heads] = 0.0
        c = np.cumsum(d)
        free = np.repeat(start, lengths) + (c - np.repeat(c[heads], lengths))
        del c, d
        out.append(_fold(free, lo, hi))
        del free
    return ts, out[0], out[1], offsets


def _block_order(rng, offsets: np.ndarray) -> np.ndarray:
    """Row order that concatenates journey blocks in a seeded random order."""
    lengths = np.diff(offsets)
    order = rng.permutation(lengths.shape[0])
    new_len = lengths[order]
    new_off = np.zeros(order.shape[0] + 1, dtype=np.int64)
    np.cumsum(new_len, out=new_off[1:])
    src_start = np.repeat(offsets[:-1][order], new_len)
    return src_start + (np.arange(int(new_off[-1]), dtype=np.int64) - np.repeat(new_off[:-1], new_len))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def make_c0(seed=None, n_journeys=2000, min_len=100, max_len=900) -> Records:
    """Small plain workload: uniform lengths, fully shuffled rows."""
    rng = rng_for(0, seed)
    lengths = rng.integers(min_len, max_len + 1, size=n_journeys)
    ids = journey_ids(rng, n_journeys)
    ts, lat, lon, offsets = walks(rng, lengths)
    spd = speeds(rng, ts.shape[0])
    jid = np.repeat(ids, lengths)
    perm = rng.permutation(ts.shape[0])
    r = Records(jid[perm], ts[perm], lat[perm], lon[perm], spd[perm],
                dict(config="c0", n_journeys=n_journeys, layout="shuffled"))
    return r


def c1_lengths(rng, n_journeys, median=1500.0, sigma=1.0, cap=86_400):
    L = np.rint(rng.lognormal(np.log(median), sigma, size=n_journeys)).astype(np.int64)
    return np.clip(L, 1, cap)


def make_c1(seed=None, n_journeys=50_000, median=1500.0, cap=86_400, dup_frac=0.05,
            swap_frac=0.02, shuffled=False) -> Records:
    """Full-day plain workload: lognormal lengths, per-journey files in random
    order, 5 % duplicated timestamps and 2 % rows swapped with their successor."""
    rng = rng_for(1, seed)
    lengths = c1_lengths(rng, n_journeys, median=median, cap=cap)
    ids = journey_ids(rng, n_journeys)
    ts, lat, lon, offsets = walks(rng, lengths)
    n = ts.shape[0]
    spd = speeds(rng, n)
    jid = np.repeat(ids, lengths)
    # duplicated timestamps: a non-first sample takes its predecessor's time stamp
    is_head = np.zeros(n, dtype=bool)
    is_head[offsets[:-1]] = True
    dup = (rng.random(n) < dup_frac) & ~is_head
    idx = np.nonzero(dup)[0]
    ts_orig = ts.copy()
    ts[idx] = ts_orig[idx - 1]
    del ts_orig
    # out-of-order rows: swap a row with its journey successor (non-overlapping swaps)
    is_last = np.zeros(n, dtype=bool)
    is_last[offsets[1:] - 1] = True
    cand = (rng.random(n) < swap_frac) & ~is_last
    cand[1:] &= ~cand[:-1]
    a = np.nonzero(cand)[0]
    order = np.arange(n, dtype=np.int64)
    order[a], order[a + 1] = a + 1, a
    if shuffled:
        order = order[rng.permutation(n)]
    else:
        order = order[_block_order(rng, offsets)]
    r = Records(jid[order], ts[order], lat[order], lon[order], spd[order],
                dict(config="c1", n_journeys=n_journeys,
                     layout="shuffled" if shuffled else "journey files, random order"))
    return r


def c2_shard_sizes(n_shards=115, total=400_000_000, lo=10_000, hi=20_000_000, alpha=1.2,
                   seed=None):
    """Capped rank-size (Zipf) shard sizes summing to `total`, in a seeded shard order."""
    k = np.arange(1, n_shards + 1, dtype=np.float64)

    def sizes(c):
        return np.minimum(hi, np.maximum(lo, np.rint(c * k ** -alpha))).astype(np.int64)

    a, b = 1.0, float(total) * 10
    for _ in range(200):
        mid = 0.5 * (a + b)
        if sizes(mid).sum() < total:
            a = mid
        else:
            b = mid
    s = sizes(b)
    s[-1] += total - int(s.sum())              # land exactly on the total
    rng = rng_for(2, seed)
    return s[rng.permutation(n_shards)]


def make_shard(rng, n_records: int, period_ms=1000, mean_journey=1200.0, cap=86_400) -> Records:
    """One county-day shard: Poisson journey count, lognormal length weights,
    time-interleaved feed order."""
    j = max(1, int(rng.poisson(n_records / mean_journey)))
    j = min(j, n_records)
    w = rng.lognormal(0.0, 1.0, size=j)
    exact = w / w.sum() * n_records
    L = np.floor(exact).astype(np.int64)
    L = np.maximum(L, 1)
    rem = n_records - int(L.sum())
    if rem > 0:
        frac_order = np.argsort(-(exact - np.floor(exact)), kind="stable")
        L[frac_order[:rem]] += 1
    while int(L.sum()) > n_records:           # only when the floor-at-1 pushed us over
        i = int(np.argmax(L))
        L[i] -= int(L.sum()) - n_records
        L[i] = max(L[i], 1)
    L = np.minimum(L, cap)
    ids = journey_ids(rng, j)
    ts, lat, lon, offsets = walks(rng, L, period_ms=period_ms)
    spd = speeds(rng, ts.shape[0])
    jid = np.repeat(ids, L)
    order = feed_order(rng, ts)
    return Records(jid[order], ts[order], lat[order], lon[order], spd[order],
                   dict(n_journeys=j))


def feed_order(rng, ts):
    """Feed (arrival) order: by time stamp, ties in random order (one sort of
    the time offset with 32 random bits below it)."""
    t = ts - ts.min() if ts.shape[0] else ts
    assert ts.shape[0] == 0 or int(t.max()) < (1 << 31)
    key = (t << 32) | rng.integers(0, 1 << 32, size=ts.shape[0], dtype=np.int64)
    return np.argsort(key)


def make_c2(seed=None, n_shards=115, total=400_000_000, lo=10_000, hi=20_000_000, workers=None):
    """Batched workload: list of shards (each an independent problem).  Shards
    are drawn from their own seed streams, so drawing them on several threads
    gives the same records."""
    sizes = c2_shard_sizes(n_shards, total, lo, hi, seed=seed)
    children = np.random.SeedSequence(SEED_BASE + 2 if seed is None else seed + 1).spawn(n_shards)
    jobs = [(c, int(s)) for c, s in zip(children, sizes)]
    if workers is None:
        workers = min(8, len(jobs))
    if workers <= 1:
        return [make_shard(np.random.default_rng(c), s) for c, s in jobs]
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda js: make_shard(np.random.default_rng(js[0]), js[1]), jobs))


def make_stream(seed=None, n_journeys=2000, median=1500.0, sigma=1.0, cap=86_400, heavy_frac=0.0,
                heavy_share=0.3, heavy_cap=500_000, heavy_period_ms=50, span_s=None, config_index=3) -> Records:
    """A stream of records in feed (event-time) order: journeys start uniformly
    over a window so that many are open at once; 1 Hz samples, and optionally
    a small fraction of heavy journeys sampled at 20 Hz that hold a given share
    of all records (the skewed stream)."""
    rng = rng_for(config_index, seed)
    L = c1_lengths(rng, n_journeys, median=median, sigma=sigma, cap=cap)
    period = np.full(n_journeys, 1000, dtype=np.int64)
    if heavy_frac > 0:
        nh = max(1, int(round(heavy_frac * n_journeys)))
        hv = rng.choice(n_journeys, size=nh, replace=False)
        light = int(L.sum() - L[hv].sum())
        want = int(heavy_share / (1.0 - heavy_share) * light)
        w = rng.lognormal(0.0, 1.0, size=nh)
        Lh = np.minimum(np.maximum(np.rint(w / w.sum() * want), 1), heavy_cap).astype(np.int64)
        L[hv] = Lh
        period[hv] = heavy_period_ms
    ids = journey_ids(rng, n_journeys)
    dur = (L - 1) * period
    if span_s is None:
        span_s = int(np.median(dur) // 1000) + 1
    start = T0_MS + 1000 * rng.integers(0, max(1, span_s), size=n_journeys).astype(np.int64)
    parts = []
    for per in np.unique(period):
        sel = np.nonzero(period == per)[0]
        ts, lat, lon, _ = walks(rng, L[sel], period_ms=int(per), start_ms=start[sel])
        parts.append((np.repeat(ids[sel], L[sel]), ts, lat, lon))
    jid = np.concatenate([p[0] for p in parts])
    ts = np.concatenate([p[1] for p in parts])
    lat = np.concatenate([p[2] for p in parts])
    lon = np.concatenate([p[3] for p in parts])
    spd = speeds(rng, ts.shape[0])
    order = feed_order(rng, ts)
    return Records(jid[order], ts[order], lat[order], lon[order], spd[order],
                   dict(n_journeys=n_journeys, heavy_frac=heavy_frac))


def headings(rng, journey_id) -> np.ndarray:
    """A sensor heading column (whole degrees, as in Table 1) for records in
    which each journey's records are contiguous: a random start per journey
    and a slow random walk (2 degrees per record), float32 in [0, 360)."""
    n = journey_id.shape[0]
    start = np.ones(n, dtype=bool)
    start[1:] = journey_id[1:] != journey_id[:-1]
    step = rng.normal(0.0, 2.0, n)
    step[start] = rng.uniform(0.0, 360.0, int(start.sum()))
    c = np.cumsum(step)
    first = np.maximum.accumulate(np.where(start, np.arange(n), 0))
    base = c[first] - step[first]
    h = np.floor(np.mod(c - base, 360.0))
    return h.astype(np.float32)


CSV_HEADER = b"Journey Id,Timestamp,Latitude,Longitude,Postal Code,Speed,Heading\n"


def _digits(v, width):
    """Decimal digits (ASCII) of non-negative integers, zero-padded: (n, width) uint8."""
    v = np.asarray(v, dtype=np.int64).copy()
    out = np.empty((v.shape[0], width), dtype=np.uint8)
    for i in range(width - 1, -1, -1):
        out[:, i] = ord("0") + (v % 10)
        v //= 10
    return out


def _civil(days):
    """(year, month, day) of days since 1970-01-01 (proleptic Gregorian)."""
    z = days + 719468
    era = np.floor_divide(z, 146097)
    doe = z - era * 146097
    yoe = (doe - doe // 1460 + doe // 36524 - doe // 146096) // 365
    y = yoe + era * 400
    doy = doe - (365 * yoe + yoe // 4 - yoe // 100)
    mp = (5 * doy + 2) // 153
    d = doy - (153 * mp + 2) // 5 + 1
    m = np.where(mp < 10, mp + 3, mp - 9)
    return y + (m <= 2), m, d


def to_csv(records, heading, header=True) -> bytes:
    """Table-1-shaped text of records (fixed-width fields, one row per line):
    a 7-character journey id (5 digits and 2 letters from the id), UTC time
    with milliseconds, signed latitude / longitude with 6 decimals, a postal
    code, speed with 2 decimals, whole-degree heading."""
    jid, ts, lat, lon, spd = records.columns() if hasattr(records, "columns") else records
    n = jid.shape[0]
    jid = np.asarray(jid, dtype=np.int64)
    idd = _digits(np.abs(jid) % 100_000, 5)
    letters = np.stack([ord("a") + (np.abs(jid) // 100_000) % 26, ord("a") + (np.abs(jid) // 2_600_000) % 26], 1)
    days = np.floor_divide(ts, 86_400_000)
    msd = ts - days * 86_400_000
    y, mo, d = _civil(days)
    hh, mi, se, ms = msd // 3_600_000, (msd // 60_000) % 60, (msd // 1000) % 60, msd % 1000
    def signed(v, idig):
        q = np.rint(np.abs(v) * 1e6).astype(np.int64)
        sign = np.where(np.asarray(v) < 0, ord("-"), ord("+")).astype(np.uint8)[:, None]
        return np.concatenate([sign, _digits(q // 1_000_000, idig), np.full((n, 1), ord("."), np.uint8),
                               _digits(q % 1_000_000, 6)], 1)
    sq = np.rint(np.clip(np.asarray(spd, dtype=np.float64), 0, 999.99) * 100).astype(np.int64)
    hq = np.rint(np.mod(np.asarray(heading, dtype=np.float64), 360.0)).astype(np.int64) % 360
    c = lambda ch: np.full((n, 1), ord(ch), np.uint8)  # noqa: E731
    parts = [idd, letters.astype(np.uint8), c(","),
             _digits(y, 4), c("-"), _digits(mo, 2), c("-"), _digits(d, 2), c(" "), _digits(hh, 2), c(":"),
             _digits(mi, 2), c(":"), _digits(se, 2), c("."), _digits(ms, 3), c(","),
             signed(lat, 3), c(","), signed(lon, 3), c(","), _digits(65000 + np.abs(jid) % 1000, 5), c(","),
             _digits(sq // 100, 3), c("."), _digits(sq % 100, 2), c(","), _digits(hq, 3), c("\n")]
    body = np.concatenate(parts, 1).tobytes()
    return (CSV_HEADER if header else b"") + body


def chunk_sizes(rng, n, lo, hi):
    """Consecutive chunk sizes, log-uniform on [lo, hi], covering n records."""
    out = []
    left = n
    while left > 0:
        s = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        s = max(1, min(s, left))
        out.append(s)
        left -= s
    return out


def make(config: str, seed=None, **kw):
    if config == "c0":
        return make_c0(seed, **kw)
    if config == "c1":
        return make_c1(seed, **kw)
    if config == "c2":
        return make_c2(seed, **kw)
    raise ValueError(f"unknown config {config!r}")
