"""Pins for the CPU oracle: it is checked against things other than itself --
closed forms, library routines (math.fsum, numpy.lexsort), 50-digit mpmath
references computed with *different* formulas, the paper's Table 1 rows, and
brute force on tiny inputs.  Each test names the mistake it would catch."""
import csv
import datetime as dt
import itertools
import json
import math
import os

import mpmath
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2305_07454_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R = 6371008.8
pytestmark = []


# --------------------------------------------------------------------------
# exact summation
# --------------------------------------------------------------------------

def test_fsum_matches_math_fsum_random(oracle_mod):
    rng = np.random.default_rng(1)
    for n in (0, 1, 2, 7, 1000, 20000):
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-20, 20, size=n)
        assert oracle.fsum(x) == math.fsum(x)


def test_fsum_cancellation_and_halfway(oracle_mod):
    cases = [
        [1e100, 1.0, -1e100, 1e-100],
        [1.0, 1e-16, 1e-16],                       # half-way correction
        [0.1] * 10,
        [2.0 ** 53, 1.0, 1.0],
        [2.0 ** 53, -0.5, -2.0 ** -54],
        [1e308, 1e308 * 0.5, -1e308],
    ]
    for c in cases:
        assert oracle.fsum(np.array(c)) == math.fsum(c)


# --------------------------------------------------------------------------
# ordering
# --------------------------------------------------------------------------

def test_sort_matches_lexsort_with_ties(oracle_mod):
    rng = np.random.default_rng(2)
    n = 50000
    jid = rng.integers(-5, 40, size=n).astype(np.int64) * (2 ** 58)   # negative ids, big values
    ts = rng.integers(-3, 30, size=n).astype(np.int64)               # many ties
    perm = oracle.sort(jid, ts)
    ref = np.lexsort((np.arange(n), ts, jid))
    assert np.array_equal(perm.astype(np.int64), ref)


def test_sort_brute_force_tiny(oracle_mod):
    # every ordering of a tiny multiset: output keys sorted, ties in input order
    base = [(3, 5), (1, 2), (3, 5), (1, 1), (2, 7), (1, 2)]
    for p in itertools.permutations(range(len(base))):
        rows = [base[i] for i in p]
        jid = np.array([r[0] for r in rows], dtype=np.int64)
        ts = np.array([r[1] for r in rows], dtype=np.int64)
        perm = oracle.sort(jid, ts).tolist()
        assert perm == sorted(range(len(rows)), key=lambda i: (rows[i][0], rows[i][1], i))


def test_sort_signed_extremes(oracle_mod):
    jid = np.array([2 ** 63 - 1, -2 ** 63, 0, -1, 2 ** 63 - 1], dtype=np.int64)
    ts = np.array([5, 9, 1, 2, 4], dtype=np.int64)
    assert oracle.sort(jid, ts).tolist() == [1, 3, 2, 4, 0]


# --------------------------------------------------------------------------
# late records of a stream (the serving form's reading of time going backwards)
# --------------------------------------------------------------------------

# Hand-worked cases: (journey ids, time stamps, push sizes, expected late flags).
LATE_CASES = [
    # one journey; the fourth record comes in a later push, older than 5000
    ([9, 9, 9, 9], [0, 1000, 5000, 3000], [3, 1], [0, 0, 0, 1]),
    # the same records in one push: the sort orders them, nothing is late
    ([9, 9, 9, 9], [0, 1000, 5000, 3000], [4], [0, 0, 0, 0]),
    # two journeys interleaved; equal to the newest earlier time is not late
    ([1, 1, 2, 1, 2, 1, 1], [10, 20, 100, 15, 100, 20, 5], [3, 4], [0, 0, 0, 1, 0, 0, 1]),
    # late records never become history: 6 is still below 10
    ([4, 4, 4, 4], [10, 5, 7, 6], [1, 2, 1], [0, 1, 1, 1]),
    # history is the largest earlier time, not the last push's
    ([4, 4, 4], [50, 60, 55], [1, 1, 1], [0, 0, 1]),
    ([4, 4, 4], [50, 30, 40], [2, 1], [0, 0, 1]),
    # records of one push join history only after that push: 20 < 40 in one push is fine
    ([4, 4, 4], [10, 40, 20], [1, 2], [0, 0, 0]),
    # a record of another journey is never compared across journeys
    ([1, 2, 2], [100, 5, 6], [1, 1, 1], [0, 0, 0]),
    # empty pushes change nothing
    ([3, 3], [9, 8], [1, 0, 1], [0, 1]),
]


@pytest.mark.parametrize("jid,ts,sizes,late", LATE_CASES)
def test_stream_late_by_hand(oracle_mod, jid, ts, sizes, late):
    got = oracle.stream_late(np.array(jid, np.int64), np.array(ts, np.int64), sizes)
    assert got.astype(int).tolist() == late


def test_stream_late_invariants(oracle_mod):
    rng = np.random.default_rng(12)
    n = 5000
    jid = rng.integers(0, 40, n).astype(np.int64)
    ts = rng.integers(0, 10_000, n).astype(np.int64)
    sizes = gen.chunk_sizes(rng, n, 10, 400)
    # a single push never has late records
    assert not oracle.stream_late(jid, ts, [n]).any()
    # times non-decreasing per journey in arrival order: no split makes one late
    mono = np.empty(n, np.int64)
    for j in np.unique(jid):
        w = np.flatnonzero(jid == j)
        mono[w] = np.sort(ts[w])
    assert not oracle.stream_late(jid, mono, sizes).any()
    # a late record's time is below some earlier-push time of its journey
    late = oracle.stream_late(jid, ts, sizes)
    assert late.any()
    push = np.repeat(np.arange(len(sizes)), sizes)
    for i in np.flatnonzero(late)[:200]:
        earlier = (jid == jid[i]) & (push < push[i])
        assert earlier.any() and ts[earlier].max() > ts[i]
    # and a record below nothing earlier is never late
    for i in np.flatnonzero(~late)[:200]:
        earlier = (jid == jid[i]) & (push < push[i]) & ~late
        assert not earlier.any() or ts[i] >= ts[earlier].max()


# --------------------------------------------------------------------------
# kinematics: closed forms and 50-digit references
# --------------------------------------------------------------------------

def _feat(lat, lon, ts=None, jid=None):
    n = len(lat)
    jid = np.zeros(n, np.int64) if jid is None else np.asarray(jid, np.int64)
    ts = np.arange(n, dtype=np.int64) * 1000 if ts is None else np.asarray(ts, np.int64)
    return oracle.features(jid, ts, np.asarray(lat, float), np.asarray(lon, float))


def test_one_degree_of_meridian_and_equator(oracle_mod):
    exact = float(mpmath.mpf("6371008.8") * mpmath.pi / 180)        # 111195.0802335329 m
    assert abs(exact - 111195.0802335329) < 1e-9
    for lat, lon in (([0.0, 1.0], [0.0, 0.0]), ([37.0, 38.0], [-92.0, -92.0]),
                     ([0.0, 0.0], [0.0, 1.0]), ([0.0, 0.0], [-90.5, -89.5])):
        f = _feat(lat, lon)
        assert abs(f["step_m"][1] - exact) <= 2e-16 * exact


def test_quarter_and_half_circumference(oracle_mod):
    f = _feat([0.0, 90.0], [0.0, 0.0])
    assert abs(f["step_m"][1] - float(mpmath.mpf("6371008.8") * mpmath.pi / 2)) < 1e-8
    f = _feat([0.0, 0.0], [0.0, 180.0])                 # antipodes: exercises the clamp
    assert abs(f["step_m"][1] - float(mpmath.mpf("6371008.8") * mpmath.pi)) < 1e-8
    assert f["flags"][1] & oracle.FLAG_BEARING_OK


def test_cardinal_bearings(oracle_mod):
    f = _feat([10.0, 10.001], [20.0, 20.0])
    assert f["bearing_deg"][1] == 0.0
    f = _feat([0.0, 0.0], [20.0, 20.001])
    assert abs(f["bearing_deg"][1] - 90.0) < 1e-12
    f = _feat([10.0, 9.999], [20.0, 20.0])
    assert f["bearing_deg"][1] == 180.0
    f = _feat([0.0, 0.0], [20.0, 19.999])
    assert abs(f["bearing_deg"][1] - 270.0) < 1e-12


def _mp_ref(lat1, lon1, lat2, lon2):
    """Chord-length distance and textbook bearing at 50 digits (different formulas)."""
    mpmath.mp.dps = 50
    d2r = mpmath.pi / 180
    p1, l1, p2, l2 = (mpmath.mpf(v) * d2r for v in (lat1, lon1, lat2, lon2))
    u1 = (mpmath.cos(p1) * mpmath.cos(l1), mpmath.cos(p1) * mpmath.sin(l1), mpmath.sin(p1))
    u2 = (mpmath.cos(p2) * mpmath.cos(l2), mpmath.cos(p2) * mpmath.sin(l2), mpmath.sin(p2))
    chord = mpmath.sqrt(sum((a - b) ** 2 for a, b in zip(u1, u2)))
    dist = 2 * mpmath.mpf("6371008.8") * mpmath.asin(chord / 2)
    y = mpmath.sin(l2 - l1) * mpmath.cos(p2)
    x = mpmath.cos(p1) * mpmath.sin(p2) - mpmath.sin(p1) * mpmath.cos(p2) * mpmath.cos(l2 - l1)
    b = mpmath.atan2(y, x) * 180 / mpmath.pi
    if b < 0:
        b += 360
    return dist, b


def test_haversine_and_bearing_vs_mpmath(oracle_mod):
    rng = np.random.default_rng(3)
    n = 400
    lat1 = rng.uniform(36.0, 40.6, n)
    lon1 = rng.uniform(-95.8, -89.1, n)
    lat2 = lat1 + rng.normal(0, 2e-4, n)
    lon2 = lon1 + rng.normal(0, 2e-4, n)
    lat = np.empty(2 * n)
    lon = np.empty(2 * n)
    lat[0::2], lat[1::2] = lat1, lat2
    lon[0::2], lon[1::2] = lon1, lon2
    jid = np.repeat(np.arange(n), 2)
    f = _feat(lat, lon, jid=jid, ts=np.tile([0, 1000], n))
    for i in range(n):
        d, b = _mp_ref(lat1[i], lon1[i], lat2[i], lon2[i])
        got_d, got_b = f["step_m"][2 * i + 1], f["bearing_deg"][2 * i + 1]
        assert abs(got_d - float(d)) <= 1e-15 * float(d)
        diff = abs(got_b - float(b))
        assert min(diff, 360.0 - diff) <= 1e-12


def test_long_steps_vs_mpmath(oracle_mod):
    rng = np.random.default_rng(4)
    for _ in range(100):
        a = rng.uniform(-80, 80, 2)
        o = rng.uniform(-179, 179, 2)
        f = _feat(a, o)
        d, b = _mp_ref(a[0], o[0], a[1], o[1])
        assert abs(f["step_m"][1] - float(d)) <= 1e-13 * float(d)
        diff = abs(f["bearing_deg"][1] - float(b))
        assert min(diff, 360.0 - diff) <= 1e-9


def test_dt_speed_accel_on_meridian_walk(oracle_mod):
    # step k along a meridian of k*delta degrees: arc = R*pi/180*k*delta (closed form),
    # so v_k = arc_k/dt and a_k = R*pi/180*delta/dt^2 exactly in real arithmetic.
    delta = 1e-5
    k = np.arange(12)
    lat = 37.0 + delta * k * (k + 1) / 2
    lon = np.full(12, -92.0)
    ts = np.arange(12, dtype=np.int64) * 2000        # 2 s apart
    f = _feat(lat, lon, ts=ts)
    assert np.all(f["dt_s"][1:] == 2.0)
    arc = R * math.pi / 180 * delta * k[1:]
    assert np.allclose(f["step_m"][1:], arc, rtol=1e-9)
    assert np.allclose(f["speed_mps"][1:], arc / 2.0, rtol=1e-9)
    acc = R * math.pi / 180 * delta / 4.0
    assert np.all(f["flags"][2:] & oracle.FLAG_ACCEL_OK)
    assert not f["flags"][1] & oracle.FLAG_ACCEL_OK          # predecessor is the journey head
    assert np.allclose(f["accel_mps2"][2:], acc, rtol=1e-6)
    assert np.all(f["bearing_deg"][1:] == 0.0)
    assert np.all(f["dheading_deg"][2:] == 0.0)


def _bearing_step(lat, lon, brg_deg, d=1e-4):
    """A point roughly d degrees from (lat, lon) along compass bearing brg."""
    b = math.radians(brg_deg)
    return lat + d * math.cos(b), lon + d * math.sin(b) / math.cos(math.radians(lat))


@pytest.mark.parametrize("b1,b2,expect", [(350, 10, 20), (10, 350, -20), (0, 180, 180),
                                          (180, 0, 180), (90, 270, 180), (270, 90, 180),
                                          (45, 45, 0), (300, 120, 180)])
def test_heading_change_wrap(oracle_mod, b1, b2, expect):
    lat0, lon0 = 38.0, -92.0
    lat1, lon1 = _bearing_step(lat0, lon0, b1)
    lat2, lon2 = _bearing_step(lat1, lon1, b2)
    f = _feat([lat0, lat1, lat2], [lon0, lon1, lon2])
    assert f["flags"][2] & oracle.FLAG_DHEAD_OK
    got = f["dheading_deg"][2]
    assert -180.0 < got <= 180.0
    if expect == 180 and b1 % 180 == 0:
        assert got == 180.0               # exact meridian reversal lands on +180, never -180
    diff = abs(got - expect)
    assert min(diff, 360.0 - diff) < 0.01


def test_flags_heads_duplicates_and_bad_coordinates(oracle_mod):
    nan, inf = float("nan"), float("inf")
    jid = [1, 1, 1, 1, 2, 2, 2, 3]
    ts = [0, 1000, 1000, 2000, 0, 1000, 2000, 5]
    lat = [37.0, 37.001, 37.001, 37.002, 38.0, nan, 38.002, inf]
    lon = [-92.0, -92.0, -92.0, -92.0, -91.0, -91.0, -91.0, -91.0]
    f = oracle.features(np.array(jid), np.array(ts), np.array(lat), np.array(lon))
    F = oracle
    assert f["flags"][0] == F.FLAG_FIRST
    assert f["flags"][1] == F.FLAG_SPEED_OK | F.FLAG_BEARING_OK
    # identical coordinates and timestamp: zero step, no speed, no bearing
    assert f["flags"][2] == F.FLAG_DT_ZERO
    assert f["step_m"][2] == 0.0 and f["bearing_deg"][2] == 0.0
    # predecessor had no speed -> no accel; predecessor had no bearing -> no heading change
    assert f["flags"][3] == F.FLAG_SPEED_OK | F.FLAG_BEARING_OK
    assert f["flags"][4] == F.FLAG_FIRST
    assert f["flags"][5] == F.FLAG_BAD_COORD                  # non-finite at k
    assert f["flags"][6] == F.FLAG_BAD_COORD                  # non-finite at predecessor
    assert f["flags"][7] == F.FLAG_FIRST | F.FLAG_BAD_COORD
    for k in (0, 2, 4, 5, 6, 7):
        assert all(f[c][k] == 0.0 for c in ("step_m", "speed_mps", "accel_mps2", "dheading_deg"))


# --------------------------------------------------------------------------
# summaries
# --------------------------------------------------------------------------

def _plain(cols, spec):
    return oracle.run_plain(cols, spec)


def test_summary_against_numpy_and_fsum(oracle_mod):
    r = gen.make_c1(seed=11, n_journeys=60, median=300.0)
    out = _plain(r.columns(), gen.GRIDS["c1"])
    jid, ts, lat, lon, spd = out["sorted"]
    f, s = out["features"], out["summary"]
    u, first, counts = np.unique(jid, return_index=True, return_counts=True)
    assert np.array_equal(s["journey_id"], u)
    assert np.array_equal(s["first"], first)
    assert np.array_equal(s["n_points"], counts)
    assert int(s["n_points"].sum()) == r.n
    for j in range(len(u)):
        a, b = first[j], first[j] + counts[j]
        assert s["distance_m"][j] == math.fsum(f["step_m"][a:b])
        assert s["sum_speed"][j] == math.fsum(spd[a:b].astype(np.float64))
        assert s["max_speed"][j] == spd[a:b].max()
        assert s["t_start_ms"][j] == ts[a:b].min() and s["t_end_ms"][j] == ts[a:b].max()
        assert s["lat_min"][j] == lat[a:b].min() and s["lon_max"][j] == lon[a:b].max()
        ok = (f["flags"][a:b] & oracle.FLAG_SPEED_OK) != 0
        assert s["max_derived_speed"][j] == (f["speed_mps"][a:b][ok].max() if ok.any() else 0.0)
        assert s["n_dt_zero"][j] == int(((f["flags"][a:b] & oracle.FLAG_DT_ZERO) != 0).sum())


def test_summary_bbox_signed_zero_and_no_finite_points(oracle_mod):
    jid = np.array([1, 1, 2, 2], np.int64)
    ts = np.array([0, 1000, 0, 1000], np.int64)
    lat = np.array([-0.0, 0.0, np.nan, np.nan])
    lon = np.array([0.0, -0.0, 1.0, 2.0])
    spd = np.ones(4, np.float32)
    f = oracle.features(jid, ts, lat, lon)
    s = oracle.summary(jid, ts, lat, lon, spd, f)
    for k in ("lat_min", "lat_max", "lon_min", "lon_max"):
        assert s[k][0] == 0.0 and math.copysign(1.0, s[k][0]) == 1.0
    assert s["lat_min"][1] == math.inf and s["lat_max"][1] == -math.inf


def test_summary_max_derived_speed_only_over_speed_ok(oracle_mod):
    jid = np.zeros(3, np.int64)
    ts = np.array([0, 1000, 1000], np.int64)
    z = np.zeros(3)
    feat = dict(step_m=z, speed_mps=np.array([0.0, 5.0, 99.0]),
                flags=np.array([oracle.FLAG_FIRST, oracle.FLAG_SPEED_OK, oracle.FLAG_DT_ZERO], np.uint8))
    s = oracle.summary(jid, ts, np.full(3, 37.0), np.full(3, -92.0), np.ones(3, np.float32), feat)
    assert s["max_derived_speed"][0] == 5.0 and s["n_dt_zero"][0] == 1


def test_summary_distance_is_sum_of_steps_negative_zero_speed(oracle_mod):
    jid = np.array([7, 7, 7], np.int64)
    ts = np.array([0, 1000, 2000], np.int64)
    lat = np.array([37.0, 37.0001, 37.0003])
    lon = np.array([-92.0, -92.0, -92.0])
    spd = np.array([-0.0, -0.0, -0.0], np.float32)
    f = oracle.features(jid, ts, lat, lon)
    s = oracle.summary(jid, ts, lat, lon, spd, f)
    assert s["distance_m"][0] == math.fsum(f["step_m"])
    assert math.copysign(1.0, float(s["max_speed"][0])) == 1.0      # -0.0 counted as +0.0
    assert math.copysign(1.0, float(s["sum_speed"][0])) == 1.0      # exact zero sum is +0.0


# --------------------------------------------------------------------------
# grid aggregate
# --------------------------------------------------------------------------

def _brute_grid(jid, ts, lat, lon, spd, spec):
    groups = {}
    n_out = 0
    for i in range(len(jid)):
        la, lo = float(lat[i]), float(lon[i])
        if not (math.isfinite(la) and math.isfinite(lo)):
            n_out += 1
            continue
        y = math.floor((la - spec.lat0_deg) / spec.dlat_deg)
        x = math.floor((lo - spec.lon0_deg) / spec.dlon_deg)
        t = (int(ts[i]) - spec.t0_ms) // spec.bin_ms
        if not (0 <= y < spec.n_lat and 0 <= x < spec.n_lon and t >= 0 and (spec.n_t <= 0 or t < spec.n_t)):
            n_out += 1
            continue
        k = (t * spec.n_lat + y) * spec.n_lon + x
        g = groups.setdefault(k, [0, set(), [], []])
        g[0] += 1
        g[1].add(int(jid[i]))
        g[2].append(float(spd[i]))
        g[3].append(float(spd[i]) + 0.0)
    return groups, n_out


def test_grid_brute_force(oracle_mod):
    r = gen.make_c0(seed=5, n_journeys=40, min_len=20, max_len=200)
    spec = gen.grid_for(0.01, 60_000)
    jid, ts, lat, lon, spd = r.columns()
    lat = lat.copy()
    lat[::97] = 35.5              # some out-of-box points
    lat[5] = float("nan")
    res, n_out = oracle.grid(jid, ts, lat, lon, spd, spec)
    ref, ref_out = _brute_grid(jid, ts, lat, lon, spd, spec)
    assert n_out == ref_out
    assert res["key"].tolist() == sorted(ref)
    for i, k in enumerate(res["key"].tolist()):
        c, js, ss, ss0 = ref[k]
        assert res["count"][i] == c
        assert res["n_journeys"][i] == len(js)
        assert res["sum_speed"][i] == math.fsum(ss)
        assert res["min_speed"][i] == min(ss0) and res["max_speed"][i] == max(ss0)
    assert int(res["count"].sum()) + n_out == r.n
    pairs = {(k, j) for k, v in ref.items() for j in v[1]}
    assert int(res["n_journeys"].sum()) == len(pairs)


@pytest.mark.parametrize("n_dir,offset,cases", [
    # literal floor division by 90 degrees (Algorithm 2): [0, 90) -> 0 ...
    (4, 0.0, [(0.0, 0), (45.0, 0), (89.999, 0), (90.0, 1), (180.0, 2), (269.5, 2), (270.0, 3), (359.9, 3)]),
    # centred on N, E, S, W: N = [315, 45), E = [45, 135), S = [135, 225), W = [225, 315)
    (4, 45.0, [(0.0, 0), (44.999, 0), (45.0, 1), (134.9, 1), (135.0, 2), (224.9, 2), (225.0, 3), (315.0, 0),
               (359.9, 0)]),
    # eight sectors of 45 degrees
    (8, 0.0, [(0.0, 0), (44.9, 0), (45.0, 1), (200.0, 4), (315.0, 7), (359.0, 7)]),
    # no direction: outside [0, 360) or NaN -> the extra sector n_dir
    (4, 0.0, [(360.0, 4), (-0.5, 4), (float("nan"), 4), (1e300, 4)]),
])
def test_dir_sector_values(oracle_mod, n_dir, offset, cases):
    for h, want in cases:
        assert oracle_mod.dir_sector(h, True, n_dir, offset) == want, (h, n_dir, offset)
    # a bearing without CV_FLAG_BEARING_OK has no direction
    assert oracle_mod.dir_sector(10.0, False, n_dir, offset) == n_dir


def _remap_plain(groups, cells, n_dir, sector):
    """Plain lattice keys -> direction-lattice keys with every record in one sector."""
    k = groups["key"]
    return ((k // cells) * (n_dir + 1) + sector) * cells + k % cells


def test_grid_dir_reduces_to_plain_lattice(oracle_mod):
    # one sector with every heading valid, or no valid heading at all: the
    # direction lattice is the plain one with the keys spread by (n_dir + 1)
    r = gen.make_c1(seed=13, n_journeys=25, median=500.0)
    spec = gen.GRIDS["c1"]
    cells = spec.n_lat * spec.n_lon
    plain, n_out = oracle_mod.grid(*r.columns(), spec)
    for n_dir, hd, sector in ((1, np.full(r.n, 123.0, np.float32), 0),
                              (4, np.full(r.n, np.nan, np.float32), 4),
                              (4, np.full(r.n, -3.0, np.float32), 4)):
        g, no = oracle_mod.grid_dir(*r.columns(), spec, n_dir, 0.0, heading=hd)
        assert no == n_out
        np.testing.assert_array_equal(g["key"], _remap_plain(plain, cells, n_dir, sector))
        for f in ("count", "n_journeys", "sum_speed", "min_speed", "max_speed"):
            np.testing.assert_array_equal(g[f], plain[f], err_msg=f)


def test_grid_dir_marginals_over_sectors(oracle_mod):
    # summed over sectors: counts and extrema of a (time bin, cell) are the
    # plain lattice's; a journey counted in a cell is counted in at least one
    # of its sectors and in at most all of them
    r = gen.make_c1(seed=14, n_journeys=25, median=500.0)
    spec = gen.GRIDS["c1"]
    cells = spec.n_lat * spec.n_lon
    rng = np.random.default_rng(5)
    hd = rng.integers(0, 360, r.n).astype(np.float32)
    hd[rng.random(r.n) < 0.05] = np.nan
    g, _ = oracle_mod.grid_dir(*r.columns(), spec, 4, 45.0, heading=hd)
    plain, _ = oracle_mod.grid(*r.columns(), spec)
    k = g["key"]
    tb, sec, cell = k // (5 * cells), (k // cells) % 5, k % cells
    pk = tb * cells + cell
    assert set(sec.tolist()) <= set(range(5))
    idx = np.searchsorted(plain["key"], pk)
    assert np.all(plain["key"][idx] == pk)
    cnt = np.zeros(len(plain["key"]), np.int64)
    njs = np.zeros(len(plain["key"]), np.int64)
    mn = np.full(len(plain["key"]), np.inf)
    mx = np.full(len(plain["key"]), -np.inf)
    np.add.at(cnt, idx, g["count"].astype(np.int64))
    np.add.at(njs, idx, g["n_journeys"].astype(np.int64))
    np.minimum.at(mn, idx, g["min_speed"].astype(np.float64))
    np.maximum.at(mx, idx, g["max_speed"].astype(np.float64))
    np.testing.assert_array_equal(cnt, plain["count"])
    np.testing.assert_array_equal(mn, plain["min_speed"].astype(np.float64))
    np.testing.assert_array_equal(mx, plain["max_speed"].astype(np.float64))
    assert np.all(njs >= plain["n_journeys"]) and np.all(njs <= 5 * plain["n_journeys"])


def test_grid_dir_brute_force_tiny(oracle_mod):
    # every group of a tiny input from a dictionary of (key -> records)
    rng = np.random.default_rng(15)
    n = 60
    jid = rng.integers(1, 5, n).astype(np.int64)
    ts = gen.T0_MS + rng.integers(0, 3, n).astype(np.int64) * 300_000 + rng.integers(0, 1000, n)
    lat = 38.0 + rng.integers(0, 3, n) * 0.01 + 0.001
    lon = -92.0 + rng.integers(0, 2, n) * 0.01 + 0.001
    spd = rng.gamma(2.0, 4.0, n).astype(np.float32)
    hd = rng.choice(np.array([0.0, 10.0, 95.0, 180.0, 266.0, 359.0, np.nan], np.float32), n)
    spec = gen.GridSpec(37.9, -92.1, 0.01, 0.01, 40, 40, gen.T0_MS, 300_000, 10)
    g, n_out = oracle_mod.grid_dir(jid, ts, lat, lon, spd, spec, 4, 0.0, heading=hd)
    groups = {}
    for i in range(n):
        ilat = math.floor((lat[i] - spec.lat0_deg) / spec.dlat_deg)
        ilon = math.floor((lon[i] - spec.lon0_deg) / spec.dlon_deg)
        tb = (int(ts[i]) - spec.t0_ms) // spec.bin_ms
        h = float(hd[i])
        sec = 4 if math.isnan(h) else int(h // 90.0)
        key = ((tb * 5 + sec) * spec.n_lat + ilat) * spec.n_lon + ilon
        groups.setdefault(key, []).append(i)
    assert n_out == 0 and list(g["key"]) == sorted(groups)
    for j, key in enumerate(sorted(groups)):
        rows = groups[key]
        assert g["count"][j] == len(rows)
        assert g["n_journeys"][j] == len(set(jid[rows].tolist()))
        assert g["sum_speed"][j] == math.fsum(float(spd[i]) for i in rows)
        assert g["min_speed"][j] == min(spd[rows]) and g["max_speed"][j] == max(spd[rows])


def test_grid_dir_bearing_equals_heading_on_exact_values(oracle_mod):
    # the derived-bearing form takes a bearing where its flag says so: on
    # bearings that float32 holds exactly it equals the sensor-heading form
    r = gen.make_c1(seed=16, n_journeys=20, median=400.0)
    spec = gen.GRIDS["c1"]
    rng = np.random.default_rng(6)
    b = rng.choice(np.array([0.0, 12.5, 89.75, 90.0, 100.25, 200.0, 300.75, 359.5]), r.n)
    ok = rng.random(r.n) < 0.9
    flags = np.where(ok, 0x10, 0x04).astype(np.uint8)
    hd = np.where(ok, b, np.nan).astype(np.float32)
    for nd, off in ((4, 0.0), (4, 45.0), (8, 22.5)):
        gb, nb = oracle_mod.grid_dir(*r.columns(), spec, nd, off, bearing=b, flags=flags)
        gh, nh = oracle_mod.grid_dir(*r.columns(), spec, nd, off, heading=hd)
        assert nb == nh
        for f in gb:
            np.testing.assert_array_equal(gb[f], gh[f], err_msg=f)


def _groups(rows):
    """Group table from (key, count, n_journeys, sum_speed) rows."""
    k, c, j, sm = zip(*rows)
    return {"key": np.array(k, np.int64), "count": np.array(c, np.uint32), "n_journeys": np.array(j, np.uint32),
            "sum_speed": np.array(sm, np.float64)}


def test_lattice_dense_by_hand(oracle_mod):
    spec = gen.GridSpec(0.0, 0.0, 1.0, 1.0, 2, 3, 0, 60_000, 10)   # 2 x 3 cells
    # (tbin 1, ilat 1, ilon 2): key (1*2+1)*3+2 = 11; (tbin 0, 0, 0): key 0; tbin 5: outside t in [0, 3)
    g = _groups([(0, 2, 1, 3.0), (11, 4, 2, 10.0), ((5 * 2 + 1) * 3 + 1, 1, 1, 7.0)])
    out = oracle_mod.lattice_dense(g, spec, 0, 0, 3)
    want = np.zeros((3, 2, 2, 3), np.float32)
    want[0, 0, 0, 0], want[0, 1, 0, 0] = 1.5, 1.0
    want[1, 0, 1, 2], want[1, 1, 1, 2] = 2.5, 2.0
    np.testing.assert_array_equal(out, want)
    # t_first moves the window: tbin 1 is the first image
    out = oracle_mod.lattice_dense(g, spec, 0, 1, 5)
    assert out[0, 0, 1, 2] == 2.5 and out[4, 0, 1, 1] == 7.0 and out.sum() == 2.5 + 2.0 + 7.0 + 1.0
    # four sectors (D = 5): key ((tbin * 5 + sector) * 2 + ilat) * 3 + ilon
    g = _groups([(((2 * 5 + 3) * 2 + 0) * 3 + 1, 3, 3, 9.0), (((0 * 5 + 4) * 2 + 1) * 3 + 0, 1, 1, 0.5)])
    out = oracle_mod.lattice_dense(g, spec, 4, 0, 3)
    assert out.shape == (3, 10, 2, 3)
    assert out[2, 6, 0, 1] == 3.0 and out[2, 7, 0, 1] == 3.0       # sector 3: speed 9/3, volume 3
    assert out[0, 8, 1, 0] == 0.5 and out[0, 9, 1, 0] == 1.0       # sector 4 (no direction)
    assert np.count_nonzero(out) == 4


def test_lattice_normalize_by_hand(oracle_mod):
    lat = np.zeros((2, 4, 1, 3), np.float32)
    # channels 0/1: speeds 2.5, 5, 10 with volumes 1, 1, 3 (cell (t=1, x=2) empty)
    lat[0, 0, 0, :], lat[0, 1, 0, :] = (2.5, 5.0, 10.0), (1, 1, 3)
    # channels 2/3: one occupied cell (constant channel), its speed 0
    lat[1, 3, 0, 1] = 4.0
    out, mm = oracle_mod.lattice_normalize(lat)
    np.testing.assert_array_equal(out[0, 0, 0], np.array([0.0, 1.0 / 3.0, 1.0], np.float32))
    np.testing.assert_array_equal(out[0, 1, 0], np.array([0.0, 0.0, 1.0], np.float32))
    assert np.all(out[1, :2] == 0) and np.all(out[:, 2:] == 0)
    np.testing.assert_array_equal(mm[:2], np.array([[2.5, 10.0], [1.0, 3.0]], np.float32))
    np.testing.assert_array_equal(mm[2:], np.array([[0.0, 0.0], [4.0, 4.0]], np.float32))
    # a channel pair with no occupied cell: NaN bounds
    out, mm = oracle_mod.lattice_normalize(np.zeros((1, 2, 1, 1), np.float32))
    assert np.all(np.isnan(mm)) and np.all(out == 0)


def test_groups_filter_by_hand(oracle_mod):
    g = _groups([(0, 4, 2, 40.0), (1, 2, 1, 10.0), (2, 5, 5, 5.0), (3, 0, 0, 0.0), (4, 1, 3, 30.0)])
    # mean speeds 10, 5, 1, -, 30; volumes 2, 1, 5, 0, 3
    assert oracle_mod.groups_filter(g, 2, 0.0, 15.0).tolist() == [0, 2]
    assert oracle_mod.groups_filter(g, 1, 5.0, 10.0).tolist() == [0, 1]
    assert oracle_mod.groups_filter(g, 0, -1.0, 1e9).tolist() == [0, 1, 2, 4]
    assert oracle_mod.groups_filter(g, 6, -1.0, 1e9).tolist() == []


def test_drop_duplicates_table1_and_by_hand(oracle_mod):
    # Table 1's fourth row repeats its first: after the sort they are adjacent
    # (same journey and time) and the later one (input row 3) goes
    cols = _table1()
    perm = oracle_mod.sort(cols[0], cols[1])
    s = oracle_mod.sorted_records(cols, perm)
    keep = oracle_mod.drop_duplicates(s)
    assert sorted(perm[keep].tolist()) == [0, 1, 2]
    # same journey and time: a different latitude is kept, an identical row
    # is not; the same row in another journey is kept; -0.0 and 0.0 differ in
    # their bits (kept)
    jid = np.array([1, 1, 1, 1, 2, 2, 2], np.int64)
    ts = np.array([5, 5, 5, 6, 5, 5, 5], np.int64)
    lat = np.array([1.0, 1.5, 1.0, 1.0, 1.0, 0.0, -0.0])
    lon = np.full(7, 2.0)
    spd = np.array([3, 3, 3, 3, 3, 3, 3], np.float32)
    assert oracle_mod.drop_duplicates((jid, ts, lat, lon, spd)).tolist() == [0, 1, 3, 4, 5, 6]
    spd[2] = 3.5  # the third row now differs in speed
    assert oracle_mod.drop_duplicates((jid, ts, lat, lon, spd)).tolist() == [0, 1, 2, 3, 4, 5, 6]


def test_split_trips_by_hand(oracle_mod):
    jid = np.array([1, 1, 1, 1, 2, 2, 3], np.int64)
    ts = np.array([0, 100, 200, 301, 0, 1000, 7], np.int64)
    trip, tj = oracle_mod.split_trips(jid, ts, 100)     # a gap of exactly 100 stays, 101 splits
    assert trip.tolist() == [0, 0, 0, 1, 2, 3, 4] and tj.tolist() == [1, 1, 2, 2, 3]
    trip, tj = oracle_mod.split_trips(jid, ts, 10**6)   # no gap large enough: trips are journeys
    assert trip.tolist() == [0, 0, 0, 0, 1, 1, 2] and tj.tolist() == [1, 2, 3]
    trip, tj = oracle_mod.split_trips(jid, ts, 0)       # every increase splits
    assert trip.tolist() == [0, 1, 2, 3, 4, 5, 6]


def test_csv_table1_rows_by_hand(oracle_mod):
    # Table 1's first two rows: ids packed from their ASCII bytes ("3" 0x33,
    # "4" 0x34, "5" 0x35, "6" 0x36, "r" 0x72, "d" 0x64, "1" 0x31, "2" 0x32,
    # "t" 0x74, "f" 0x66), times from 2021-05-09 00:00 UTC = 1 620 518 400 000 ms
    text = (b"Journey Id,Timestamp,Latitude,Longitude,Postal Code,Speed,Heading\n"
            b"33456rd,2021-05-09 03:48:42,37.664087,-92.6546,65536,105.98,33\n"
            b"31224tf,2021-05-09 03:49:42,37.667707,-92.6490,65536,0,53\n")
    (jid, ts, lat, lon, spd), hd, ok = oracle_mod.csv_extract(text)
    assert ok.tolist() == [1, 1]
    assert jid.tolist() == [0x3333343536726400, 0x3331323234746600]
    assert ts.tolist() == [1620518400000 + (3 * 3600 + 48 * 60 + 42) * 1000, 1620518400000 + (3 * 3600 + 49 * 60 + 42) * 1000]
    assert lat.tolist() == [37.664087, 37.667707] and lon.tolist() == [-92.6546, -92.649]
    assert spd.tolist() == [np.float32(105.98), 0.0] and hd.tolist() == [33.0, 53.0]


@pytest.mark.parametrize("field,ok", [
    (b"5", True), (b"5.", True), (b".5", True), (b"+5", True), (b"-0", True), (b"037.5", True),
    (b"9007199254740991", True), (b"0." + b"0" * 21 + b"1", True),
    (b" 5", False), (b"5 ", False), (b"1e5", False), (b"nan", False), (b"inf", False), (b".", False),
    (b"-", False), (b"", False), (b"1.2.3", False), (b"9007199254740992", False),
    (b"0." + b"0" * 22 + b"1", False),
])
def test_csv_decimal_grammar(oracle_mod, field, ok):
    row = b"a1,2021-05-09 00:00:00," + field + b",-92.5,65536,1.5,10\n"
    (_, _, lat, _, _), _, good = oracle_mod.csv_extract(row, has_header=False)
    assert bool(good[0]) == ok
    if ok:
        assert lat[0] == float(field) and math.copysign(1.0, lat[0]) == math.copysign(1.0, float(field))


@pytest.mark.parametrize("stamp,ms", [
    (b"2020-02-29 00:00:00", 1582934400000), (b"2000-02-29 12:00:00", 951825600000),
    (b"1970-01-01 00:00:00.5", 500), (b"1970-01-01 00:00:00.05", 50), (b"1970-01-01 00:00:00.005", 5),
    (b"2021-02-29 00:00:00", None), (b"1900-02-29 00:00:00", None), (b"2021-05-09 24:00:00", None),
    (b"2021-05-09 00:60:00", None), (b"2021-05-09 00:00:60", None), (b"1970-01-01 00:00:00.0005", None),
    (b"2021-05-09T00:00:00", None), (b"0000-01-01 00:00:00", None), (b"2021-5-09 00:00:00", None),
])
def test_csv_timestamp_rule(oracle_mod, stamp, ms):
    (_, ts, _, _, _), _, good = oracle_mod.csv_extract(b"a1," + stamp + b",38.5,-92.5,1,2,3", has_header=False)
    assert bool(good[0]) == (ms is not None)
    if ms is not None:
        assert ts[0] == ms


def test_csv_lines_and_fields(oracle_mod):
    # CRLF; an empty line and a quoted row are malformed; no final newline;
    # an empty heading is NaN; ids of 8 bytes fit and 9 do not
    text = (b"h\r\n" b"abcdefgh,2021-05-09 00:00:00,1,2,3,4,5\r\n" b"\n"
            b'"q",2021-05-09 00:00:00,1,2,3,4,5\n' b"abcdefghi,2021-05-09 00:00:00,1,2,3,4,5\n"
            b"x,2021-05-09 00:00:01,1,2,3,4,\n" b"x,2021-05-09 00:00:02,1,2,3,4")
    (jid, ts, _, _, _), hd, ok = oracle_mod.csv_extract(text)
    assert ok.tolist() == [1, 0, 0, 0, 1, 0]
    assert jid[0] == int.from_bytes(b"abcdefgh", "big") and math.isnan(hd[4])
    assert oracle_mod.csv_extract(b"h\n")[2].tolist() == []
    assert oracle_mod.csv_extract(b"")[2].tolist() == []
    assert oracle_mod.csv_extract(b"x,2021-05-09 00:00:02,1,2,3,4,5", has_header=False)[2].tolist() == [1]


def test_grid_line_cases(oracle_mod):
    # Alg. 2 reading: floor of the rounded quotient, not Python's exact-quotient //
    spec = gen.GridSpec(36.0, -95.8, 0.005, 0.005, 920, 1340, 0, 300_000, 288)
    key, n_out = oracle.grid_keys(np.array([0, 0]), np.array([38.75, 36.01]),
                                  np.array([-95.8, -95.8]), spec)
    assert key[0] // 1340 == 550          # fl(2.75/0.005) = 550.0, while 2.75 // 0.005 = 549
    spec = gen.GridSpec(36.0, -95.8, 0.01, 0.01, 460, 670, 0, 300_000, 288)
    key, _ = oracle.grid_keys(np.array([0]), np.array([36.01]), np.array([-95.8]), spec)
    assert key[0] // 670 == 0             # (36.01-36.0)/0.01 = 0.999999999999801
    # cells where a reciprocal-multiply would land on the next bin: IEEE division
    # and the exact rational quotient of the binary inputs both floor one lower
    from fractions import Fraction
    for lat, step, expect in ((38.68, 0.01, 267), (38.805, 0.005, 560), (36.561, 0.001, 560)):
        sp = gen.GridSpec(36.0, -95.8, step, step, 4600, 6700, 0, 300_000, 288)
        key, _ = oracle.grid_keys(np.array([0]), np.array([lat]), np.array([-95.8]), sp)
        assert key[0] // 6700 == expect
        assert math.floor((Fraction(lat) - Fraction(36.0)) / Fraction(step)) == expect
        assert math.floor((lat - 36.0) * (1.0 / step)) == expect + 1
    # time bins floor toward -inf: ts before t0 is out of grid; the last bin edge is exclusive
    key, n_out = oracle.grid_keys(np.array([-1, 0, 299_999, 300_000, 288 * 300_000 - 1, 288 * 300_000]),
                                  np.full(6, 37.0), np.full(6, -92.0), spec)
    assert n_out == 2 and key[0] == -1 and key[5] == -1
    assert [int(k) // (460 * 670) for k in key[1:5]] == [0, 0, 1, 287]
    # box edges are half-open
    key, n_out = oracle.grid_keys(np.zeros(4, np.int64), np.array([36.0, 40.6, 37.0, 37.0]),
                                  np.array([-92.0, -92.0, -95.8, -89.1]), spec)
    assert key[0] >= 0 and key[1] == -1 and key[2] >= 0 and key[3] == -1


def test_grid_distinct_journeys_with_cell_reentry(oracle_mod):
    # one journey oscillating across a cell boundary inside one time bin, a second
    # journey visiting one of the cells once
    spec = gen.GridSpec(36.0, -95.8, 0.01, 0.01, 460, 670, 0, 300_000, 288)
    lat = np.array([37.004, 37.012, 37.003, 37.011, 37.002, 37.005])
    jid = np.array([1, 1, 1, 1, 1, 2])
    ts = np.array([0, 1000, 2000, 3000, 4000, 0])
    res, _ = oracle.grid(jid, ts, lat, np.full(6, -92.0), np.ones(6, np.float32), spec)
    assert res["count"].tolist() == [4, 2]
    assert res["n_journeys"].tolist() == [2, 1]


# --------------------------------------------------------------------------
# the paper's own sample rows (Table 1)
# --------------------------------------------------------------------------

def _table1():
    rows = [r for r in csv.reader(open(os.path.join(GOLDEN, "table1_records.csv")))
            if r and not r[0].startswith("#")][1:]
    names = sorted({r[0] for r in rows})
    t0 = dt.datetime(2021, 5, 9, tzinfo=dt.timezone.utc)
    jid = np.array([names.index(r[0]) for r in rows], np.int64)
    ts = np.array([int((dt.datetime.strptime(r[1], "%Y-%m-%d %H:%M:%S").replace(tzinfo=dt.timezone.utc)
                        - t0).total_seconds() * 1000) for r in rows], np.int64)
    lat = np.array([float(r[2]) for r in rows])
    lon = np.array([float(r[3]) for r in rows])
    spd = np.array([float(r[5]) for r in rows], np.float32)
    return jid, ts, lat, lon, spd


def test_table1_golden(oracle_mod):
    exp = json.load(open(os.path.join(GOLDEN, "table1_expected.json")))
    cols = _table1()
    spec = gen.GridSpec(**exp["grid"])
    out = oracle.run_plain(cols, spec)
    assert out["perm"].tolist() == exp["sorted_input_rows"]
    assert out["features"]["flags"].tolist() == exp["flags_sorted"]
    s = out["summary"]
    for i, j in enumerate(exp["journeys"]):
        for k, v in j.items():
            assert s[k][i] == v, k
    g = out["groups"]
    assert out["n_out"] == exp["n_out_of_grid"]
    for i, e in enumerate(exp["groups"]):
        assert g["key"][i] == e["key"] and g["count"][i] == e["count"]
        assert g["n_journeys"][i] == e["n_journeys"]
        sp = [float(np.float32(v)) for v in e["speeds"]]
        assert g["sum_speed"][i] == math.fsum(sp)
        assert g["min_speed"][i] == np.float32(min(sp)) and g["max_speed"][i] == np.float32(max(sp))


# --------------------------------------------------------------------------
# brute force on tiny random inputs (hypothesis)
# --------------------------------------------------------------------------

@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.integers(0, 3), st.integers(0, 4), st.integers(0, 5), st.integers(0, 5),
                          st.sampled_from([0.0, 1.5, 3.25, -0.0, 39.5])), min_size=0, max_size=30))
def test_tiny_random_plain_path(rows):
    oracle.lib()
    n = len(rows)
    jid = np.array([r[0] for r in rows], np.int64)
    ts = np.array([r[1] * 1000 for r in rows], np.int64)
    lat = np.array([37.0 + 0.004 * r[2] for r in rows])
    lon = np.array([-92.0 + 0.004 * r[3] for r in rows])
    spd = np.array([r[4] for r in rows], np.float32)
    spec = gen.GridSpec(36.0, -95.8, 0.01, 0.01, 460, 670, 0, 2000, 3)
    out = oracle.run_plain((jid, ts, lat, lon, spd), spec)
    # order
    assert out["perm"].tolist() == sorted(range(n), key=lambda i: (rows[i][0], rows[i][1], i))
    # summary invariants
    s = out["summary"]
    assert len(s["journey_id"]) == len(set(jid.tolist()))
    assert int(s["n_points"].sum()) == n
    # grid vs brute force
    ref, ref_out = _brute_grid(jid, ts, lat, lon, spd, spec)
    g = out["groups"]
    assert out["n_out"] == ref_out
    assert g["key"].tolist() == sorted(ref)
    assert g["n_journeys"].tolist() == [len(ref[k][1]) for k in sorted(ref)]
    assert g["sum_speed"].tolist() == [math.fsum(ref[k][2]) for k in sorted(ref)]
