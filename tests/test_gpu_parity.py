"""HIP path vs the oracle, element by element, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import check_features, check_groups, check_sort, check_summary, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    cvetl.lib()
    oracle.lib()
    return cvetl


def _run_both(cv, cols, spec, **kw):
    print(f"[parity] n={len(cols[0])} spec={spec}", flush=True)
    exp = oracle.run_plain(cols, spec)
    rec = cv.to_device(cols)
    got = cv.run_plain(rec, spec, **kw)
    return got, exp


def _check_all(got, exp):
    check_sort(got["perm"], got["sorted"], exp["perm"], exp["sorted"])
    check_features(got["features"], exp["features"])
    check_summary(got["summary"], exp["summary"])
    check_groups(got["groups"], got["n_out"], exp["groups"], exp["n_out"])


def test_c0_full_size(cv):
    r = gen.make_c0()
    got, exp = _run_both(cv, r.columns(), gen.GRIDS["c0"])
    _check_all(got, exp)


def test_c1_shaped(cv):
    r = gen.make_c1(seed=77, n_journeys=160)
    got, exp = _run_both(cv, r.columns(), gen.GRIDS["c1"])
    _check_all(got, exp)


def test_c1_shuffled_variant(cv):
    r = gen.make_c1(seed=78, n_journeys=80, shuffled=True)
    got, exp = _run_both(cv, r.columns(), gen.GRIDS["c1"])
    _check_all(got, exp)


def test_c2_shard_high_cardinality(cv):
    rng = np.random.default_rng(np.random.SeedSequence(5))
    r = gen.make_shard(rng, 300_000)
    got, exp = _run_both(cv, r.columns(), gen.GRIDS["c2"])
    _check_all(got, exp)


@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 2047, 2048, 2049, 4095, 4096, 4097, 8193])
def test_ragged_sizes(cv, n):
    r = gen.make_c0(seed=1000 + n, n_journeys=max(1, n // 40 + 1), min_len=1, max_len=80)
    cols = tuple(c[:n] for c in r.columns())
    got, exp = _run_both(cv, cols, gen.GRIDS["c0"])
    _check_all(got, exp)


def _adversarial():
    rng = np.random.default_rng(9)
    n = 6000
    ids = np.array([-(2 ** 63), 2 ** 63 - 1, -1, 0, 1, 12345, -99999], dtype=np.int64)
    jid = ids[rng.integers(0, len(ids), n)]
    ts = gen.T0_MS + rng.integers(-5, 40, n).astype(np.int64) * 30_000      # ties, before t0
    lat = rng.uniform(35.9, 40.7, n)                                          # some outside the box
    lon = rng.uniform(-95.9, -89.0, n)
    lat[rng.random(n) < 0.01] = np.nan
    lon[rng.random(n) < 0.01] = np.inf
    dup = rng.random(n) < 0.05                                                 # exact duplicates of a neighbour
    idx = np.nonzero(dup)[0]
    idx = idx[idx > 0]
    lat[idx], lon[idx], ts[idx], jid[idx] = lat[idx - 1], lon[idx - 1], ts[idx - 1], jid[idx - 1]
    spd = rng.uniform(0, 40, n).astype(np.float32)
    spd[rng.random(n) < 0.1] = np.float32(-0.0)
    spd[rng.random(n) < 0.1] = np.float32(0.0)
    return jid, ts, lat, lon, spd


def test_adversarial_ids_ties_duplicates_bad_coords(cv):
    cols = _adversarial()
    spec = gen.grid_for(0.01, 60_000)
    got, exp = _run_both(cv, cols, spec)
    _check_all(got, exp)


def test_unbounded_time_bins(cv):
    r = gen.make_c1(seed=3, n_journeys=40, median=600.0)
    got, exp = _run_both(cv, r.columns(), gen.GRIDS["c3"])
    _check_all(got, exp)


def test_long_segments_cell_reentry(cv):
    # 20 Hz journeys inside one long time bin, so (journey, bin) segments of tens
    # of thousands of records cross many tiles: journey 5 oscillates across a
    # cell edge (many re-entries found inside the LDS halo); journey 6 returns to
    # a cell after thousands of records elsewhere (found only by the global-memory
    # continuation of the backward scan)
    L = 30_000
    k = np.arange(L)
    lat5 = 37.01 + 0.0001 * np.sin(k / 37.0)
    lon5 = -92.004 + 0.0001 * np.cos(k / 53.0)
    pieces = [(2000, 37.015), (6000, 37.025), (3000, 37.015), (5000, 37.035), (1000, 37.025), (13000, 37.015)]
    lat6 = np.concatenate([np.full(m, v) + 1e-6 * np.arange(m) / m for m, v in pieces])
    lon6 = np.full(L, -91.995)
    jid = np.repeat(np.array([5, 6], np.int64), L)
    ts = gen.T0_MS + np.tile(k * 50, 2)
    lat = np.concatenate([lat5, lat6])
    lon = np.concatenate([lon5, lon6])
    spd = np.tile((k % 40).astype(np.float32), 2)
    spec = gen.GridSpec(36.0, -95.8, 0.01, 0.01, 460, 670, gen.T0_MS, 3_600_000, 24)
    got, exp = _run_both(cv, (jid, ts, lat, lon, spd), spec)
    _check_all(got, exp)
    # journey 6 visits 3 cells; each counts it once
    assert int(exp["groups"]["n_journeys"].max()) == 1 and len(exp["groups"]["key"]) >= 5


def test_long_segments_many_cells(cv):
    # 20 Hz journeys inside one hour-long time bin over 0.0001-degree cells: a
    # looping drift meets hundreds of cells in every tile, some new and some
    # entered thousands of records earlier in the same segment, so the
    # block-wide backward scan of a segment's earlier records runs several
    # rounds of pending keys; under every LDS table size
    rng = np.random.default_rng(12)
    L = 40_000
    k = np.arange(L)
    cols_j, cols_t, cols_la, cols_lo = [], [], [], []
    for j, (pa, pb) in enumerate(((150.0, 110.0), (90.0, 230.0))):
        cols_j.append(np.full(L, 11 + j, np.int64))
        cols_t.append(gen.T0_MS + k * 50)
        cols_la.append(37.0 + 2e-6 * k + 0.002 * np.sin(k / pa) + 1e-5 * rng.standard_normal(L))
        cols_lo.append(-92.0 + 0.002 * np.cos(k / pb) + 1e-5 * rng.standard_normal(L))
    cols = (np.concatenate(cols_j), np.concatenate(cols_t), np.concatenate(cols_la), np.concatenate(cols_lo),
            rng.gamma(2.0, 5.0, 2 * L).astype(np.float32))
    spec = gen.GridSpec(36.9, -92.1, 0.0001, 0.0001, 4000, 4000, gen.T0_MS, 3_600_000, 24)
    exp = oracle.run_plain(cols, spec)
    assert int(exp["groups"]["n_journeys"].max()) == 2 and len(exp["groups"]["key"]) > 10_000
    rec = cv.to_device(cols)
    print(f"[parity] long segments, n={2 * L}", flush=True)
    got = cv.run_plain(rec, spec)
    check_groups(got["groups"], got["n_out"], exp["groups"], exp["n_out"])


def test_step_angles_across_the_series_bound(cv):
    # consecutive fixes from millimetres to a quarter of the globe apart, dense
    # around the size where the half central angle (and the haversine's sqrt)
    # leaves the small-argument series for the library functions (2^-7 rad:
    # steps of about 100 km), in every direction
    rng = np.random.default_rng(21)
    n = 6000
    ang = np.concatenate([10.0 ** rng.uniform(-10, -0.3, n // 2),
                          (2.0 ** -6) * np.exp(rng.uniform(-0.05, 0.05, n - n // 2))])
    rng.shuffle(ang)
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    lat = np.empty(n)
    lon = np.empty(n)
    lat[0], lon[0] = 38.5, -92.5
    for i in range(1, n):
        d = np.degrees(ang[i])
        la = lat[i - 1] + d * np.cos(az[i])
        if abs(la) > 80.0:
            la = lat[i - 1] - d * np.cos(az[i])
        lat[i] = la
        lon[i] = (lon[i - 1] + d * np.sin(az[i]) + 180.0) % 360.0 - 180.0
    jid = np.repeat(np.arange(1, 7, dtype=np.int64), n // 6)
    ts = gen.T0_MS + 1000 * np.tile(np.arange(n // 6, dtype=np.int64), 6)
    spd = rng.gamma(2.0, 5.0, n).astype(np.float32)
    got, exp = _run_both(cv, (jid, ts, lat, lon, spd), gen.GRIDS["c1"])
    _check_all(got, exp)
    # the serving form: the same records in two pushes
    import torch
    st = cv.Stream(gen.GRIDS["c1"], 64, 1 << 16, n)
    rec = cv.to_device((jid, ts, lat, lon, spd))
    h = n // 2 + 17
    f1, _ = st.push({k: v[:h] for k, v in rec.items()})
    f2, _ = st.push({k: v[h:] for k, v in rec.items()})
    torch.cuda.synchronize()
    fs = {k: torch.cat([f1[k], f2[k]])[torch.from_numpy(exp["perm"].astype(np.int64)).cuda()] for k in f1}
    check_features(fs, exp["features"])


def test_table1_rows(cv):
    import json, os
    from test_oracle_pins import _table1, GOLDEN
    e = json.load(open(os.path.join(GOLDEN, "table1_expected.json")))
    cols = _table1()
    got, exp = _run_both(cv, cols, gen.GridSpec(**e["grid"]))
    _check_all(got, exp)
    assert host(got["perm"]).tolist() == e["sorted_input_rows"]


def test_empty_input(cv):
    import torch
    rec = cv.empty_records(0)
    perm, srt, r = cv.cv_sort_records(rec)
    assert perm.numel() == 0 and r["count"] == 0
    feat = cv.cv_journey_features(srt)
    summ, rs = cv.cv_journey_summary(srt, feat)
    groups, rg = cv.cv_grid_aggregate(srt, gen.GRIDS["c0"])
    assert rs["count"] == 0 and rg["count"] == 0 and rg["n_out_of_grid"] == 0
    torch.cuda.synchronize()


def test_capacity_retry_and_reporting(cv):
    r = gen.make_c0(seed=21, n_journeys=300, min_len=50, max_len=200)
    rec = cv.to_device(r)
    # too-small dictionary and output capacities: device reports, wrapper retries
    perm, srt, _, = cv.cv_sort_records(rec, max_journeys=None)
    _, _, res = cv.cv_sort_records(rec, max_journeys=16, sync=False)
    rr = cv.read_result(res)
    assert rr["status"] == cv.CV_ERR_CAPACITY and rr["required"] >= 300
    feat = cv.cv_journey_features(srt)
    _, res = cv.cv_journey_summary(srt, feat, capacity=10, sync=False)
    rr = cv.read_result(res)
    assert rr["status"] == cv.CV_ERR_CAPACITY and rr["required"] == 300
    summ, rs = cv.cv_journey_summary(srt, feat)
    assert rs["count"] == 300
    _, res = cv.cv_grid_aggregate(srt, gen.GRIDS["c0"], capacity=8, sync=False)
    rr = cv.read_result(res)
    assert rr["status"] == cv.CV_ERR_CAPACITY and rr["required"] > 8
    groups, rg = cv.cv_grid_aggregate(srt, gen.GRIDS["c0"])
    exp, _ = oracle.grid(*oracle.sorted_records(r.columns(), oracle.sort(r.journey_id, r.ts_ms)), gen.GRIDS["c0"])
    assert rg["count"] == len(exp["key"])


def test_deterministic_bitwise(cv):
    r = gen.make_c1(seed=91, n_journeys=60, median=900.0)
    rec = cv.to_device(r)
    a = cv.run_plain(rec, gen.GRIDS["c1"])
    b = cv.run_plain(rec, gen.GRIDS["c1"])
    for part in ("features", "summary", "groups"):
        for k in a[part]:
            assert np.array_equal(host(a[part][k]).view(np.uint8), host(b[part][k]).view(np.uint8)), (part, k)


def _wide_keys(seed, n, n_ids, tbits):
    """Records whose (journey rank, time offset) key is wide: n_ids distinct ids
    and time stamps spanning exactly tbits bits."""
    rng = np.random.default_rng(seed)
    ids = rng.choice(np.arange(-2 ** 40, 2 ** 40, 7919, dtype=np.int64), n_ids, replace=False)
    jid = ids[rng.integers(0, n_ids, n)]
    jid[:n_ids] = ids
    ts = gen.T0_MS + rng.integers(0, 2 ** tbits, n, dtype=np.int64)
    ts[0], ts[1] = gen.T0_MS, gen.T0_MS + 2 ** tbits - 1
    lat = rng.uniform(36.0, 40.6, n)
    lon = rng.uniform(-95.8, -89.1, n)
    spd = rng.uniform(0, 40, n).astype(np.float32)
    return jid, ts, lat, lon, spd


@pytest.mark.parametrize("tbits", [40, 45, 50, 54])
def test_packed_radix_passes(cv, tbits):
    # 5000 records (13 index bits), 1000 ids (10 rank bits): the key has
    # 10 + tbits bits, and passes from the first digit boundary p0 with
    # key_bits - d p0 + 13 <= 64 (d-bit digits) move packed (key | index) words
    n, n_ids = 5000, 1000
    cols = _wide_keys(100 + tbits, n, n_ids, tbits)
    got, exp = _run_both(cv, cols, gen.GRIDS["c0"])
    _check_all(got, exp)
    kb = 10 + tbits
    db = cv.cv_tuning_get("radix_bits")
    p0 = max(0, -(-(kb + 13 - 64) // db))
    assert got["sort_result"]["key_bits"] == kb
    assert got["sort_result"]["packed_pass"] == p0


@pytest.mark.parametrize("tbits", [15, 23])
@pytest.mark.parametrize("runs", [False, True])
def test_wide_first_digit(cv, tbits, runs):
    # 1000 ids (10 rank bits) and time offsets of tbits bits: a key of 8k + 1
    # bits (25, 33), packed from the first pass, takes a 9-bit first digit and
    # one pass fewer; the same input with 8-bit digits only must give the same
    # order.  Interleaved ids take the tiled key packing, ids in runs the
    # windowed one; 300 007 records span many tiles with a ragged last one.
    n, n_ids = 300_007, 1000
    cols = _wide_keys(300 + tbits, n, n_ids, tbits)
    if runs:
        o = np.argsort(cols[0], kind="stable")
        cols = tuple(c[o] for c in cols)
    kb = 10 + tbits
    exp = oracle.run_plain(cols, gen.GRIDS["c0"])
    rec = cv.to_device(cols)
    prev = cv.cv_tuning_get("radix_wide_first")
    try:
        for wide in (1, 0):
            cv.cv_tuning_set("radix_wide_first", wide)
            print(f"[parity] wide first digit {wide} key bits {kb} runs {runs} n={n}", flush=True)
            got = cv.run_plain(rec, gen.GRIDS["c0"])
            _check_all(got, exp)
            sr = got["sort_result"]
            assert sr["key_bits"] == kb and sr["packed_pass"] == 0
            shape_wide = cv.cv_tuning_get("sort_block") >= 512 and wide
            assert sr["flags"] == (9 if shape_wide else 8)
    finally:
        cv.cv_tuning_set("radix_wide_first", prev)


def test_every_sort_tile_shape(cv):
    # the record sort (and the group-key sort) under every compiled tile shape,
    # on an input of many tiles with a ragged last tile
    r = gen.make_c1(seed=12, n_journeys=70, median=900.0, shuffled=True)
    cols = r.columns()
    exp = oracle.run_plain(cols, gen.GRIDS["c1"])
    rec = cv.to_device(cols)
    prev = cv.cv_tuning_get("sort_shape")
    try:
        for sh in range(cv.cv_tuning_get("sort_shapes")):
            cv.cv_tuning_set("sort_shape", sh)
            print(f"[parity] sort shape {sh} tile {cv.cv_tuning_get('sort_tile')} n={r.n}", flush=True)
            got = cv.run_plain(rec, gen.GRIDS["c1"])
            check_sort(got["perm"], got["sorted"], exp["perm"], exp["sorted"])
            check_groups(got["groups"], got["n_out"], exp["groups"], exp["n_out"])
    finally:
        cv.cv_tuning_set("sort_shape", prev)


def test_extremes_in_exact_sums(cv):
    # speeds across the whole float32 range the sums must carry exactly
    # (subnormals, tiny and large magnitudes, both signs, signed zeros) and
    # steps far below the fast fixed-point range
    r = gen.make_c0(seed=404, n_journeys=60, min_len=50, max_len=400)
    rng = np.random.default_rng(405)
    n = r.n
    pool = np.array([1e-45, 3e-42, -7e-40, 1.2e-38, 1e-30, -1e-20, 9.3e-10, -1e-9, 2.0 ** -30, -(2.0 ** -31),
                     0.0, -0.0, 1.0, -3.5, 511.99, -1000.0, 1023.9, 7.25e-3], dtype=np.float32)
    spd = np.where(rng.random(n) < 0.5, pool[rng.integers(0, len(pool), n)],
                   rng.uniform(-40, 40, n).astype(np.float32)).astype(np.float32)
    # and steps below a micrometre: points a hair away from their predecessor
    # in (journey, time) order
    order = np.lexsort((r.ts_ms, r.journey_id))
    lat = r.lat_deg.copy()
    near = np.nonzero(rng.random(n) < 0.1)[0]
    near = near[near > 0]
    lat[order[near]] = lat[order[near - 1]] + rng.choice([1e-12, -3e-13, 2e-15], near.size)
    cols = (r.journey_id, r.ts_ms, lat, r.lon_deg, spd)
    got, exp = _run_both(cv, cols, gen.GRIDS["c0"])
    _check_all(got, exp)


def test_summary_flags_column_at_any_alignment(cv):
    # the journey counts read the features' flags 16 bytes per lane when the
    # column is 16-byte aligned, byte by byte otherwise: same rows either way
    import torch
    r = gen.make_c1(seed=46, n_journeys=40, median=600.0)
    print(f"[parity] unaligned flags n={r.n}", flush=True)
    rec = cv.to_device(r)
    _, srt, _ = cv.cv_sort_records(rec)
    feat = cv.cv_journey_features(srt)
    a, ra = cv.cv_journey_summary(srt, feat)
    buf = torch.zeros(r.n + 1, dtype=torch.uint8, device=feat["flags"].device)
    buf[1:] = feat["flags"]
    feat2 = dict(feat)
    feat2["flags"] = buf[1:]
    b, rb = cv.cv_journey_summary(srt, feat2)
    assert ra["count"] == rb["count"]
    for k in a:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("case", ["c0", "c1_small", "long_segments", "ragged"])
def test_grid_from_first_flags_equals_id_compare(cv, case):
    # the grid with journey starts from the kinematics' FIRST flags and the one
    # that compares journey ids give the same bits, and both equal the oracle
    import torch
    if case == "c0":
        cols, spec = gen.make_c0(seed=5).columns(), gen.GRIDS["c0"]
    elif case == "c1_small":
        cols, spec = gen.make_c1(seed=8, n_journeys=60, median=900.0).columns(), gen.GRIDS["c1"]
    elif case == "long_segments":
        # a few journeys re-entering cells within long one-hour bins
        r = gen.make_c1(seed=9, n_journeys=6, median=30_000.0)
        cols = r.columns()
        spec = gen.GridSpec(36.0, -95.8, 0.0005, 0.0005, 9200, 13400, gen.T0_MS, 3_600_000, 24)
    else:
        cols, spec = gen.make_c1(seed=10, n_journeys=33, median=700.0, shuffled=True).columns(), gen.GRIDS["c1"]
    print(f"[parity] grid from flags, {case}, n={len(cols[0])}", flush=True)
    exp = oracle.run_plain(cols, spec)
    rec = cv.to_device(cols)
    perm, srt, _ = cv.cv_sort_records(rec)
    feat = cv.cv_journey_features(srt)
    a, ra = cv.cv_grid_aggregate(srt, spec, flags=feat["flags"])
    b, rb = cv.cv_grid_aggregate(srt, spec)
    assert ra["count"] == rb["count"] and ra["n_out_of_grid"] == rb["n_out_of_grid"]
    for k in a:
        assert torch.equal(a[k], b[k]), k
    check_groups(a, ra["n_out_of_grid"], exp["groups"], exp["n_out"])


@pytest.mark.parametrize("unit,factor", [(1000, 1000), (50, 50), (1024, 1024), (375, 125), (7, 1), (2 ** 40, 2 ** 40)])
def test_time_offsets_common_factor(cv, unit, factor):
    # time stamps on a grid of `unit` ms (a sampling period), unordered: the
    # key's time offset is divided by the offsets' common factor of the form
    # 2^a 5^b, so it needs fewer bits; the sorted time stamps, decoded from the
    # key, must equal the oracle's exactly
    rng = np.random.default_rng(unit % 997 + 3)
    n, n_ids = 40_000, 300
    ids = rng.choice(np.arange(-2 ** 40, 2 ** 40, 7919, dtype=np.int64), n_ids, replace=False)
    jid = ids[rng.integers(0, n_ids, n)]
    steps = rng.integers(0, 5000, n).astype(np.int64)
    steps[:3] = [0, 1, 2]  # consecutive multiples: the common factor is unit's own
    ts = gen.T0_MS - 123 * unit + unit * steps
    lat = rng.uniform(36.0, 40.6, n)
    lon = rng.uniform(-95.8, -89.1, n)
    spd = rng.uniform(0, 40, n).astype(np.float32)
    got, exp = _run_both(cv, (jid, ts, lat, lon, spd), gen.GRIDS["c0"])
    _check_all(got, exp)
    span = int(ts.max() - ts.min())
    assert span % factor == 0
    assert got["sort_result"]["key_bits"] == _bw(n_ids - 1) + _bw(span // factor)


def _bw(x):
    return int(x).bit_length()


@pytest.mark.parametrize("bin_ms", [1, 7, 60_000, 2 ** 30 - 1, 2 ** 30, 2 ** 31 + 5])
def test_time_bins_across_offset_ranges(cv, bin_ms):
    # an unbounded time axis, so every time bin is a key: offsets from t0
    # around 0, on and next to bin edges, around +-2^30 (where the quotient's
    # correction leaves 32-bit arithmetic) and around 2^52 (where the integer
    # division takes over), negative offsets (out of the grid) included
    rng = np.random.default_rng(bin_ms % 1000 + 5)
    spec = gen.GridSpec(36.0, -95.8, 0.5, 0.5, 10, 14, gen.T0_MS, bin_ms, 0)
    centres = [0, 2 ** 30, -(2 ** 30), 2 ** 31, 2 ** 40 + 3, 2 ** 52, 2 ** 53 + 9, 5 * bin_ms, 2 ** 30 // bin_ms * bin_ms]
    offs = []
    for c in centres:
        offs += [c + d for d in range(-3, 4)]
        offs += [(c // bin_ms + e) * bin_ms + d for e in (-1, 0, 1) for d in (-1, 0, 1)]
    offs = np.array(sorted(set(offs)), dtype=np.int64)
    n = len(offs) * 3
    ts = gen.T0_MS + np.repeat(offs, 3)
    jid = np.repeat(np.arange(n // 12 + 1, dtype=np.int64), 12)[:n]
    lat = rng.uniform(36.0, 40.9, n)
    lon = rng.uniform(-95.8, -88.9, n)
    spd = rng.uniform(0, 40, n).astype(np.float32)
    got, exp = _run_both(cv, (jid, ts, lat, lon, spd), spec)
    _check_all(got, exp)
    assert len(exp["groups"]["key"]) > len(offs) // 2


def test_cell_boundaries_and_neighbours(cv):
    # coordinates on cell boundaries k * d from the origin and one or two ulps
    # either side, and time stamps on bin edges: every key must equal the
    # oracle's floor of the IEEE quotient (the kernel divides as the oracle
    # does; a boundary is where any shortcut would show)
    rng = np.random.default_rng(47)
    spec = gen.GRIDS["c1"]
    n = 6000
    k_lat = rng.integers(0, spec.n_lat, n)
    k_lon = rng.integers(0, spec.n_lon, n)
    lat = spec.lat0_deg + k_lat * spec.dlat_deg
    lon = spec.lon0_deg + k_lon * spec.dlon_deg
    nudge = rng.integers(-2, 3, (2, n))
    for _ in range(2):
        lat = np.where(nudge[0] > 0, np.nextafter(lat, np.inf), np.where(nudge[0] < 0, np.nextafter(lat, -np.inf), lat))
        lon = np.where(nudge[1] > 0, np.nextafter(lon, np.inf), np.where(nudge[1] < 0, np.nextafter(lon, -np.inf), lon))
        nudge = np.where(np.abs(nudge) == 2, nudge, 0)
    jid = np.repeat(np.arange(60, dtype=np.int64), n // 60)
    ts = spec.t0_ms + rng.integers(0, 288, n).astype(np.int64) * spec.bin_ms + rng.integers(-1, 2, n)
    ts = np.sort(ts.reshape(60, -1), axis=1).reshape(-1)
    spd = rng.uniform(0, 40, n).astype(np.float32)
    got, exp = _run_both(cv, (jid, ts, lat, lon, spd), spec)
    _check_all(got, exp)
