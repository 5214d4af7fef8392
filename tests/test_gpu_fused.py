"""Sort fused with the kinematics (cv_sort_records_features and its batched
form) against the oracle, and bit for bit against the two separate calls
(cv_sort_records + cv_journey_features), on ragged sizes around the fused
kernel's 512-record tile, adversarial columns and uneven shards, with input
both in journey runs (the gather reads the columns) and interleaved (it reads
the payload packed per record)."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import assert_exact, check_features, check_sort, host

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


def _same_bits(name, a, b):
    assert_exact(name, host(a), host(b))


def _fused_vs_separate(cv, cols, mj):
    rec = cv.to_device(cols)
    perm, srt, feat, r = cv.cv_sort_records_features(rec, mj)
    perm2, srt2, _ = cv.cv_sort_records(rec, max_journeys=mj)
    feat2 = cv.cv_journey_features(srt2)
    _same_bits("perm", perm, perm2)
    for k in srt:
        _same_bits(f"sorted.{k}", srt[k], srt2[k])
    for k in feat:
        _same_bits(f"features.{k}", feat[k], feat2[k])
    return perm, srt, feat, r


@pytest.mark.parametrize("n", [1, 2, 3, 511, 512, 513, 1023, 1024, 1025, 4097, 70001])
def test_fused_ragged_sizes(cv, n):
    r = gen.make_c0(seed=2000 + n, n_journeys=max(1, n // 40 + 1), min_len=1, max_len=80)
    cols = tuple(c[:n] for c in r.columns())
    print(f"[fused] n={n}", flush=True)
    perm, srt, feat, _ = _fused_vs_separate(cv, cols, 1 << 16)
    exp = oracle.run_plain(cols, gen.GRIDS["c0"])
    check_sort(perm, srt, exp["perm"], exp["sorted"])
    check_features(feat, exp["features"])


def test_fused_adversarial_columns(cv):
    rng = np.random.default_rng(19)
    n = 9000
    ids = np.array([-(2 ** 63), 2 ** 63 - 1, -1, 0, 1, 12345], dtype=np.int64)
    jid = ids[rng.integers(0, len(ids), n)]
    ts = gen.T0_MS + rng.integers(-5, 40, n).astype(np.int64) * 30_000
    lat = rng.uniform(35.9, 40.7, n)
    lon = rng.uniform(-95.9, -89.0, n)
    lat[rng.random(n) < 0.02] = np.nan
    lon[rng.random(n) < 0.02] = -np.inf
    spd = rng.uniform(0, 40, n).astype(np.float32)
    cols = (jid, ts, lat, lon, spd)
    print(f"[fused] adversarial n={n}", flush=True)
    perm, srt, feat, _ = _fused_vs_separate(cv, cols, 64)
    exp = oracle.run_plain(cols, gen.grid_for(0.01, 60_000))
    check_sort(perm, srt, exp["perm"], exp["sorted"])
    check_features(feat, exp["features"])


def test_fused_wide_timestamps(cv):
    # a time span too wide for the packed key: time stamps are gathered from
    # the input column rather than rebuilt from the sorted words
    r = gen.make_c0(seed=77, n_journeys=30, min_len=20, max_len=200)
    cols = list(r.columns())
    cols[1] = cols[1].copy()
    cols[1][::7] += np.int64(1) << 50
    print(f"[fused] wide ts n={len(cols[0])}", flush=True)
    perm, srt, feat, _ = _fused_vs_separate(cv, tuple(cols), 1024)
    exp = oracle.run_plain(tuple(cols), gen.GRIDS["c0"])
    check_sort(perm, srt, exp["perm"], exp["sorted"])
    check_features(feat, exp["features"])


def test_fused_batched_shards(cv):
    import torch
    base = gen.make_c2(seed=41, n_shards=6, total=90_000, lo=300, hi=40_000)
    empty = gen.Records(*(c[:0] for c in base[0].columns()))
    tiny = gen.Records(*(c[:1] for c in base[1].columns()))
    shards = [empty, base[0], tiny, base[1], empty, base[2], base[3], base[4], base[5], empty]
    sizes = [s.n for s in shards]
    allr = gen.concat(shards)
    print(f"[fused] batched shards={len(shards)} n={allr.n}", flush=True)
    rec = cv.to_device(allr)
    _, off_d = cv.shard_offsets(sizes, rec["journey_id"].device)
    perm, srt, feat, _ = cv.cv_sort_records_features(rec, 1 << 16, shard_offsets=off_d)
    sep = cv.BatchPipeline(allr.n, len(sizes), gen.GRIDS["c2"], 1 << 16, 1 << 16, 1 << 20,
                           rec["journey_id"].device, fused=False)
    sep.run(rec, off_d)
    torch.cuda.synchronize()
    _same_bits("perm", perm, sep.perm)
    for k in srt:
        _same_bits(f"sorted.{k}", srt[k], sep.sorted[k])
    for k in feat:
        _same_bits(f"features.{k}", feat[k], sep.feat[k])
    off = np.concatenate([[0], np.cumsum(sizes)])
    for s, sh in enumerate(shards):
        a, b = int(off[s]), int(off[s + 1])
        exp = oracle.run_plain(sh.columns(), gen.GRIDS["c2"])
        check_sort(perm[a:b], {k: v[a:b] for k, v in srt.items()}, exp["perm"], exp["sorted"])
        check_features({k: v[a:b] for k, v in feat.items()}, exp["features"])


def test_fused_rejects_missing_columns(cv):
    import ctypes
    L = cv.lib()
    r = gen.make_c0(seed=3, n_journeys=2, min_len=5, max_len=10)
    rec = cv.to_device(r)
    n = int(rec["journey_id"].numel())
    so = cv.CvRecordsOut()
    fs = cv.CvFeatures()
    st = L.cv_sort_records_features(ctypes.byref(cv._records_struct(rec)), 16, None, ctypes.byref(so),
                                    ctypes.byref(fs), None, None, 0, None)
    assert n > 0 and st == cv.CV_ERR_INVALID_ARGUMENT


def _mean_run(jid):
    jid = np.asarray(jid)
    return len(jid) / max(1, 1 + int(np.count_nonzero(jid[1:] != jid[:-1])))


def test_fused_contiguous_input(cv):
    # journeys in runs (per-journey files): the gather reads the input columns
    r = gen.make_c1(seed=44, n_journeys=60, median=900.0)
    assert _mean_run(r.journey_id) >= 8
    print(f"[fused] contiguous n={r.n}", flush=True)
    perm, srt, feat, _ = _fused_vs_separate(cv, r.columns(), 1024)
    exp = oracle.run_plain(r.columns(), gen.GRIDS["c1"])
    check_sort(perm, srt, exp["perm"], exp["sorted"])
    check_features(feat, exp["features"])


def test_fused_payload_forms_agree(cv):
    # the same records (no repeated (id, time) pair, so the sorted order does
    # not depend on the input order) once in journey runs and once interleaved:
    # the gather reads the columns in the first case and the packed per-record
    # payload in the second; sorted columns and features must be the same bits
    rng = np.random.default_rng(45)
    n_j, per = 300, 200
    jid = np.repeat(rng.choice(np.arange(10**6, dtype=np.int64), n_j, replace=False), per)
    ts = gen.T0_MS + np.tile(np.arange(per, dtype=np.int64) * 1000, n_j) + np.repeat(rng.integers(0, 10**6, n_j), per)
    lat = 38.0 + np.cumsum(rng.normal(0, 2e-4, n_j * per))
    lon = -92.0 + np.cumsum(rng.normal(0, 2e-4, n_j * per))
    lat[rng.random(n_j * per) < 0.003] = np.nan
    spd = rng.uniform(0, 40, n_j * per).astype(np.float32)
    a = (jid, ts, lat, lon, spd)
    shuf = rng.permutation(n_j * per)
    b = tuple(c[shuf] for c in a)
    assert _mean_run(a[0]) >= 8 and _mean_run(b[0]) < 8
    print(f"[fused] payload forms n={n_j * per}", flush=True)
    pa, sa, fa, _ = cv.cv_sort_records_features(cv.to_device(a), 4096)
    pb, sb, fb, _ = cv.cv_sort_records_features(cv.to_device(b), 4096)
    for k in sa:
        _same_bits(f"sorted.{k}", sa[k], sb[k])
    for k in fa:
        _same_bits(f"features.{k}", fa[k], fb[k])
    # both index the same original records
    assert np.array_equal(host(pa).astype(np.int64), shuf[host(pb).astype(np.int64)])


def _mix64(x):
    m = (1 << 64) - 1
    x &= m
    x ^= x >> 30
    x = (x * 0xbf58476d1ce4e5b9) & m
    x ^= x >> 27
    x = (x * 0x94d049bb133111eb) & m
    x ^= x >> 31
    return x


def test_dictionary_cache_slot_collisions(cv):
    # 96 journey ids whose dictionary-cache slot (top bits of the 64-bit mix
    # of the id) is the same, interleaved at random: every
    # lane of a window competes for one cache slot in the insert and in the
    # key packing, and the sort must still match the oracle
    ids = []
    x = 1
    while len(ids) < 96:
        if (_mix64(x) >> 55) == 34:  # one slot at every power-of-two slot count up to 512
            ids.append(x)
        x += 1
    rng = np.random.default_rng(48)
    per = 120
    jid = np.repeat(np.array(ids, dtype=np.int64), per)
    ts = gen.T0_MS + np.tile(np.arange(per, dtype=np.int64) * 1000, len(ids))
    lat = 38.0 + rng.normal(0, 1e-3, len(jid))
    lon = -92.0 + rng.normal(0, 1e-3, len(jid))
    spd = rng.uniform(0, 30, len(jid)).astype(np.float32)
    order = rng.permutation(len(jid))
    cols = tuple(c[order] for c in (jid, ts, lat, lon, spd))
    print(f"[fused] cache collisions n={len(jid)}", flush=True)
    perm, srt, feat, r = _fused_vs_separate(cv, cols, 1024)
    assert r["count"] == len(ids)
    exp = oracle.run_plain(cols, gen.GRIDS["c1"])
    check_sort(perm, srt, exp["perm"], exp["sorted"])
    check_features(feat, exp["features"])
