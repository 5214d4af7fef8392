"""Record hygiene: dropping exact duplicate rows and splitting journeys into
trips at time gaps.  HIP path vs the oracle's definitions, exactly."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import assert_exact, check_features, check_summary, host

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


def _with_copies(seed, frac):
    """Full-day-shaped rows (per-journey files) plus exact copies of a fraction of them (some copied
    twice), each inserted at a random later position, and near copies that
    differ in one bit of the speed."""
    r = gen.make_c1(seed=seed, n_journeys=70, median=800.0)
    rng = np.random.default_rng(seed)
    cols = [np.asarray(c) for c in r.columns()]
    n = r.n
    src = rng.choice(n, int(frac * n), replace=False)
    src = np.concatenate([src, src[: len(src) // 5]])          # triplicates too
    near = rng.choice(n, int(0.01 * n), replace=False)
    extra = [c[np.concatenate([src, near])].copy() for c in cols]
    extra[4][len(src):] = (extra[4][len(src):].view(np.uint32) ^ 1).view(np.float32)
    pos = rng.integers(0, n, len(extra[0]))
    order = np.argsort(np.concatenate([np.arange(n), pos + 0.5]), kind="stable")
    return tuple(np.concatenate([c, e])[order] for c, e in zip(cols, extra))


def test_drop_duplicates_matches_oracle(cv):
    cols = _with_copies(51, 0.03)
    print(f"[hygiene] duplicates n={len(cols[0])}", flush=True)
    rec = cv.to_device(cols)
    perm, srt, _ = cv.cv_sort_records(rec)
    kept, kperm, r = cv.cv_drop_duplicates(srt, perm)
    ep = oracle.sort(cols[0], cols[1])
    s = oracle.sorted_records(cols, ep)
    keep = oracle.drop_duplicates(s)
    assert r["count"] == len(keep) and len(keep) < len(cols[0])
    assert_exact("kept perm", host(kperm).astype(np.int64), ep[keep])
    for (k, _), c in zip(cv.RECORD_FIELDS, s):
        got = host(kept[k])
        assert_exact(f"kept {k}", got.view(np.uint8), np.ascontiguousarray(c[keep]).view(np.uint8))
    # the rest of the path on the kept records equals the oracle on the
    # input without its duplicate rows
    dedup = tuple(c[ep[np.sort(keep)]] for c in cols)
    exp = oracle.run_plain(tuple(c[ep[keep]] for c in cols), gen.GRIDS["c1"])
    feat = cv.cv_journey_features(kept)
    summ, _ = cv.cv_journey_summary(kept, feat)
    check_features(feat, exp["features"])
    check_summary(summ, exp["summary"])
    assert len(dedup[0]) == len(keep)


@pytest.mark.parametrize("gap_ms", [0, 1000, 5000, 60_000, 10**12])
def test_split_trips_matches_oracle(cv, gap_ms):
    r = gen.make_c1(seed=52, n_journeys=60, median=900.0, shuffled=True)
    # holes: drop a few stretches of records so that journeys have gaps
    rng = np.random.default_rng(52)
    m = np.ones(r.n, bool)
    for a in rng.integers(0, r.n - 200, 40):
        m[a:a + rng.integers(5, 150)] = False
    cols = tuple(np.asarray(c)[m] for c in r.columns())
    print(f"[hygiene] trips n={len(cols[0])} gap={gap_ms}", flush=True)
    rec = cv.to_device(cols)
    perm, srt, _ = cv.cv_sort_records(rec)
    tid, tj, res = cv.cv_split_trips(srt, gap_ms)
    ep = oracle.sort(cols[0], cols[1])
    s = oracle.sorted_records(cols, ep)
    et, ej = oracle.split_trips(s[0], s[1], gap_ms)
    assert_exact("trip_id", host(tid), et)
    assert_exact("trip_journey", host(tj), ej)
    assert res["count"] == len(ej)
    if gap_ms == 5000:
        # trips as journeys: the summary of the records keyed by trip
        trip_rec = dict(srt)
        trip_rec["journey_id"] = tid
        feat = cv.cv_journey_features(trip_rec)
        summ, _ = cv.cv_journey_summary(trip_rec, feat)
        exp = oracle.run_plain((et, s[1], s[2], s[3], s[4]), gen.GRIDS["c1"])
        check_summary(summ, exp["summary"])


def test_hygiene_empty_and_capacity(cv):
    import torch
    empty = cv.empty_records(0)
    kept, _, r = cv.cv_drop_duplicates(empty)
    assert r["count"] == 0
    tid, tj, r = cv.cv_split_trips(empty, 1000)
    assert r["count"] == 0
    rr = gen.make_c0(seed=53, n_journeys=5, min_len=20, max_len=40)
    perm, srt, _ = cv.cv_sort_records(cv.to_device(rr))
    with pytest.raises(cv.CvError):
        cv.cv_split_trips(srt, 1000, capacity=2)
