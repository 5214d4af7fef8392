"""Serving form: a stream of chunks pushed in batches must give the plain
path's results on the concatenation (oracle), and each chunk's response must
not depend on which other chunks share its push ("alone == in the mix")."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import check_features, check_groups, check_summary, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    cvetl.lib()
    return cvetl


def _pool(seed=41, n_journeys=60, median=600.0, heavy=0.0):
    return gen.make_stream(seed=seed, n_journeys=n_journeys, median=median, heavy_frac=heavy, heavy_cap=20_000)


def _slices(n, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)])
    return [(int(off[i]), int(off[i + 1])) for i in range(len(sizes))]


def _to_sorted_order(feat, perm):
    """Features indexed by input position -> indexed by sorted position."""
    import torch
    idx = torch.from_numpy(perm.astype(np.int64)).to(next(iter(feat.values())).device)
    return {k: v[idx] for k, v in feat.items()}


@pytest.mark.parametrize("grid_name,heavy", [("c3", 0.0), ("c4", 0.05)])
def test_stream_matches_oracle_on_concatenation(cv, grid_name, heavy):
    import torch
    r = _pool(seed=41 if heavy == 0 else 42, heavy=heavy)
    grid = gen.GRIDS[grid_name]
    rng = np.random.default_rng(7)
    sizes = gen.chunk_sizes(rng, r.n, 500, 30_000)
    print(f"[stream] n={r.n} chunks={len(sizes)} grid={grid_name}", flush=True)
    st = cv.Stream(grid, max_journeys=4096, max_groups=1 << 18, max_batch=max(sizes))
    rec = cv.to_device(r)
    feats = []
    for a, b in _slices(r.n, sizes):
        f, res = st.push({k: v[a:b] for k, v in rec.items()})
        feats.append(f)
    torch.cuda.synchronize()
    got_f = {k: torch.cat([f[k] for f in feats]) for k in feats[0]}
    journeys, groups, rj, rg = st.flush(4096, 1 << 18)
    exp = oracle.run_plain(r.columns(), grid)
    check_features(_to_sorted_order(got_f, exp["perm"]), exp["features"])
    check_summary(journeys, exp["summary"])
    check_groups(groups, rj["n_out_of_grid"], exp["groups"], exp["n_out"])
    assert rj["n_late"] == 0


def test_alone_equals_in_the_mix(cv):
    import torch
    r = _pool(seed=43)
    grid = gen.GRIDS["c3"]
    sizes = gen.chunk_sizes(np.random.default_rng(8), r.n, 2_000, 20_000)
    sl = _slices(r.n, sizes)
    rec = cv.to_device(r)
    mb = r.n
    a = cv.Stream(grid, 4096, 1 << 18, mb)
    b = cv.Stream(grid, 4096, 1 << 18, mb)
    fa, fb = [], []
    # a: one chunk per push; b: groups of three consecutive chunks per push
    for x, y in sl:
        fa.append(a.push({k: v[x:y] for k, v in rec.items()})[0])
    i = 0
    while i < len(sl):
        grp = sl[i:i + 3]
        x, y = grp[0][0], grp[-1][1]
        f, _ = b.push({k: v[x:y] for k, v in rec.items()})
        for (cx, cy) in grp:
            fb.append({k: v[cx - x:cy - x] for k, v in f.items()})
        i += 3
    torch.cuda.synchronize()
    for c, (u, v) in enumerate(zip(fa, fb)):
        for k in u:
            assert torch.equal(u[k].view(torch.uint8), v[k].view(torch.uint8)), (c, k)
    ja, ga, _, _ = a.flush(4096, 1 << 18)
    jb, gb, _, _ = b.flush(4096, 1 << 18)
    for k in ja:
        assert torch.equal(ja[k].view(torch.uint8), jb[k].view(torch.uint8)), k
    for k in ga:
        assert torch.equal(ga[k].view(torch.uint8), gb[k].view(torch.uint8)), k


def test_late_records_flagged(cv):
    import torch
    grid = gen.GRIDS["c3"]
    jid = np.array([9, 9, 9, 9], np.int64)
    ts = gen.T0_MS + np.array([0, 1000, 5000, 3000], np.int64)   # last one arrives late
    lat = np.array([37.0, 37.0001, 37.0002, 37.0003])
    lon = np.full(4, -92.0)
    spd = np.ones(4, np.float32)
    st = cv.Stream(grid, 64, 4096, 16)
    rec = cv.to_device((jid, ts, lat, lon, spd))
    f1, r1 = st.push({k: v[:3] for k, v in rec.items()})
    f2, r2 = st.push({k: v[3:] for k, v in rec.items()})
    torch.cuda.synchronize()
    assert cv.read_result(r2)["n_late"] == 1
    assert int(host(f2["flags"])[0]) == 0x80 and host(f2["step_m"])[0] == 0.0
    journeys, groups, rj, rg = st.flush(64, 4096)
    assert int(host(journeys["n_points"])[0]) == 4 and rj["n_late"] == 1
    assert int(host(groups["count"]).sum()) == 4


def _delayed_arrival(n, rng, frac, reach):
    """Arrival order in which a fraction of the records is held back by up to
    `reach` positions (so that some arrive after later records of their
    journey were pushed)."""
    key = np.arange(n, dtype=np.float64)
    pick = rng.random(n) < frac
    key[pick] += rng.integers(1, reach, int(pick.sum()))
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("grid_name,heavy", [("c3", 0.0), ("c4", 0.05)])
def test_late_records_in_bulk(cv, grid_name, heavy):
    """Late records in quantity: kinematics and distinct-journey flags follow
    the non-late records alone; counts, sums and extrema of cells and journeys
    include every record."""
    import torch
    r = _pool(seed=44 if heavy == 0 else 45, heavy=heavy)
    grid = gen.GRIDS[grid_name]
    rng = np.random.default_rng(9)
    order = _delayed_arrival(r.n, rng, 0.03, 20_000)
    cols = tuple(np.ascontiguousarray(c[order]) for c in r.columns())
    sizes = gen.chunk_sizes(rng, r.n, 500, 30_000)
    bounds = _slices(r.n, sizes)
    late = oracle.stream_late(cols[0], cols[1], sizes)
    print(f"[stream-late] n={r.n} chunks={len(sizes)} late={int(late.sum())} grid={grid_name}", flush=True)
    assert late.sum() > 100
    st = cv.Stream(grid, max_journeys=4096, max_groups=1 << 18, max_batch=max(sizes))
    rec = cv.to_device(cols)
    feats, n_late = [], 0
    for a, b in bounds:
        f, res = st.push({k: v[a:b] for k, v in rec.items()})
        feats.append(f)
        n_late += cv.read_result(res)["n_late"]
    torch.cuda.synchronize()
    got = {k: host(torch.cat([f[k] for f in feats])) for k in feats[0]}
    journeys, groups, rj, rg = st.flush(4096, 1 << 18)
    assert n_late == int(late.sum()) and rj["n_late"] == int(late.sum())
    # kinematics: the non-late records on their own
    keep = np.flatnonzero(~late)
    sub = tuple(c[keep] for c in cols)
    exp_nl = oracle.run_plain(sub, grid)
    check_features({k: torch.from_numpy(v[keep][exp_nl["perm"]]) for k, v in got.items()}, exp_nl["features"])
    lt = np.flatnonzero(late)
    assert np.all(got["flags"][lt] == 0x80)
    for k in ("step_m", "dt_s", "speed_mps", "accel_mps2", "bearing_deg", "dheading_deg"):
        assert np.all(got[k][lt] == 0.0), k
    # journeys: every record, late ones with zero kinematics
    full = {k: np.zeros(r.n, dtype=v.dtype) for k, v in exp_nl["features"].items()}
    for k, v in exp_nl["features"].items():
        full[k][keep[exp_nl["perm"]]] = v
    full["flags"][lt] = 0x80
    perm = oracle.sort(cols[0], cols[1])
    s_all = oracle.sorted_records(cols, perm)
    check_summary(journeys, oracle.summary(*s_all, {k: v[perm] for k, v in full.items()}))
    # cells: count / sum / extrema over every record, distinct journeys over the non-late ones
    exp_g, n_out = oracle.grid(*s_all, grid)
    nj = dict(zip(exp_nl["groups"]["key"].tolist(), exp_nl["groups"]["n_journeys"].tolist()))
    exp_g["n_journeys"] = np.array([nj.get(k, 0) for k in exp_g["key"].tolist()], dtype=np.uint32)
    check_groups(groups, rj["n_out_of_grid"], exp_g, n_out)


def _push_all(st, rec, bounds):
    feats = []
    for a, b in bounds:
        f, _ = st.push({k: v[a:b] for k, v in rec.items()})
        feats.append(f)
    return feats


@pytest.mark.parametrize("grid_name,heavy", [("c3", 0.0), ("c4", 0.05)])
def test_snapshot_restore_resumes_bit_identically(cv, grid_name, heavy):
    """push[0:k], snapshot, restore into a fresh stream, push[k:]: every
    response and the flush equal the uninterrupted run bit for bit, and the
    flush equals the oracle on the concatenation."""
    import torch
    r = _pool(seed=46 if heavy == 0 else 47, heavy=heavy)
    grid = gen.GRIDS[grid_name]
    sizes = gen.chunk_sizes(np.random.default_rng(10), r.n, 500, 30_000)
    bounds = _slices(r.n, sizes)
    k = len(bounds) // 2
    print(f"[snapshot] n={r.n} chunks={len(sizes)} split at {k} grid={grid_name}", flush=True)
    rec = cv.to_device(r)
    mb = max(sizes)
    whole = cv.Stream(grid, 4096, 1 << 18, mb)
    fw = _push_all(whole, rec, bounds)
    first = cv.Stream(grid, 4096, 1 << 18, mb)
    f1 = _push_all(first, rec, bounds[:k])
    snap = first.snapshot()
    first.close()
    resumed = cv.Stream(grid, 4096, 1 << 18, 2 * mb)   # the per-push capacity may differ
    resumed.restore(snap)
    f2 = _push_all(resumed, rec, bounds[k:])
    torch.cuda.synchronize()
    for c, (u, v) in enumerate(zip(fw, f1 + f2)):
        for key in u:
            assert torch.equal(u[key].view(torch.uint8), v[key].view(torch.uint8)), (c, key)
    ja, ga, rja, rga = whole.flush(4096, 1 << 18)
    jb, gb, rjb, rgb = resumed.flush(4096, 1 << 18)
    for key in ja:
        assert torch.equal(ja[key].view(torch.uint8), jb[key].view(torch.uint8)), key
    for key in ga:
        assert torch.equal(ga[key].view(torch.uint8), gb[key].view(torch.uint8)), key
    assert rja == rjb and rga == rgb
    exp = oracle.run_plain(r.columns(), grid)
    check_summary(jb, exp["summary"])
    check_groups(gb, rjb["n_out_of_grid"], exp["groups"], exp["n_out"])


def test_restore_rejects_other_capacities(cv):
    grid = gen.GRIDS["c3"]
    a = cv.Stream(grid, 4096, 1 << 18, 1000)
    snap = a.snapshot()
    b = cv.Stream(grid, 8192, 1 << 18, 1000)
    with pytest.raises(cv.CvError):
        b.restore(snap)
    c = cv.Stream(gen.GRIDS["c4"], 4096, 1 << 18, 1000)
    with pytest.raises(cv.CvError):
        c.restore(snap)


def test_stream_extreme_journey_ids(cv):
    """Journey ids INT64_MIN and INT64_MAX (INT64_MIN is the journey table's
    empty-slot marker) next to ordinary ones, over several pushes."""
    import torch
    r = _pool(seed=48, n_journeys=12, median=400.0)
    jid = r.journey_id.copy()
    u = np.unique(jid)
    jid[jid == u[0]] = np.iinfo(np.int64).min
    jid[jid == u[1]] = np.iinfo(np.int64).max
    jid[jid == u[2]] = -1
    cols = (jid, r.ts_ms, r.lat_deg, r.lon_deg, r.speed_mps)
    grid = gen.GRIDS["c3"]
    sizes = gen.chunk_sizes(np.random.default_rng(11), r.n, 200, 3_000)
    st = cv.Stream(grid, 256, 1 << 16, max(sizes))
    rec = cv.to_device(cols)
    feats = _push_all(st, rec, _slices(r.n, sizes))
    torch.cuda.synchronize()
    got_f = {k: torch.cat([f[k] for f in feats]) for k in feats[0]}
    journeys, groups, rj, rg = st.flush(256, 1 << 16)
    exp = oracle.run_plain(cols, grid)
    assert host(journeys["journey_id"])[0] == np.iinfo(np.int64).min
    assert host(journeys["journey_id"])[-1] == np.iinfo(np.int64).max
    check_features(_to_sorted_order(got_f, exp["perm"]), exp["features"])
    check_summary(journeys, exp["summary"])
    check_groups(groups, rj["n_out_of_grid"], exp["groups"], exp["n_out"])
