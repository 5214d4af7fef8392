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
