"""Full-size parity on the full-day workload (~123 M records), in the launch
configuration the benchmark times (preallocated Pipeline, same capacities).

The order is checked by its defining properties on every record; journeys
are sampled and recomputed one by one by the oracle from their own input
records (journeys are independent); grid cells are sampled and recomputed
from all records that the oracle's binning puts in them; and the oracle over
the whole day is compared with every output element by element."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import assert_exact, assert_rel, check_features, host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def day():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl, tune
    print("[fullsize] generating the full-day workload", flush=True)
    r = gen.make_c1()
    prev = cvetl.cv_tuning_get("sort_shape")
    tune.apply(r.n)        # the tile shape the benchmark uses for this size
    print(f"[fullsize] sort shape {cvetl.cv_tuning_get('sort_shape')}", flush=True)
    grid = gen.GRIDS["c1"]
    rec = cvetl.to_device(r)
    out = cvetl.run_plain(rec, grid)
    J = out["summary_result"]["count"]
    G = out["grid_result"]["count"]
    del out
    pipe = cvetl.Pipeline(r.n, grid, max_journeys=max(1024, 2 * J), journey_capacity=J,
                          group_capacity=max(4096, int(1.25 * G)))
    pipe.run(rec)
    pipe.run(rec)          # second run over the same workspace, as in the timed loop
    res = pipe.results()
    assert all(x["status"] == 0 for x in res)
    print(f"[fullsize] n={r.n} J={J} G={G}", flush=True)
    yield r, grid, pipe, res, J, G
    cvetl.cv_tuning_set("sort_shape", prev)


def test_order_properties_every_record(day):
    r, grid, pipe, res, J, G = day
    perm = u32(host(pipe.perm)).astype(np.int64)
    n = r.n
    assert np.bincount(perm, minlength=n).max() == 1           # a permutation
    jid = r.journey_id[perm]
    ts = r.ts_ms[perm]
    assert np.array_equal(host(pipe.sorted["journey_id"]), jid)
    assert np.array_equal(host(pipe.sorted["ts_ms"]), ts)
    assert np.array_equal(host(pipe.sorted["lat_deg"]).view(np.uint64), r.lat_deg[perm].view(np.uint64))
    assert np.array_equal(host(pipe.sorted["speed_mps"]).view(np.uint32), r.speed_mps[perm].view(np.uint32))
    dj = np.diff(jid)
    assert np.all(dj >= 0)
    same = dj == 0
    dt = np.diff(ts)
    assert np.all(dt[same] >= 0)
    tie = same & (dt == 0)
    assert np.all(np.diff(perm)[tie] > 0)                      # stable: ties keep input order


def test_sampled_journeys(day):
    r, grid, pipe, res, J, G = day
    rng = np.random.default_rng(17)
    summ = {k: host(v[:J]) for k, v in pipe.journeys.items()}
    assert int(u32(summ["n_points"]).astype(np.int64).sum()) == r.n
    assert np.all(np.diff(summ["journey_id"]) > 0)
    feat = {k: host(v) for k, v in pipe.feat.items()}
    pick = rng.choice(J, size=150, replace=False)
    pick = np.concatenate([pick, [0, J - 1, int(np.argmax(u32(summ["n_points"])))]])
    for j in pick:
        jj = summ["journey_id"][j]
        idx = np.nonzero(r.journey_id == jj)[0]
        cols = tuple(c[idx] for c in r.columns())
        exp = oracle.run_plain(cols, grid)
        a = int(u32(summ["first"])[j])
        m = int(u32(summ["n_points"])[j])
        assert m == len(idx)
        check_features({k: _t(v[a:a + m]) for k, v in feat.items()}, exp["features"])
        es = exp["summary"]
        for k in ("journey_id", "t_start_ms", "t_end_ms", "sum_speed", "max_speed", "lat_min", "lon_max"):
            assert_exact(k, summ[k][j:j + 1], es[k])
        assert_exact("n_dt_zero", u32(summ["n_dt_zero"])[j:j + 1], es["n_dt_zero"])
        assert_rel("distance_m", summ["distance_m"][j:j + 1], es["distance_m"])
        assert_rel("max_derived_speed", summ["max_derived_speed"][j:j + 1], es["max_derived_speed"])


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a))


def test_sampled_grid_cells(day):
    r, grid, pipe, res, J, G = day
    rg = res[2]
    g = {k: host(v[:G]) for k, v in pipe.groups.items()}
    assert np.all(np.diff(g["key"]) > 0)
    assert int(u32(g["count"]).astype(np.int64).sum()) + rg["n_out_of_grid"] == r.n
    key, n_out = oracle.grid_keys(r.ts_ms, r.lat_deg, r.lon_deg, grid)
    assert n_out == rg["n_out_of_grid"]
    rng = np.random.default_rng(18)
    pick = rng.choice(G, size=300, replace=False)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    for i in pick:
        k = g["key"][i]
        lo, hi = np.searchsorted(ks, [k, k + 1])
        idx = order[lo:hi]
        assert hi > lo
        exp, eo = oracle.grid(*(c[idx] for c in r.columns()), grid)
        assert eo == 0 and len(exp["key"]) == 1 and exp["key"][0] == k
        assert u32(g["count"])[i] == exp["count"][0]
        assert u32(g["n_journeys"])[i] == exp["n_journeys"][0]
        assert_exact("sum_speed", g["sum_speed"][i:i + 1], exp["sum_speed"])
        assert_exact("min_speed", g["min_speed"][i:i + 1], exp["min_speed"])
        assert_exact("max_speed", g["max_speed"][i:i + 1], exp["max_speed"])


def test_whole_day_every_output_equals_oracle(day):
    # the oracle over the whole day (some 20 s of host time): every record's
    # order, sorted columns and kinematics, every journey row and every group row
    from _parity import check_groups, check_sort, check_summary
    r, grid, pipe, res, J, G = day
    print(f"[fullsize] oracle over all {r.n} records", flush=True)
    exp = oracle.run_plain(r.columns(), grid)
    n = r.n
    check_sort(pipe.perm[:n], {k: v[:n] for k, v in pipe.sorted.items()}, exp["perm"], exp["sorted"])
    check_features({k: v[:n] for k, v in pipe.feat.items()}, exp["features"])
    check_summary({k: v[:J] for k, v in pipe.journeys.items()}, exp["summary"])
    check_groups({k: v[:G] for k, v in pipe.groups.items()}, res[2]["n_out_of_grid"], exp["groups"], exp["n_out"])
