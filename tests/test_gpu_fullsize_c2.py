"""Full-size parity on the batched workload (115 county-day shards of capped
Zipf sizes, 400 M records, 0.001 deg x 1 min), in the launch configuration the
benchmark times (BatchPipeline sized by a first run, tuned as the benchmark
tunes it): the two largest shards, the smallest and five seeded random ones are
recomputed by the oracle on their own records and compared element by element
in every output column (order, sorted columns, kinematics, journey rows, group
rows, per-shard out-of-grid counts).  Every shard's journey and group counts
and record totals are checked as invariants."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import check_features, check_groups, check_sort, check_summary, host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl, tune
    oracle.lib()
    print("[fullsize c2] generating the batched workload", flush=True)
    shards = gen.make_c2()
    sizes = [s.n for s in shards]
    allr = gen.concat(shards)
    n = allr.n
    grid = gen.GRIDS["c2"]
    prev = cvetl.cv_tuning_get("sort_shape")
    tune.apply(n, workload="c2")
    dev = torch.device("cuda:0")
    rec = cvetl.to_device(allr, dev)
    del allr
    off_h, off_d = cvetl.shard_offsets(sizes, dev)
    bp0, res0 = cvetl.cv_batch_run(rec, sizes, grid)
    J, G, mj = res0[1]["count"], res0[2]["count"], bp0.max_journeys
    del bp0
    torch.cuda.empty_cache()
    bp = cvetl.BatchPipeline(n, len(sizes), grid, mj, J, max(4096, int(1.25 * G)), dev)
    bp.run(rec, off_d)
    bp.run(rec, off_d)  # a second run over the same workspace, as in the timed loop
    torch.cuda.synchronize()
    res = bp.results()
    assert all(x["status"] == 0 for x in res), res
    print(f"[fullsize c2] n={n} J={J} G={G} shards={len(sizes)}", flush=True)
    yield shards, sizes, grid, bp, res
    cvetl.cv_tuning_set("sort_shape", prev)


def test_every_shard_invariants(batch):
    shards, sizes, grid, bp, res = batch
    jo = host(bp.journey_offsets).astype(np.int64)
    go = host(bp.group_offsets).astype(np.int64)
    sout = host(bp.shard_n_out).astype(np.int64)
    assert jo[0] == 0 and go[0] == 0 and jo[-1] == res[1]["count"] and go[-1] == res[2]["count"]
    npts = u32(host(bp.journeys["n_points"][:jo[-1]])).astype(np.int64)
    cnt = u32(host(bp.groups["count"][:go[-1]])).astype(np.int64)
    for s, m in enumerate(sizes):
        assert npts[jo[s]:jo[s + 1]].sum() == m
        assert cnt[go[s]:go[s + 1]].sum() + sout[s] == m
        assert jo[s + 1] - jo[s] == shards[s].meta["n_journeys"]
    assert sout.sum() == res[2]["n_out_of_grid"]


def _pick(sizes):
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[-1]), int(order[-2]), int(order[0])]
    rng = np.random.default_rng(2305)
    rest = [i for i in range(len(sizes)) if i not in pick]
    return pick + [int(x) for x in rng.choice(rest, size=5, replace=False)]


@pytest.mark.parametrize("k", range(8))
def test_shard_equals_oracle(batch, k):
    shards, sizes, grid, bp, res = batch
    s = _pick(sizes)[k]
    off = np.concatenate([[0], np.cumsum(sizes)])
    a, b = int(off[s]), int(off[s + 1])
    jo = host(bp.journey_offsets).astype(np.int64)
    go = host(bp.group_offsets).astype(np.int64)
    print(f"[fullsize c2] shard {s}: {sizes[s]} records", flush=True)
    exp = oracle.run_plain(shards[s].columns(), grid)
    check_sort(bp.perm[a:b], {c: v[a:b] for c, v in bp.sorted.items()}, exp["perm"], exp["sorted"])
    check_features({c: v[a:b] for c, v in bp.feat.items()}, exp["features"])
    check_summary({c: v[jo[s]:jo[s + 1]] for c, v in bp.journeys.items()}, exp["summary"])
    check_groups({c: v[go[s]:go[s + 1]] for c, v in bp.groups.items()}, int(host(bp.shard_n_out)[s]),
                 exp["groups"], exp["n_out"])
