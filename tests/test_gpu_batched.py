"""Batched form: many uneven shards in one set of launches; every shard must
equal the plain path (and the oracle) applied to it alone."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import check_features, check_groups, check_sort, check_summary, host, u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    cvetl.lib()
    return cvetl


def _shards(seed, n_shards, total, lo, hi):
    shards = gen.make_c2(seed=seed, n_shards=n_shards, total=total, lo=lo, hi=hi)
    return [s for s in shards]


def _check_batch(cv, shards, grid):
    import torch
    sizes = [s.n for s in shards]
    allr = gen.concat(shards)
    print(f"[batched] shards={len(shards)} n={allr.n} sizes={sizes[:8]}...", flush=True)
    rec = cv.to_device(allr)
    bp, res = cv.cv_batch_run(rec, sizes, grid)
    jo = host(bp.journey_offsets)
    go = host(bp.group_offsets)
    sout = host(bp.shard_n_out)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for s, sh in enumerate(shards):
        a, b = int(off[s]), int(off[s + 1])
        exp = oracle.run_plain(sh.columns(), grid)
        perm = {"x": bp.perm[a:b]}["x"]
        srt = {k: v[a:b] for k, v in bp.sorted.items()}
        check_sort(perm, srt, exp["perm"], exp["sorted"])
        check_features({k: v[a:b] for k, v in bp.feat.items()}, exp["features"])
        check_summary({k: v[int(jo[s]):int(jo[s + 1])] for k, v in bp.journeys.items()}, exp["summary"])
        gs = {k: v[int(go[s]):int(go[s + 1])] for k, v in bp.groups.items()}
        check_groups(gs, int(sout[s]) if len(shards) else 0, exp["groups"], exp["n_out"])
    n_out = sum(oracle.run_plain(sh.columns(), grid)["n_out"] for sh in shards) if len(shards) < 4 else None
    if n_out is not None:
        assert res[2]["n_out_of_grid"] == n_out
    torch.cuda.synchronize()


def test_batched_uneven_shards(cv):
    shards = _shards(31, 12, 300_000, 500, 120_000)
    # records outside the grid in some shards (outside the box, non-finite): counted per shard
    for i in (1, 4, 7):
        sh = shards[i]
        sh.lat_deg[::53] = 35.5
        sh.lon_deg[7::211] = np.nan
    _check_batch(cv, shards, gen.GRIDS["c2"])


def test_batched_empty_shards_and_shared_ids(cv):
    base = _shards(32, 5, 60_000, 2_000, 30_000)
    # one journey id X ends shard 1 and starts shard 2 after the sort (adjacent
    # records, same id): it must still be two journeys
    a, b = base[1], base[2]
    X = np.int64(2 ** 62)
    amax, bmin = a.journey_id.max(), b.journey_id.min()
    a.journey_id[:] = np.where(a.journey_id == amax, X, a.journey_id % (2 ** 61))
    b.journey_id[:] = np.where(b.journey_id == bmin, X, X + 1 + b.journey_id % (2 ** 61))
    empty = gen.Records(*(c[:0] for c in base[0].columns()))
    shards = [empty, base[0], base[1], empty, empty, base[2], base[3], base[4], empty]
    _check_batch(cv, shards, gen.GRIDS["c1"])


def test_batched_single_shard_equals_plain(cv):
    r = gen.make_c1(seed=5, n_journeys=40, median=500.0)
    _check_batch(cv, [r], gen.GRIDS["c1"])
