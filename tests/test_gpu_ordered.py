"""Input whose timestamps never decrease within a shard (a time-ordered feed):
the sort key keeps only the (shard, journey rank) bits, because a stable sort
by journey alone already leaves each journey's records in time order.  One
decrease anywhere inside a shard brings the time bits back.  Every case is
compared with the oracle, element by element, and the key width says which
key was used."""
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


def _bits(x):
    return int(x).bit_length()


def _feed(seed, n, n_ids, step_ms=1000):
    """Records in time order with interleaved journey ids and many equal
    timestamps (ties across and within journeys)."""
    rng = np.random.default_rng(seed)
    ids = np.unique(rng.integers(-2 ** 62, 2 ** 62, n_ids, dtype=np.int64))
    jid = ids[rng.integers(0, len(ids), n)]
    k = min(len(ids), n)
    jid[:k] = ids[:k]
    rng.shuffle(jid)
    ts = gen.T0_MS + step_ms * np.sort(rng.integers(0, max(1, n // 3), n)).astype(np.int64)
    lat = 38.0 + np.cumsum(rng.normal(0, 2e-3, n))
    lon = -92.0 + np.cumsum(rng.normal(0, 2e-3, n))
    spd = rng.uniform(0, 40, n).astype(np.float32)
    return [jid, ts, lat, lon, spd]


def _run_both(cv, cols, spec):
    print(f"[ordered] n={len(cols[0])}", flush=True)
    exp = oracle.run_plain(tuple(cols), spec)
    got = cv.run_plain(cv.to_device(tuple(cols)), spec)
    check_sort(got["perm"], got["sorted"], exp["perm"], exp["sorted"])
    check_features(got["features"], exp["features"])
    check_summary(got["summary"], exp["summary"])
    check_groups(got["groups"], got["n_out"], exp["groups"], exp["n_out"])
    return got


@pytest.mark.parametrize("n", [20_000, 1_500_000])
def test_time_ordered_input_sorts_by_journey_alone(cv, n):
    cols = _feed(41 + n, n, 300)
    got = _run_both(cv, cols, gen.GRIDS["c1"])
    J = len(np.unique(cols[0]))
    assert got["sort_result"]["key_bits"] == _bits(J - 1)
    assert got["sort_result"]["packed_pass"] == 0


@pytest.mark.parametrize("where", [1, 63, 64, 65, 511, 512, 4095, 4096, 100_001, -1])
def test_one_decrease_keeps_the_time_bits(cv, where):
    n = 1_500_000 if where == 100_001 else 20_000
    cols = _feed(7, n, 300)
    p = where % n
    cols[1][p] = cols[1][p - 1] - 1  # the only place where time goes back
    got = _run_both(cv, cols, gen.GRIDS["c1"])
    J = len(np.unique(cols[0]))
    # the decrease by 1 ms leaves the offsets no common factor above 1
    tspan = int(cols[1].max() - cols[1].min())
    assert got["sort_result"]["key_bits"] == _bits(J - 1) + _bits(tspan)


def _batched(cv, shards, grid):
    sizes = [len(s[0]) for s in shards]
    allc = tuple(np.concatenate([s[i] for s in shards]) for i in range(5))
    print(f"[ordered batched] shards={len(shards)} n={len(allc[0])}", flush=True)
    bp, res = cv.cv_batch_run(cv.to_device(allc), sizes, grid)
    jo, go, sout = host(bp.journey_offsets), host(bp.group_offsets), host(bp.shard_n_out)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for s, sh in enumerate(shards):
        a, b = int(off[s]), int(off[s + 1])
        exp = oracle.run_plain(tuple(sh), grid)
        check_sort(bp.perm[a:b], {k: v[a:b] for k, v in bp.sorted.items()}, exp["perm"], exp["sorted"])
        check_features({k: v[a:b] for k, v in bp.feat.items()}, exp["features"])
        check_summary({k: v[int(jo[s]):int(jo[s + 1])] for k, v in bp.journeys.items()}, exp["summary"])
        check_groups({k: v[int(go[s]):int(go[s + 1])] for k, v in bp.groups.items()}, int(sout[s]),
                     exp["groups"], exp["n_out"])
    J = len(np.unique(allc[0]))
    # an id in two shards keeps the shard above the rank in the key; otherwise
    # the ranks follow (shard, id) order and keep the shards apart themselves
    seen = {}
    for s, sh in enumerate(shards):
        for x in np.unique(sh[0]):
            seen.setdefault(int(x), set()).add(s)
    multi = any(len(v) > 1 for v in seen.values())
    _batched.last_result = res[0]
    return res[0]["key_bits"], J, len(shards), multi


def test_batched_shards_each_in_time_order(cv):
    # every shard is time-ordered, and each later shard starts earlier in time
    # than the one before it ends: the shard starts are not decreases
    shards = [_feed(100 + i, m, 40) for i, m in enumerate([3000, 1, 70_000, 5000, 64, 40_000])]
    kb, J, S, multi = _batched(cv, shards, gen.GRIDS["c2"])
    assert not multi and kb == _bits(J - 1)


def test_batched_decrease_inside_one_shard(cv):
    shards = [_feed(200 + i, m, 40) for i, m in enumerate([3000, 70_000, 5000])]
    shards[1][1][777] = shards[1][1][776] - 1
    kb, J, S, multi = _batched(cv, shards, gen.GRIDS["c2"])
    t = np.concatenate([s[1] for s in shards])
    assert not multi and kb == _bits(J - 1) + _bits(int(t.max() - t.min()))


@pytest.mark.parametrize("where", ["boundary", "distant", "same_window"])
def test_batched_id_in_two_shards(cv, where):
    # one journey id met in two shards: as the last record of one shard and
    # the first of the next (a run of equal ids across the shard start), in
    # shards far apart, or in two shards that start inside one window of 64
    # records; the key then carries the shard above the rank
    sizes = [3000, 70_000, 5000, 20, 40_000] if where != "same_window" else [3000, 10, 30, 5000]
    shards = [_feed(300 + i, m, 40) for i, m in enumerate(sizes)]
    x = int(shards[0][0][0])
    if where == "boundary":
        shards[0][0][-1] = x
        shards[1][0][0] = x
    elif where == "distant":
        shards[4][0][777] = x
    else:
        shards[2][0][5] = x  # shards 1 and 2 start within 40 records of each other
    kb, J, S, multi = _batched(cv, shards, gen.GRIDS["c2"])
    assert multi and kb == _bits(S - 1) + _bits(J - 1)


def test_batched_ids_repeat_across_many_shard_starts(cv):
    # 40 shards whose ids are all distinct, many shard starts in one wave's
    # range (tiny shards), each time-ordered: ranks in (shard, id) order
    sizes = [1 + (i * 37) % 300 for i in range(40)]
    shards = [_feed(500 + i, m, 3) for i, m in enumerate(sizes)]
    kb, J, S, multi = _batched(cv, shards, gen.GRIDS["c2"])
    assert not multi and kb == _bits(J - 1)


def test_batched_rank_key_with_a_wide_first_digit(cv):
    # time-ordered shards with some 80 000 journeys: a 17-bit rank key, which
    # takes a 9-bit first digit and two passes (the key packing then counts
    # its first digit per record instead of from the tile's multisplit)
    shards = [_feed(900 + i, 150_000, 10_000) for i in range(8)]
    kb, J, S, multi = _batched(cv, shards, gen.GRIDS["c2"])
    assert not multi and kb == _bits(J - 1) == 17
    wide = cv.cv_tuning_get("radix_wide_first") and cv.cv_tuning_get("sort_block") >= 512
    assert _batched.last_result["flags"] == (9 if wide else 8)
