"""The checking build (libcvetl_debug.so, CVETL_DEBUG): its checker kernels
find nothing on correct runs of the plain, batched and ordered paths (whose
outputs still equal the oracle's), and the checker itself flags a planted
disorder in a caller's array."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import check_features, check_groups, check_sort, check_summary, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dbg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    oracle.lib()
    prev = cvetl.use_library("debug")
    _flags(cvetl, reset=True)
    yield cvetl
    cvetl.use_library(prev)


def _flags(cv, reset=True):
    import ctypes
    f = ctypes.c_uint32(0)
    assert cv.lib().cv_debug_flags(ctypes.byref(f), 1 if reset else 0) == 0
    return f.value


def test_checks_pass_on_the_plain_path(dbg):
    cv = dbg
    r = gen.make_c0(seed=91, n_journeys=300)
    print(f"[debug] plain n={r.n}", flush=True)
    exp = oracle.run_plain(r.columns(), gen.GRIDS["c0"])
    got = cv.run_plain(cv.to_device(r), gen.GRIDS["c0"])
    check_sort(got["perm"], got["sorted"], exp["perm"], exp["sorted"])
    check_features(got["features"], exp["features"])
    check_summary(got["summary"], exp["summary"])
    check_groups(got["groups"], got["n_out"], exp["groups"], exp["n_out"])
    assert _flags(cv) == 0


def test_checks_pass_on_batched_shards(dbg):
    cv = dbg
    shards = [gen.make_c1(seed=70 + i, n_journeys=m, median=400.0) for i, m in enumerate([5, 1, 30, 12])]
    sizes = [s.n for s in shards]
    allc = tuple(np.concatenate([s.columns()[i] for s in shards]) for i in range(5))
    print(f"[debug] batched shards={len(sizes)} n={sum(sizes)}", flush=True)
    bp, res = cv.cv_batch_run(cv.to_device(allc), sizes, gen.GRIDS["c2"])
    jo, go, sout = host(bp.journey_offsets), host(bp.group_offsets), host(bp.shard_n_out)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for s, sh in enumerate(shards):
        a, b = int(off[s]), int(off[s + 1])
        exp = oracle.run_plain(sh.columns(), gen.GRIDS["c2"])
        check_sort(bp.perm[a:b], {k: v[a:b] for k, v in bp.sorted.items()}, exp["perm"], exp["sorted"])
        check_summary({k: v[int(jo[s]):int(jo[s + 1])] for k, v in bp.journeys.items()}, exp["summary"])
        check_groups({k: v[int(go[s]):int(go[s + 1])] for k, v in bp.groups.items()}, int(sout[s]),
                     exp["groups"], exp["n_out"])
    assert _flags(cv) == 0


def test_checker_flags_a_planted_disorder(dbg):
    import torch
    cv = dbg
    a = torch.tensor([1, 2, 3, 5, 4, 9], dtype=torch.int64, device="cuda")
    b = torch.arange(1000, dtype=torch.int64, device="cuda")
    L = cv.lib()
    assert L.cv_debug_check_ascending(b.data_ptr(), b.numel(), None) == 0
    assert _flags(cv) == 0
    assert L.cv_debug_check_ascending(a.data_ptr(), a.numel(), None) == 0
    f = _flags(cv, reset=True)
    assert f & cv.CV_DEBUG_CHECK
    assert _flags(cv) == 0
