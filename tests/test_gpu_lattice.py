"""Dense lattice, per-channel normalisation and group filter: HIP path vs the
oracle's definitions, exactly (float32 values bit for bit, indices equal)."""
import numpy as np
import pytest

import oracle
from paper_2305_07454_amd import gen

from _parity import assert_exact, host

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


@pytest.fixture(scope="module")
def case(cv):
    """Full-day-shaped records (per-journey files) on a coarser grid over the same box (0.02 degrees, 15
    minutes, 96 bins: tensors of tens of MB): the GPU group tables (with and
    without four heading sectors) and the oracle's own group tables."""
    import torch
    r = gen.make_c1(seed=41, n_journeys=80, median=900.0, shuffled=True)
    hd = gen.headings(np.random.default_rng(41), r.journey_id)
    grid = gen.GridSpec(36.0, -95.8, 0.02, 0.02, 230, 335, gen.T0_MS, 900_000, 96)
    rec = cv.to_device(r)
    perm, srt, _ = cv.cv_sort_records(rec)
    g0, _ = cv.cv_grid_aggregate(srt, grid)
    hs = cv.cv_gather_column(torch.from_numpy(hd).cuda(), perm)
    g4, _ = cv.cv_grid_aggregate_dir(srt, grid, 4, 45.0, heading=hs)
    p = oracle.sort(r.journey_id, r.ts_ms)
    s = oracle.sorted_records(r.columns(), p)
    e0, _ = oracle.grid(*s, grid)
    e4, _ = oracle.grid_dir(*s, grid, 4, 45.0, heading=hd[p])
    return grid, {0: (g0, e0), 4: (g4, e4)}


@pytest.mark.parametrize("n_dir", [0, 4])
@pytest.mark.parametrize("t_first,n_t", [(0, 96), (30, 20), (90, 10)])
def test_dense_and_normalized_lattice(cv, case, n_dir, t_first, n_t):
    grid, tabs = case
    got_g, exp_g = tabs[n_dir]
    print(f"[lattice] n_dir={n_dir} t_first={t_first} n_t={n_t} groups={len(exp_g['key'])}", flush=True)
    lat = cv.cv_lattice_dense(got_g, grid, n_dir, t_first, n_t)
    exp = oracle.lattice_dense(exp_g, grid, n_dir, t_first, n_t)
    assert_exact("lattice", host(lat).view(np.uint32).ravel(), exp.view(np.uint32).ravel())
    norm, mm = cv.cv_lattice_normalize(lat, grid, n_dir)
    en, emm = oracle.lattice_normalize(exp)
    assert_exact("normalized", host(norm).view(np.uint32).ravel(), en.view(np.uint32).ravel())
    assert_exact("min/max", host(mm).view(np.uint32).ravel(), emm.view(np.uint32).ravel())


def test_dense_lattice_of_no_groups(cv, case):
    import torch
    grid, _ = case
    empty = {k: torch.empty(0, dtype=dt, device="cuda") for k, dt in cv.GROUP_FIELDS}
    lat = cv.cv_lattice_dense(empty, grid, 0, 0, 3)
    assert int(torch.count_nonzero(lat)) == 0
    _, mm = cv.cv_lattice_normalize(lat, grid, 0)
    assert bool(torch.isnan(mm).all())


@pytest.mark.parametrize("vmin,lo,hi", [(1, 0.0, 1e9), (2, 5.0, 20.0), (3, -1.0, 8.0), (1000, 0.0, 1e9)])
def test_groups_filter(cv, case, vmin, lo, hi):
    _, tabs = case
    for n_dir in (0, 4):
        got_g, exp_g = tabs[n_dir]
        idx, r = cv.cv_groups_filter(got_g, vmin, lo, hi)
        want = oracle.groups_filter(exp_g, vmin, lo, hi)
        assert_exact("filter", host(idx).astype(np.int64), want)
        assert r["count"] == len(want)


def test_groups_filter_capacity(cv, case):
    _, tabs = case
    got_g, exp_g = tabs[0]
    want = oracle.groups_filter(exp_g, 1, 0.0, 1e9)
    with pytest.raises(cv.CvError):
        cv.cv_groups_filter(got_g, 1, 0.0, 1e9, capacity=len(want) - 1)
