"""The allocation-free journey summary (library-owned per-GPU scratch) against
the workspace entry point, through the C ABI: every output column bit for bit
on two calls in a row, the second on a smaller input, and the host-side
rejection of sizes beyond the scratch array."""
import ctypes

import numpy as np
import pytest

from paper_2305_07454_amd import gen

from _parity import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_07454_amd import cvetl
    cvetl.lib()
    return cvetl


def _sorted_and_features(cv, r):
    rec = cv.to_device(r.columns())
    _, srt, _ = cv.cv_sort_records(rec)
    feat = cv.cv_journey_features(srt)
    return srt, feat


def _compare(cv, srt, feat, cap):
    import torch
    want, rw = cv.cv_journey_summary(srt, feat, capacity=cap)
    # outputs start as 0xFF bytes so that an unwritten row cannot pass as zeros
    out = {k: torch.full((cap,), -1, dtype=dt, device="cuda") if dt != torch.float32 and dt != torch.float64
           else torch.full((cap,), float("nan"), dtype=dt, device="cuda") for k, dt in cv.JOURNEY_FIELDS}
    res = cv.cv_journey_summary_noalloc(srt, feat, out, capacity=cap)
    torch.cuda.synchronize()
    r = cv.read_result(res)
    assert r["status"] == 0 and r["count"] == rw["count"], (r, rw)
    J = r["count"]
    for k, _ in cv.JOURNEY_FIELDS:
        a, b = host(out[k][:J]), host(want[k])
        assert a.dtype == b.dtype and a.shape == b.shape, k
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"column {k} differs"
    return J


def test_noalloc_summary_matches_workspace_entry_twice(cv):
    big = gen.make_c1(seed=4242, n_journeys=300, median=900.0)
    small = gen.make_c1(seed=4243, n_journeys=37, median=400.0)
    assert small.n < big.n
    print(f"[noalloc] first call n={big.n}, second n={small.n}", flush=True)
    srt, feat = _sorted_and_features(cv, big)
    j1 = _compare(cv, srt, feat, cap=400)
    srt2, feat2 = _sorted_and_features(cv, small)
    j2 = _compare(cv, srt2, feat2, cap=64)
    assert j1 == 300 and j2 == 37


def test_noalloc_summary_rejects_sizes_beyond_the_scratch(cv):
    L = cv.lib()
    n = 1 << 20
    need = ctypes.c_size_t()
    assert L.cv_summary_workspace_size(n, 1 << 20, ctypes.byref(need)) == 0
    assert need.value > 32 << 20
    rec = cv.CvRecords()
    rec.n = n  # null columns: the size check comes first and nothing is enqueued
    js = cv.CvJourneys()
    fs = cv.CvFeatures()
    st = L.cv_journey_summary_noalloc(ctypes.byref(rec), ctypes.byref(fs), ctypes.byref(js), 1 << 20, None, None)
    assert st == cv.CV_ERR_WORKSPACE
