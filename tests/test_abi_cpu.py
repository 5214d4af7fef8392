"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments on the host before touching a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cvetl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cv_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2305_07454_amd import cvetl
    if not os.path.exists(cvetl.LIB_PATH):
        from paper_2305_07454_amd import build
        build.build()
    return cvetl.lib()


def test_header_symbols_exported(L):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_abi_version_and_strerror(L):
    assert L.cv_abi_version() == 1
    from paper_2305_07454_amd import cvetl
    assert cvetl.strerror(cvetl.CV_ERR_CAPACITY) == "output capacity exceeded"
    assert "unknown" in cvetl.strerror(99)


def test_workspace_queries_host_only(L):
    from paper_2305_07454_amd import cvetl, gen
    sz = ctypes.c_size_t()
    assert L.cv_sort_workspace_size(1000, 10, ctypes.byref(sz)) == 0 and sz.value > 0
    small = sz.value
    assert L.cv_sort_workspace_size(10_000_000, 10, ctypes.byref(sz)) == 0 and sz.value > small
    assert L.cv_sort_workspace_size(1 << 32, 10, ctypes.byref(sz)) == cvetl.CV_ERR_INVALID_ARGUMENT
    assert L.cv_summary_workspace_size(1000, 100, ctypes.byref(sz)) == 0
    spec = cvetl._spec_struct(gen.GRIDS["c1"])
    assert L.cv_grid_workspace_size(1000, ctypes.byref(spec), 100, ctypes.byref(sz)) == 0
    bad = cvetl._spec_struct(gen.GRIDS["c1"])
    bad.dlat_deg = 0.0
    assert L.cv_grid_workspace_size(1000, ctypes.byref(bad), 100, ctypes.byref(sz)) == cvetl.CV_ERR_INVALID_ARGUMENT
    bad = cvetl._spec_struct(gen.GRIDS["c1"])
    bad.bin_ms = 0
    assert L.cv_grid_workspace_size(1000, ctypes.byref(bad), 100, ctypes.byref(sz)) == cvetl.CV_ERR_INVALID_ARGUMENT
    bad = cvetl._spec_struct(gen.GRIDS["c1"])
    bad.n_t = 1 << 40
    bad.n_lat = 1 << 20
    assert L.cv_grid_workspace_size(1000, ctypes.byref(bad), 100, ctypes.byref(sz)) == cvetl.CV_ERR_INVALID_ARGUMENT


def test_argument_errors_before_any_launch(L):
    from paper_2305_07454_amd import cvetl
    rec = cvetl.CvRecords(None, None, None, None, None, 10)
    assert L.cv_journey_features(ctypes.byref(rec), ctypes.byref(cvetl.CvFeatures()), None) == \
        cvetl.CV_ERR_INVALID_ARGUMENT
    assert L.cv_journey_features(None, None, None) == cvetl.CV_ERR_INVALID_ARGUMENT
    # missing workspace is reported before anything is enqueued
    assert L.cv_sort_records(ctypes.byref(rec), 10, None, None, None, None, 0, None) == \
        cvetl.CV_ERR_INVALID_ARGUMENT
    big = cvetl.CvRecords(None, None, None, None, None, 1 << 32)
    assert L.cv_sort_records(ctypes.byref(big), 10, None, None, None, None, 0, None) == \
        cvetl.CV_ERR_INVALID_ARGUMENT
    ok = cvetl.CvRecords(8, 8, 8, 8, 8, 10)   # non-null dummies; fails on the workspace check first
    assert L.cv_sort_records(ctypes.byref(ok), 10, ctypes.c_void_p(8), None, None, None, 0, None) == \
        cvetl.CV_ERR_WORKSPACE
    assert L.cv_journey_summary(ctypes.byref(ok), ctypes.byref(cvetl.CvFeatures()),
                                ctypes.byref(cvetl.CvJourneys()), 10, None, None, 0, None) == \
        cvetl.CV_ERR_WORKSPACE
    # the allocation-free summary: sizes beyond its scratch array are refused on the host
    many = cvetl.CvRecords(8, 8, 8, 8, 8, 1 << 20)
    assert L.cv_journey_summary_noalloc(ctypes.byref(many), ctypes.byref(cvetl.CvFeatures()),
                                        ctypes.byref(cvetl.CvJourneys()), 1 << 20, None, None) == \
        cvetl.CV_ERR_WORKSPACE
    assert L.cv_journey_summary_noalloc(ctypes.byref(big), ctypes.byref(cvetl.CvFeatures()),
                                        ctypes.byref(cvetl.CvJourneys()), 10, None, None) == \
        cvetl.CV_ERR_INVALID_ARGUMENT
    spec = cvetl._spec_struct(__import__("paper_2305_07454_amd.gen", fromlist=["x"]).GRIDS["c0"])
    assert L.cv_grid_aggregate(ctypes.byref(ok), ctypes.byref(spec), ctypes.byref(cvetl.CvGroups()), 10, None,
                               None, 0, None) == cvetl.CV_ERR_WORKSPACE


def test_timing_registry_host_only(L):
    from paper_2305_07454_amd import cvetl
    cvetl.cv_timing_reset()
    assert cvetl.cv_timing_read("nothing") == (0.0, 0)


def test_tuning_values_checked_before_narrowing(L):
    # a 64-bit value whose low 32 bits name a valid shape is still refused
    from paper_2305_07454_amd import cvetl
    prev = ctypes.c_int64()
    assert L.cv_tuning_get(b"sort_shape", ctypes.byref(prev)) == 0
    for v in (1 << 32, (1 << 32) + 1, -(1 << 63), -1):
        assert L.cv_tuning_set(b"sort_shape", ctypes.c_int64(v)) == cvetl.CV_ERR_INVALID_ARGUMENT
    got = ctypes.c_int64()
    assert L.cv_tuning_get(b"sort_shape", ctypes.byref(got)) == 0 and got.value == prev.value
    assert L.cv_tuning_set(b"grid_lds_slots", ctypes.c_int64(256)) == cvetl.CV_ERR_INVALID_ARGUMENT


def test_wide_first_digit_knob(L):
    # host-only: the knob takes 0 or 1 and reads back; other values are refused
    from paper_2305_07454_amd import cvetl
    prev = ctypes.c_int64()
    assert L.cv_tuning_get(b"radix_wide_first", ctypes.byref(prev)) == 0 and prev.value in (0, 1)
    try:
        for v in (0, 1):
            got = ctypes.c_int64()
            assert L.cv_tuning_set(b"radix_wide_first", ctypes.c_int64(v)) == 0
            assert L.cv_tuning_get(b"radix_wide_first", ctypes.byref(got)) == 0 and got.value == v
        for v in (2, -1, 1 << 32):
            assert L.cv_tuning_set(b"radix_wide_first", ctypes.c_int64(v)) == cvetl.CV_ERR_INVALID_ARGUMENT
        blk = ctypes.c_int64()
        assert L.cv_tuning_get(b"sort_block", ctypes.byref(blk)) == 0 and blk.value in (256, 512, 1024)
        assert L.cv_tuning_set(b"sort_block", ctypes.c_int64(512)) == cvetl.CV_ERR_INVALID_ARGUMENT
    finally:
        L.cv_tuning_set(b"radix_wide_first", prev)


def test_debug_entry_points_only_in_the_checking_build(L):
    from paper_2305_07454_amd import cvetl
    flags = ctypes.c_uint32(7)
    assert L.cv_debug_flags(ctypes.byref(flags), 0) == cvetl.CV_ERR_UNSUPPORTED
    assert L.cv_debug_check_ascending(None, 10, None) == cvetl.CV_ERR_UNSUPPORTED
    # the checking build exports every declared symbol as well
    if os.path.exists(cvetl.DEBUG_LIB_PATH):
        D = ctypes.CDLL(cvetl.DEBUG_LIB_PATH)
        for name in _declared():
            assert hasattr(D, name), name
        assert D.cv_debug_check_ascending(None, 10, None) == cvetl.CV_ERR_INVALID_ARGUMENT
