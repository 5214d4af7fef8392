"""Thin ctypes binding of ``libcvetl.so`` (the gfx950 HIP library).

Argument marshalling only: every step of the ETL path runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  The functions carry the C-ABI names:

* ``cv_sort_records(records, ...)      -> (perm, sorted_records, result)``
* ``cv_journey_features(sorted)        -> features``
* ``cv_journey_summary(sorted, feat)   -> (journeys, result)``
* ``cv_grid_aggregate(sorted, grid)    -> (groups, result)``
* ``cv_sort_records_features(records, max_journeys, shard_offsets=None)
  -> (perm, sorted_records, features, result)``: the sort and the kinematics
  in one call (the preallocated ``Pipeline`` / ``BatchPipeline`` use it)

A record batch is a dict of device tensors with the keys of ``RECORD_FIELDS``.
There is no CPU fallback: loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcvetl.so")

RECORD_FIELDS = (("journey_id", torch.int64), ("ts_ms", torch.int64), ("lat_deg", torch.float64),
                 ("lon_deg", torch.float64), ("speed_mps", torch.float32))
FEATURE_FIELDS = (("step_m", torch.float64), ("dt_s", torch.float64), ("speed_mps", torch.float64),
                  ("accel_mps2", torch.float64), ("bearing_deg", torch.float64),
                  ("dheading_deg", torch.float64), ("flags", torch.uint8))
JOURNEY_FIELDS = (("journey_id", torch.int64), ("first", torch.int32), ("n_points", torch.int32),
                  ("t_start_ms", torch.int64), ("t_end_ms", torch.int64), ("distance_m", torch.float64),
                  ("sum_speed", torch.float64), ("max_speed", torch.float32),
                  ("max_derived_speed", torch.float64), ("n_dt_zero", torch.int32),
                  ("lat_min", torch.float64), ("lat_max", torch.float64), ("lon_min", torch.float64),
                  ("lon_max", torch.float64))
GROUP_FIELDS = (("key", torch.int64), ("count", torch.int32), ("n_journeys", torch.int32),
                ("sum_speed", torch.float64), ("min_speed", torch.float32), ("max_speed", torch.float32))

CV_OK, CV_ERR_INVALID_ARGUMENT, CV_ERR_WORKSPACE, CV_ERR_CAPACITY = 0, 1, 2, 3
CV_ERR_RANGE, CV_ERR_DEVICE, CV_ERR_UNSUPPORTED = 4, 5, 6
CV_DEBUG_SORT_ORDER, CV_DEBUG_PERM_RANGE, CV_DEBUG_JOURNEY_ORDER, CV_DEBUG_GROUP_ORDER, CV_DEBUG_CHECK = 1, 2, 4, 8, 16

FLAG_FIRST, FLAG_DT_ZERO, FLAG_SPEED_OK, FLAG_ACCEL_OK = 0x01, 0x02, 0x04, 0x08
FLAG_BEARING_OK, FLAG_DHEAD_OK, FLAG_BAD_COORD = 0x10, 0x20, 0x40

P = ctypes.c_void_p


class CvRecords(ctypes.Structure):
    _fields_ = [("journey_id", P), ("ts_ms", P), ("lat_deg", P), ("lon_deg", P), ("speed_mps", P),
                ("n", ctypes.c_uint64)]


class CvRecordsOut(ctypes.Structure):
    _fields_ = [("journey_id", P), ("ts_ms", P), ("lat_deg", P), ("lon_deg", P), ("speed_mps", P)]


class CvFeatures(ctypes.Structure):
    _fields_ = [(k, P) for k, _ in FEATURE_FIELDS]


class CvJourneys(ctypes.Structure):
    _fields_ = [(k, P) for k, _ in JOURNEY_FIELDS]


class CvGridSpec(ctypes.Structure):
    _fields_ = [("lat0_deg", ctypes.c_double), ("lon0_deg", ctypes.c_double), ("dlat_deg", ctypes.c_double),
                ("dlon_deg", ctypes.c_double), ("n_lat", ctypes.c_int64), ("n_lon", ctypes.c_int64),
                ("t0_ms", ctypes.c_int64), ("bin_ms", ctypes.c_int64), ("n_t", ctypes.c_int64)]


class CvGroups(ctypes.Structure):
    _fields_ = [(k, P) for k, _ in GROUP_FIELDS]


RESULT_DTYPE = np.dtype([("status", "<u4"), ("flags", "<u4"), ("count", "<u8"), ("required", "<u8"),
                         ("n_out_of_grid", "<u8"), ("n_late", "<u8"), ("key_bits", "<u8"),
                         ("packed_pass", "<u8"), ("n_bad", "<u8")])
assert RESULT_DTYPE.itemsize == 64


class CvError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = int(status)
        super().__init__(f"{where}: {strerror(status)} (status {status})")


DEBUG_LIB_PATH = os.path.join(PKG, "libcvetl_debug.so")
_libs = {}
_active = "release"


def lib():
    """The active library (libcvetl.so unless use_library("debug") chose the
    checking build); raises if it has not been built (no fallback path)."""
    return _load(_active)


def use_library(kind: str) -> str:
    """Make "release" (libcvetl.so) or "debug" (libcvetl_debug.so, built with
    CVETL_DEBUG: checker kernels after each stage, see cv_debug_flags) the
    library every call of this module goes through; returns the previous one."""
    global _active
    if kind not in ("release", "debug"):
        raise ValueError(kind)
    _load(kind)
    prev, _active = _active, kind
    return prev


def _load(kind):
    if kind not in _libs:
        path = LIB_PATH if kind == "release" else DEBUG_LIB_PATH
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2305_07454_amd/build.py "
                              "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        _libs[kind] = _declare(ctypes.CDLL(path))
    return _libs[kind]


def _declare(L):
    """Argument and result types of every exported call."""
    S = ctypes.c_int
    U64 = ctypes.c_uint64
    SZ = ctypes.POINTER(ctypes.c_size_t)
    L.cv_abi_version.restype = ctypes.c_uint32
    L.cv_strerror.argtypes = [S]
    L.cv_strerror.restype = ctypes.c_char_p
    L.cv_sort_workspace_size.argtypes = [U64, U64, SZ]
    L.cv_sort_workspace_size.restype = S
    L.cv_sort_records.argtypes = [ctypes.POINTER(CvRecords), U64, P, ctypes.POINTER(CvRecordsOut), P, P,
                                  ctypes.c_size_t, P]
    L.cv_sort_records.restype = S
    L.cv_sort_records_features.argtypes = [ctypes.POINTER(CvRecords), U64, P, ctypes.POINTER(CvRecordsOut),
                                           ctypes.POINTER(CvFeatures), P, P, ctypes.c_size_t, P]
    L.cv_sort_records_features.restype = S
    L.cv_journey_features.argtypes = [ctypes.POINTER(CvRecords), ctypes.POINTER(CvFeatures), P]
    L.cv_journey_features.restype = S
    L.cv_summary_workspace_size.argtypes = [U64, U64, SZ]
    L.cv_summary_workspace_size.restype = S
    L.cv_journey_summary.argtypes = [ctypes.POINTER(CvRecords), ctypes.POINTER(CvFeatures),
                                     ctypes.POINTER(CvJourneys), U64, P, P, ctypes.c_size_t, P]
    L.cv_journey_summary.restype = S
    L.cv_journey_summary_noalloc.argtypes = [ctypes.POINTER(CvRecords), ctypes.POINTER(CvFeatures),
                                             ctypes.POINTER(CvJourneys), U64, P, P]
    L.cv_journey_summary_noalloc.restype = S
    L.cv_grid_workspace_size.argtypes = [U64, ctypes.POINTER(CvGridSpec), U64, SZ]
    L.cv_grid_workspace_size.restype = S
    L.cv_grid_aggregate.argtypes = [ctypes.POINTER(CvRecords), ctypes.POINTER(CvGridSpec),
                                    ctypes.POINTER(CvGroups), U64, P, P, ctypes.c_size_t, P]
    L.cv_grid_aggregate.restype = S
    L.cv_grid_aggregate_flags.argtypes = [ctypes.POINTER(CvRecords), P, ctypes.POINTER(CvGridSpec),
                                          ctypes.POINTER(CvGroups), U64, P, P, ctypes.c_size_t, P]
    L.cv_grid_aggregate_flags.restype = S
    U32 = ctypes.c_uint32
    L.cv_batch_sort_records.argtypes = [ctypes.POINTER(CvRecords), P, U32, U64, P, ctypes.POINTER(CvRecordsOut),
                                        P, P, ctypes.c_size_t, P]
    L.cv_batch_sort_records.restype = S
    L.cv_batch_sort_records_features.argtypes = [ctypes.POINTER(CvRecords), P, U32, U64, P,
                                                 ctypes.POINTER(CvRecordsOut), ctypes.POINTER(CvFeatures), P, P,
                                                 ctypes.c_size_t, P]
    L.cv_batch_sort_records_features.restype = S
    L.cv_batch_journey_features.argtypes = [ctypes.POINTER(CvRecords), P, U32, ctypes.POINTER(CvFeatures), P]
    L.cv_batch_journey_features.restype = S
    L.cv_batch_journey_summary.argtypes = [ctypes.POINTER(CvRecords), ctypes.POINTER(CvFeatures), P, U32,
                                           ctypes.POINTER(CvJourneys), U64, P, P, P, ctypes.c_size_t, P]
    L.cv_batch_journey_summary.restype = S
    L.cv_batch_grid_aggregate.argtypes = [ctypes.POINTER(CvRecords), P, U32, ctypes.POINTER(CvGridSpec),
                                          ctypes.POINTER(CvGroups), U64, P, P, P, ctypes.c_size_t, P]
    L.cv_batch_grid_aggregate.restype = S
    L.cv_stream_state_size.argtypes = [ctypes.POINTER(CvGridSpec), U64, U64, U64, SZ]
    L.cv_stream_state_size.restype = S
    L.cv_stream_create.argtypes = [ctypes.POINTER(CvGridSpec), U64, U64, U64, P, ctypes.c_size_t, P,
                                   ctypes.POINTER(ctypes.c_void_p)]
    L.cv_stream_create.restype = S
    L.cv_stream_push.argtypes = [P, ctypes.POINTER(CvRecords), ctypes.POINTER(CvFeatures), P, P]
    L.cv_stream_push.restype = S
    L.cv_stream_flush.argtypes = [P, ctypes.POINTER(CvJourneys), U64, ctypes.POINTER(CvGroups), U64, P, P]
    L.cv_stream_flush.restype = S
    L.cv_stream_destroy.argtypes = [P]
    L.cv_stream_destroy.restype = S
    L.cv_batch_workspace_size.argtypes = [U64, ctypes.c_uint32, U64, U64, ctypes.POINTER(CvGridSpec), U64, SZ]
    L.cv_batch_workspace_size.restype = S
    L.cv_batch_run.argtypes = [ctypes.POINTER(CvRecords), P, ctypes.c_uint32, ctypes.POINTER(CvGridSpec), U64, P,
                               ctypes.POINTER(CvRecordsOut), ctypes.POINTER(CvFeatures), ctypes.POINTER(CvJourneys),
                               U64, P, ctypes.POINTER(CvGroups), U64, P, P, P, P, ctypes.c_size_t, P]
    L.cv_batch_run.restype = S
    L.cv_stream_snapshot_size.argtypes = [P, SZ]
    L.cv_stream_snapshot_size.restype = S
    L.cv_stream_snapshot.argtypes = [P, P, ctypes.c_size_t, P]
    L.cv_stream_snapshot.restype = S
    L.cv_stream_restore.argtypes = [P, P, ctypes.c_size_t, P]
    L.cv_stream_restore.restype = S
    L.cv_grid_aggregate_dir.argtypes = [ctypes.POINTER(CvRecords), P, ctypes.POINTER(CvFeatures),
                                        ctypes.POINTER(CvGridSpec), U32, ctypes.c_double,
                                        ctypes.POINTER(CvGroups), U64, P, P, ctypes.c_size_t, P]
    L.cv_grid_aggregate_dir.restype = S
    L.cv_gather_column.argtypes = [P, P, P, U64, U32, P]
    L.cv_gather_column.restype = S
    L.cv_lattice_dense.argtypes = [ctypes.POINTER(CvGroups), U64, ctypes.POINTER(CvGridSpec), U32,
                                   ctypes.c_int64, U64, P, P]
    L.cv_lattice_dense.restype = S
    L.cv_lattice_normalize_workspace_size.argtypes = [U64, ctypes.POINTER(CvGridSpec), U32, SZ]
    L.cv_lattice_normalize_workspace_size.restype = S
    L.cv_lattice_normalize.argtypes = [P, U64, ctypes.POINTER(CvGridSpec), U32, P, P, ctypes.c_size_t, P]
    L.cv_lattice_normalize.restype = S
    L.cv_groups_filter_workspace_size.argtypes = [U64, SZ]
    L.cv_groups_filter_workspace_size.restype = S
    L.cv_groups_filter.argtypes = [ctypes.POINTER(CvGroups), U64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, P, U64, P, P, ctypes.c_size_t, P]
    L.cv_groups_filter.restype = S
    L.cv_hygiene_workspace_size.argtypes = [U64, SZ]
    L.cv_hygiene_workspace_size.restype = S
    L.cv_drop_duplicates.argtypes = [ctypes.POINTER(CvRecords), P, ctypes.POINTER(CvRecordsOut), P, P, P,
                                     ctypes.c_size_t, P]
    L.cv_drop_duplicates.restype = S
    L.cv_split_trips.argtypes = [ctypes.POINTER(CvRecords), ctypes.c_int64, P, P, U64, P, P, ctypes.c_size_t, P]
    L.cv_split_trips.restype = S
    L.cv_csv_workspace_size.argtypes = [U64, U64, SZ]
    L.cv_csv_workspace_size.restype = S
    L.cv_csv_extract.argtypes = [P, U64, ctypes.c_int32, ctypes.POINTER(CvRecordsOut), P, P, U64, P, P,
                                 ctypes.c_size_t, P]
    L.cv_csv_extract.restype = S
    L.cv_tuning_set.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    L.cv_tuning_set.restype = S
    L.cv_tuning_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    L.cv_tuning_get.restype = S
    L.cv_timing_enable.argtypes = [S]
    L.cv_timing_enable.restype = S
    L.cv_timing_reset.restype = S
    L.cv_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U64)]
    L.cv_timing_read.restype = S
    L.cv_debug_flags.argtypes = [ctypes.POINTER(ctypes.c_uint32), S]
    L.cv_debug_flags.restype = S
    L.cv_debug_check_ascending.argtypes = [P, U64, P]
    L.cv_debug_check_ascending.restype = S
    return L


def strerror(status) -> str:
    return lib().cv_strerror(int(status)).decode()


def _check(status, where):
    if status != CV_OK:
        raise CvError(status, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _records_struct(rec) -> CvRecords:
    n = int(rec["journey_id"].numel())
    return CvRecords(*(_ptr(rec.get(k)) for k, _ in RECORD_FIELDS), n)


def _spec_struct(grid) -> CvGridSpec:
    return CvGridSpec(float(grid.lat0_deg), float(grid.lon0_deg), float(grid.dlat_deg), float(grid.dlon_deg),
                      int(grid.n_lat), int(grid.n_lon), int(grid.t0_ms), int(grid.bin_ms), int(grid.n_t))


def _size(fn, *args) -> int:
    out = ctypes.c_size_t(0)
    _check(fn(*args, ctypes.byref(out)), fn.__name__)
    return int(out.value)


def new_result(device="cuda"):
    return torch.zeros(64, dtype=torch.uint8, device=device)


def read_result(res) -> dict:
    a = np.frombuffer(res.cpu().numpy().tobytes(), dtype=RESULT_DTYPE)[0]
    return {k: int(a[k]) for k in ("status", "flags", "count", "required", "n_out_of_grid", "n_late", "key_bits",
                                         "packed_pass", "n_bad")}


def workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def to_device(records, device="cuda"):
    """Host numpy columns (gen.Records or a 5-tuple) -> dict of device tensors."""
    cols = records.columns() if hasattr(records, "columns") else records
    return {k: torch.from_numpy(np.ascontiguousarray(c)).to(device) for (k, _), c in zip(RECORD_FIELDS, cols)}


def empty_records(n, device="cuda"):
    return {k: torch.empty(n, dtype=dt, device=device) for k, dt in RECORD_FIELDS}


# ---------------------------------------------------------------------------
# the four calls
# ---------------------------------------------------------------------------

def cv_sort_records(rec, max_journeys=None, want_sorted=True, ws=None, stream=None, sync=True):
    """Stable (journey_id, ts_ms) order.  Returns (perm[int32], sorted dict, result dict|None)."""
    L = lib()
    n = int(rec["journey_id"].numel())
    dev = rec["journey_id"].device
    mj = int(max_journeys) if max_journeys else max(1, min(n, 1 << 20))
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    out = empty_records(n, dev) if want_sorted else None
    so = CvRecordsOut(*(_ptr(out[k]) for k, _ in RECORD_FIELDS)) if want_sorted else CvRecordsOut()
    need = _size(L.cv_sort_workspace_size, n, mj)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    st = L.cv_sort_records(ctypes.byref(_records_struct(rec)), mj, _ptr(perm), ctypes.byref(so), _ptr(res),
                           _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "cv_sort_records")
    if not sync:
        return perm, out, res
    r = read_result(res)
    if r["status"] == CV_ERR_CAPACITY and max_journeys is None:
        return cv_sort_records(rec, max_journeys=max(2 * mj, r["required"]), want_sorted=want_sorted,
                               stream=stream)
    _check(r["status"], "cv_sort_records (device)")
    return perm, out, r


def cv_sort_records_features(rec, max_journeys, ws=None, stream=None, shard_offsets=None):
    """Sort and kinematics in one call.  Returns (perm, sorted dict, features
    dict, result dict); `shard_offsets` (device uint64, S + 1) selects the
    batched form."""
    L = lib()
    n = int(rec["journey_id"].numel())
    dev = rec["journey_id"].device
    mj = int(max_journeys)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    out = empty_records(n, dev)
    feat = {k: torch.empty(n, dtype=dt, device=dev) for k, dt in FEATURE_FIELDS}
    so = CvRecordsOut(*(_ptr(out[k]) for k, _ in RECORD_FIELDS))
    fs = CvFeatures(*(_ptr(feat[k]) for k, _ in FEATURE_FIELDS))
    need = _size(L.cv_sort_workspace_size, n, mj)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    if shard_offsets is None:
        st = L.cv_sort_records_features(ctypes.byref(_records_struct(rec)), mj, _ptr(perm), ctypes.byref(so),
                                        ctypes.byref(fs), _ptr(res), _ptr(ws), ws.numel(), _stream(stream))
    else:
        st = L.cv_batch_sort_records_features(ctypes.byref(_records_struct(rec)), _ptr(shard_offsets),
                                              int(shard_offsets.numel()) - 1, mj, _ptr(perm), ctypes.byref(so),
                                              ctypes.byref(fs), _ptr(res), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "cv_sort_records_features")
    r = read_result(res)
    _check(r["status"], "cv_sort_records_features (device)")
    return perm, out, feat, r


def cv_journey_features(sorted_rec, stream=None):
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    feat = {k: torch.empty(n, dtype=dt, device=dev) for k, dt in FEATURE_FIELDS}
    fs = CvFeatures(*(_ptr(feat[k]) for k, _ in FEATURE_FIELDS))
    _check(L.cv_journey_features(ctypes.byref(_records_struct(sorted_rec)), ctypes.byref(fs), _stream(stream)),
           "cv_journey_features")
    return feat


def _feat_struct(feat):
    return CvFeatures(*(_ptr(feat.get(k)) for k, _ in FEATURE_FIELDS))


def cv_journey_summary_noalloc(sorted_rec, feat, out, capacity=None, stream=None):
    """cv_journey_summary on the library's own per-GPU scratch array (the C
    call allocates nothing; `out` is the caller's preallocated dict of
    JOURNEY_FIELDS columns).  Returns the device result tensor, unsynchronised."""
    L = lib()
    dev = sorted_rec["journey_id"].device
    cap = int(capacity) if capacity is not None else int(out["journey_id"].numel())
    js = CvJourneys(*(_ptr(out[k]) for k, _ in JOURNEY_FIELDS))
    res = new_result(dev)
    st = L.cv_journey_summary_noalloc(ctypes.byref(_records_struct(sorted_rec)), ctypes.byref(_feat_struct(feat)),
                                      ctypes.byref(js), cap, _ptr(res), _stream(stream))
    _check(st, "cv_journey_summary_noalloc")
    return res


def cv_journey_summary(sorted_rec, feat, capacity=None, stream=None, sync=True, ws=None, out=None):
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    cap = int(capacity) if capacity is not None else max(1, min(n, 1 << 20))
    if out is None:
        out = {k: torch.empty(cap, dtype=dt, device=dev) for k, dt in JOURNEY_FIELDS}
    js = CvJourneys(*(_ptr(out[k]) for k, _ in JOURNEY_FIELDS))
    need = _size(L.cv_summary_workspace_size, n, cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    st = L.cv_journey_summary(ctypes.byref(_records_struct(sorted_rec)), ctypes.byref(_feat_struct(feat)),
                              ctypes.byref(js), cap, _ptr(res), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "cv_journey_summary")
    if not sync:
        return out, res
    r = read_result(res)
    if r["status"] == CV_ERR_CAPACITY and capacity is None:
        return cv_journey_summary(sorted_rec, feat, capacity=r["required"], stream=stream)
    _check(r["status"], "cv_journey_summary (device)")
    J = r["count"]
    return {k: v[:J] for k, v in out.items()}, r


def cv_grid_aggregate(sorted_rec, grid, capacity=None, stream=None, sync=True, ws=None, out=None, flags=None):
    """flags: the kinematics' flags column of the same sorted records; the
    journey starts then come from its FIRST bits (cv_grid_aggregate_flags)."""
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    cap = int(capacity) if capacity is not None else max(1, min(n, 1 << 22))
    spec = _spec_struct(grid)
    if out is None:
        out = {k: torch.empty(cap, dtype=dt, device=dev) for k, dt in GROUP_FIELDS}
    gs = CvGroups(*(_ptr(out[k]) for k, _ in GROUP_FIELDS))
    need = _size(L.cv_grid_workspace_size, n, ctypes.byref(spec), cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    if flags is not None:
        st = L.cv_grid_aggregate_flags(ctypes.byref(_records_struct(sorted_rec)), _ptr(flags), ctypes.byref(spec),
                                       ctypes.byref(gs), cap, _ptr(res), _ptr(ws), ws.numel(), _stream(stream))
    else:
        st = L.cv_grid_aggregate(ctypes.byref(_records_struct(sorted_rec)), ctypes.byref(spec), ctypes.byref(gs),
                                 cap, _ptr(res), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "cv_grid_aggregate")
    if not sync:
        return out, res
    r = read_result(res)
    if r["status"] == CV_ERR_CAPACITY and capacity is None:
        return cv_grid_aggregate(sorted_rec, grid, capacity=r["required"], stream=stream, flags=flags)
    _check(r["status"], "cv_grid_aggregate (device)")
    G = r["count"]
    return {k: v[:G] for k, v in out.items()}, r


def cv_grid_aggregate_dir(sorted_rec, grid, n_dir=4, offset=0.0, heading=None, feat=None, capacity=None,
                          stream=None, sync=True, ws=None, out=None):
    """The lattice with a direction dimension; the sector comes from `heading`
    (float32 per sorted record) when given, else from feat's bearing."""
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    cap = int(capacity) if capacity is not None else max(1, min(n, 1 << 22))
    spec = _spec_struct(grid)
    if out is None:
        out = {k: torch.empty(cap, dtype=dt, device=dev) for k, dt in GROUP_FIELDS}
    gs = CvGroups(*(_ptr(out[k]) for k, _ in GROUP_FIELDS))
    need = _size(L.cv_grid_workspace_size, n, ctypes.byref(spec), cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    fs = _feat_struct(feat) if feat is not None else None
    st = L.cv_grid_aggregate_dir(ctypes.byref(_records_struct(sorted_rec)), _ptr(heading),
                                 ctypes.byref(fs) if fs is not None else None, ctypes.byref(spec), int(n_dir),
                                 float(offset), ctypes.byref(gs), cap, _ptr(res), _ptr(ws), ws.numel(),
                                 _stream(stream))
    _check(st, "cv_grid_aggregate_dir")
    if not sync:
        return out, res
    r = read_result(res)
    if r["status"] == CV_ERR_CAPACITY and capacity is None:
        return cv_grid_aggregate_dir(sorted_rec, grid, n_dir, offset, heading, feat, capacity=r["required"],
                                     stream=stream)
    _check(r["status"], "cv_grid_aggregate_dir (device)")
    G = r["count"]
    return {k: v[:G] for k, v in out.items()}, r


def cv_gather_column(col, perm, stream=None, out=None):
    """out[k] = col[perm[k]] on the device (a payload column in sorted order)."""
    n = int(perm.numel())
    assert int(col.numel()) == n and col.element_size() in (4, 8)
    if out is None:
        out = torch.empty_like(col)
    _check(lib().cv_gather_column(_ptr(col), _ptr(perm), _ptr(out), n, col.element_size(), _stream(stream)),
           "cv_gather_column")
    return out


def _groups_struct(groups):
    return CvGroups(*(_ptr(groups.get(k)) for k, _ in GROUP_FIELDS))


def lattice_channels(n_dir):
    return 2 * (n_dir + 1 if n_dir else 1)


def cv_lattice_dense(groups, grid, n_dir=0, t_first=0, n_t=None, out=None, stream=None):
    """Dense [n_t][C][n_lat][n_lon] float32 lattice of a group table."""
    G = int(groups["key"].numel())
    dev = groups["key"].device
    n_t = int(n_t if n_t is not None else grid.n_t)
    C = lattice_channels(n_dir)
    if out is None:
        out = torch.empty((n_t, C, int(grid.n_lat), int(grid.n_lon)), dtype=torch.float32, device=dev)
    gs = _groups_struct(groups)
    _check(lib().cv_lattice_dense(ctypes.byref(gs), G, ctypes.byref(_spec_struct(grid)), int(n_dir), int(t_first),
                                  n_t, _ptr(out), _stream(stream)), "cv_lattice_dense")
    return out


def cv_lattice_normalize(lattice, grid, n_dir=0, stream=None, minmax=None, ws=None):
    """In-place per-channel min-max normalisation; returns (lattice, [C][2] min/max)."""
    L = lib()
    C = lattice_channels(n_dir)
    n_t = int(lattice.shape[0])
    spec = _spec_struct(grid)
    if minmax is None:
        minmax = torch.empty(2 * C, dtype=torch.float32, device=lattice.device)
    need = _size(L.cv_lattice_normalize_workspace_size, n_t, ctypes.byref(spec), int(n_dir))
    if ws is None or ws.numel() < need:
        ws = workspace(need, lattice.device)
    _check(L.cv_lattice_normalize(_ptr(lattice), n_t, ctypes.byref(spec), int(n_dir), _ptr(minmax), _ptr(ws),
                                  ws.numel(), _stream(stream)), "cv_lattice_normalize")
    return lattice, minmax.view(C, 2)


def cv_groups_filter(groups, min_volume, speed_lo, speed_hi, capacity=None, stream=None):
    """Indices (ascending) of the groups kept by the volume and mean-speed filter."""
    L = lib()
    G = int(groups["count"].numel())
    dev = groups["count"].device
    cap = int(capacity) if capacity is not None else max(1, G)
    idx = torch.empty(cap, dtype=torch.int32, device=dev)
    ws = workspace(_size(L.cv_groups_filter_workspace_size, G), dev)
    res = new_result(dev)
    gs = _groups_struct(groups)
    _check(L.cv_groups_filter(ctypes.byref(gs), G, float(min_volume), float(speed_lo), float(speed_hi), _ptr(idx),
                              cap, _ptr(res), _ptr(ws), ws.numel(), _stream(stream)), "cv_groups_filter")
    r = read_result(res)
    _check(r["status"], "cv_groups_filter (device)")
    return idx[:r["count"]], r


def cv_drop_duplicates(sorted_rec, perm=None, stream=None):
    """Sorted records without exact duplicate rows; returns (records, perm of the kept, result)."""
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    out = empty_records(n, dev)
    po = torch.empty(n, dtype=torch.int32, device=dev) if perm is not None else None
    ws = workspace(_size(L.cv_hygiene_workspace_size, n), dev)
    res = new_result(dev)
    oo = CvRecordsOut(*(_ptr(out[k]) for k, _ in RECORD_FIELDS))
    _check(L.cv_drop_duplicates(ctypes.byref(_records_struct(sorted_rec)), _ptr(perm), ctypes.byref(oo), _ptr(po),
                                _ptr(res), _ptr(ws), ws.numel(), _stream(stream)), "cv_drop_duplicates")
    r = read_result(res)
    _check(r["status"], "cv_drop_duplicates (device)")
    m = r["count"]
    return {k: v[:m] for k, v in out.items()}, (po[:m] if po is not None else None), r


def cv_split_trips(sorted_rec, gap_ms, capacity=None, stream=None):
    """Trip number per sorted record and journey id per trip; returns (trip_id, trip_journey, result)."""
    L = lib()
    n = int(sorted_rec["journey_id"].numel())
    dev = sorted_rec["journey_id"].device
    cap = int(capacity) if capacity is not None else max(1, n)
    tid = torch.empty(max(1, n), dtype=torch.int64, device=dev)
    tj = torch.empty(cap, dtype=torch.int64, device=dev)
    ws = workspace(_size(L.cv_hygiene_workspace_size, n), dev)
    res = new_result(dev)
    _check(L.cv_split_trips(ctypes.byref(_records_struct(sorted_rec)), int(gap_ms), _ptr(tid), _ptr(tj), cap,
                            _ptr(res), _ptr(ws), ws.numel(), _stream(stream)), "cv_split_trips")
    r = read_result(res)
    _check(r["status"], "cv_split_trips (device)")
    return tid[:n], tj[:r["count"]], r


def cv_csv_extract(text, has_header=True, capacity=None, stream=None, out=None, heading=None, row_ok=None,
                   ws=None, sync=True):
    """Table-1-shaped CSV text (a uint8 device tensor) -> (records, heading, row_ok, result)."""
    L = lib()
    nbytes = int(text.numel())
    dev = text.device
    cap = int(capacity) if capacity is not None else max(1, nbytes // 32 + 1)
    if out is None:
        out = empty_records(cap, dev)
    if heading is None:
        heading = torch.empty(cap, dtype=torch.float32, device=dev)
    if row_ok is None:
        row_ok = torch.empty(cap, dtype=torch.uint8, device=dev)
    need = _size(L.cv_csv_workspace_size, nbytes, cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    res = new_result(dev)
    oo = CvRecordsOut(*(_ptr(out[k]) for k, _ in RECORD_FIELDS))
    _check(L.cv_csv_extract(_ptr(text), nbytes, 1 if has_header else 0, ctypes.byref(oo), _ptr(heading),
                            _ptr(row_ok), cap, _ptr(res), _ptr(ws), ws.numel(), _stream(stream)), "cv_csv_extract")
    if not sync:
        return out, heading, row_ok, res
    r = read_result(res)
    if r["status"] == CV_ERR_CAPACITY and capacity is None:
        return cv_csv_extract(text, has_header, capacity=r["required"], stream=stream)
    _check(r["status"], "cv_csv_extract (device)")
    m = r["count"]
    return {k: v[:m] for k, v in out.items()}, heading[:m], row_ok[:m], r


# ---------------------------------------------------------------------------
# tuning and timing
# ---------------------------------------------------------------------------

def cv_tuning_set(name, value):
    _check(lib().cv_tuning_set(name.encode(), int(value)), f"cv_tuning_set({name})")


def cv_tuning_get(name):
    v = ctypes.c_int64(0)
    _check(lib().cv_tuning_get(name.encode(), ctypes.byref(v)), f"cv_tuning_get({name})")
    return int(v.value)


def cv_timing_enable(on=True):
    _check(lib().cv_timing_enable(1 if on else 0), "cv_timing_enable")


def cv_timing_reset():
    _check(lib().cv_timing_reset(), "cv_timing_reset")


def cv_timing_read(family):
    ms = ctypes.c_double(0)
    cnt = ctypes.c_uint64(0)
    _check(lib().cv_timing_read(family.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "cv_timing_read")
    return float(ms.value), int(cnt.value)


def run_plain(rec, grid, max_journeys=None, journey_capacity=None, group_capacity=None, stream=None):
    """The whole plain path on one device batch: order, features, summary, grid."""
    perm, srt, rsort = cv_sort_records(rec, max_journeys=max_journeys, stream=stream)
    feat = cv_journey_features(srt, stream=stream)
    summ, rs = cv_journey_summary(srt, feat, capacity=journey_capacity, stream=stream)
    groups, rg = cv_grid_aggregate(srt, grid, capacity=group_capacity, stream=stream, flags=feat["flags"])
    return dict(perm=perm, sorted=srt, features=feat, summary=summ, groups=groups, n_out=rg["n_out_of_grid"],
                sort_result=rsort, summary_result=rs, grid_result=rg)


class Pipeline:
    """Preallocated buffers for repeated runs of the plain path on batches of
    at most `n` records: no allocation and no host synchronisation inside
    `run()`, which only enqueues the four calls on the stream."""

    def __init__(self, n, grid, max_journeys, journey_capacity, group_capacity, device="cuda", fused=True):
        L = lib()
        self.n, self.grid, self.device = int(n), grid, device
        self.fused = bool(fused)
        self.max_journeys = int(max_journeys)
        self.jcap, self.gcap = int(journey_capacity), int(group_capacity)
        self.perm = torch.empty(self.n, dtype=torch.int32, device=device)
        self.sorted = empty_records(self.n, device)
        self.feat = {k: torch.empty(self.n, dtype=dt, device=device) for k, dt in FEATURE_FIELDS}
        self.journeys = {k: torch.empty(self.jcap, dtype=dt, device=device) for k, dt in JOURNEY_FIELDS}
        self.groups = {k: torch.empty(self.gcap, dtype=dt, device=device) for k, dt in GROUP_FIELDS}
        self.spec = _spec_struct(grid)
        self.ws_sort = workspace(_size(L.cv_sort_workspace_size, self.n, self.max_journeys), device)
        self.ws_sum = workspace(_size(L.cv_summary_workspace_size, self.n, self.jcap), device)
        self.ws_grid = workspace(_size(L.cv_grid_workspace_size, self.n, ctypes.byref(self.spec), self.gcap), device)
        self.res = [new_result(device) for _ in range(3)]
        self._so = CvRecordsOut(*(_ptr(self.sorted[k]) for k, _ in RECORD_FIELDS))
        self._fs = CvFeatures(*(_ptr(self.feat[k]) for k, _ in FEATURE_FIELDS))
        self._js = CvJourneys(*(_ptr(self.journeys[k]) for k, _ in JOURNEY_FIELDS))
        self._gs = CvGroups(*(_ptr(self.groups[k]) for k, _ in GROUP_FIELDS))

    def workspace_bytes(self):
        return sum(w.numel() for w in (self.ws_sort, self.ws_sum, self.ws_grid))

    def run(self, rec, stream=None):
        L = lib()
        n = int(rec["journey_id"].numel())
        assert n <= self.n
        s = _stream(stream)
        inp = _records_struct(rec)
        if self.fused:
            _check(L.cv_sort_records_features(ctypes.byref(inp), self.max_journeys, _ptr(self.perm),
                                              ctypes.byref(self._so), ctypes.byref(self._fs), _ptr(self.res[0]),
                                              _ptr(self.ws_sort), self.ws_sort.numel(), s), "cv_sort_records_features")
            srt = CvRecords(*(_ptr(self.sorted[k]) for k, _ in RECORD_FIELDS), n)
        else:
            _check(L.cv_sort_records(ctypes.byref(inp), self.max_journeys, _ptr(self.perm), ctypes.byref(self._so),
                                     _ptr(self.res[0]), _ptr(self.ws_sort), self.ws_sort.numel(), s), "cv_sort_records")
            srt = CvRecords(*(_ptr(self.sorted[k]) for k, _ in RECORD_FIELDS), n)
            _check(L.cv_journey_features(ctypes.byref(srt), ctypes.byref(self._fs), s), "cv_journey_features")
        _check(L.cv_journey_summary(ctypes.byref(srt), ctypes.byref(self._fs), ctypes.byref(self._js), self.jcap,
                                    _ptr(self.res[1]), _ptr(self.ws_sum), self.ws_sum.numel(), s),
               "cv_journey_summary")
        # journey starts from the kinematics' FIRST flags
        _check(L.cv_grid_aggregate_flags(ctypes.byref(srt), _ptr(self.feat["flags"]), ctypes.byref(self.spec),
                                         ctypes.byref(self._gs), self.gcap, _ptr(self.res[2]), _ptr(self.ws_grid),
                                         self.ws_grid.numel(), s), "cv_grid_aggregate_flags")

    def results(self):
        """Read the three device result words (synchronises)."""
        return [read_result(r) for r in self.res]


def shard_offsets(sizes, device="cuda"):
    """Host sizes -> (host offsets numpy, device offsets tensor)."""
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(sizes, dtype=np.uint64), out=off[1:])
    return off, torch.from_numpy(off.view(np.int64)).to(device)


class BatchPipeline:
    """Preallocated buffers for the batched form: many shards in one set of
    launches.  `run()` only enqueues (one cv_batch_run call); offsets and
    results are read afterwards."""

    def __init__(self, n, n_shards, grid, max_journeys, journey_capacity, group_capacity, device="cuda",
                 fused=True):
        L = lib()
        self.n, self.S, self.grid, self.device = int(n), int(n_shards), grid, device
        self.fused = bool(fused)
        self.max_journeys = int(max_journeys)
        self.jcap, self.gcap = int(journey_capacity), int(group_capacity)
        self.perm = torch.empty(self.n, dtype=torch.int32, device=device)
        self.sorted = empty_records(self.n, device)
        self.feat = {k: torch.empty(self.n, dtype=dt, device=device) for k, dt in FEATURE_FIELDS}
        self.journeys = {k: torch.empty(self.jcap, dtype=dt, device=device) for k, dt in JOURNEY_FIELDS}
        self.groups = {k: torch.empty(self.gcap, dtype=dt, device=device) for k, dt in GROUP_FIELDS}
        self.journey_offsets = torch.empty(self.S + 1, dtype=torch.int64, device=device)
        self.group_offsets = torch.empty(self.S + 1, dtype=torch.int64, device=device)
        self.shard_n_out = torch.empty(max(self.S, 1), dtype=torch.int64, device=device)
        self.spec = _spec_struct(grid)
        self.ws = workspace(_size(L.cv_batch_workspace_size, self.n, self.S, self.max_journeys, self.jcap,
                                  ctypes.byref(self.spec), self.gcap), device)
        self.res = torch.zeros(3 * 64, dtype=torch.uint8, device=device)
        self._so = CvRecordsOut(*(_ptr(self.sorted[k]) for k, _ in RECORD_FIELDS))
        self._fs = CvFeatures(*(_ptr(self.feat[k]) for k, _ in FEATURE_FIELDS))
        self._js = CvJourneys(*(_ptr(self.journeys[k]) for k, _ in JOURNEY_FIELDS))
        self._gs = CvGroups(*(_ptr(self.groups[k]) for k, _ in GROUP_FIELDS))

    def run(self, rec, offsets_dev, stream=None):
        L = lib()
        n = int(rec["journey_id"].numel())
        assert n <= self.n and offsets_dev.numel() == self.S + 1
        s = _stream(stream)
        off = _ptr(offsets_dev)
        ws, wsn = _ptr(self.ws), self.ws.numel()
        r0, r1, r2 = (_ptr(self.res[64 * i:64 * (i + 1)]) for i in range(3))
        if self.fused:
            _check(L.cv_batch_run(ctypes.byref(_records_struct(rec)), off, self.S, ctypes.byref(self.spec),
                                  self.max_journeys, _ptr(self.perm), ctypes.byref(self._so), ctypes.byref(self._fs),
                                  ctypes.byref(self._js), self.jcap, _ptr(self.journey_offsets),
                                  ctypes.byref(self._gs), self.gcap, _ptr(self.group_offsets),
                                  _ptr(self.shard_n_out), r0, ws, wsn, s), "cv_batch_run")
            return
        srt = CvRecords(*(_ptr(self.sorted[k]) for k, _ in RECORD_FIELDS), n)
        _check(L.cv_batch_sort_records(ctypes.byref(_records_struct(rec)), off, self.S, self.max_journeys,
                                       _ptr(self.perm), ctypes.byref(self._so), r0, ws, wsn, s),
               "cv_batch_sort_records")
        _check(L.cv_batch_journey_features(ctypes.byref(srt), off, self.S, ctypes.byref(self._fs), s),
               "cv_batch_journey_features")
        _check(L.cv_batch_journey_summary(ctypes.byref(srt), ctypes.byref(self._fs), off, self.S,
                                          ctypes.byref(self._js), self.jcap, _ptr(self.journey_offsets), r1, ws, wsn,
                                          s), "cv_batch_journey_summary")
        _check(L.cv_batch_grid_aggregate(ctypes.byref(srt), off, self.S, ctypes.byref(self.spec),
                                         ctypes.byref(self._gs), self.gcap, _ptr(self.group_offsets), r2, ws, wsn, s),
               "cv_batch_grid_aggregate")

    def results(self):
        return [read_result(self.res[64 * i:64 * (i + 1)]) for i in range(3)]


def cv_batch_run(rec, sizes, grid, max_journeys=None, journey_capacity=None, group_capacity=None):
    """Batched form with self-sizing capacities (one retry on capacity)."""
    n = int(rec["journey_id"].numel())
    dev = rec["journey_id"].device
    off_h, off_d = shard_offsets(sizes, dev)
    assert int(off_h[-1]) == n
    mj = max_journeys or max(1, min(n, 1 << 20))
    jc = journey_capacity or max(1, min(n, 1 << 20))
    gc = group_capacity or max(1, min(n, 1 << 22))
    for _ in range(6):
        bp = BatchPipeline(n, len(sizes), grid, mj, jc, gc, dev)
        bp.run(rec, off_d)
        r = bp.results()
        if all(x["status"] == CV_OK for x in r):
            return bp, r
        for x in r:
            if x["status"] not in (CV_OK, CV_ERR_CAPACITY):
                raise CvError(x["status"], "cv_batch_run (device)")
        if r[0]["status"] == CV_ERR_CAPACITY:
            mj = max(2 * mj, r[0]["required"])
        if r[1]["status"] == CV_ERR_CAPACITY:
            jc = max(jc, r[1]["required"])
        if r[2]["status"] == CV_ERR_CAPACITY:
            gc = min(n, max(4 * gc, r[2]["required"]))
        del bp
    raise CvError(CV_ERR_CAPACITY, "cv_batch_run")


def stream_state_bytes(grid, max_journeys, max_groups, max_batch):
    """Bytes of device state of a stream with these capacities (host query)."""
    return _size(lib().cv_stream_state_size, ctypes.byref(_spec_struct(grid)), int(max_journeys), int(max_groups),
                 int(max_batch))


class Stream:
    """Serving form: device-resident open journeys and group table across pushes."""

    def __init__(self, grid, max_journeys, max_groups, max_batch, device="cuda", stream=None):
        L = lib()
        self.device = device
        self.max_batch = int(max_batch)
        self.spec = _spec_struct(grid)
        need = _size(L.cv_stream_state_size, ctypes.byref(self.spec), int(max_journeys), int(max_groups),
                     self.max_batch)
        self.state = workspace(need, device)
        self.handle = ctypes.c_void_p()
        _check(L.cv_stream_create(ctypes.byref(self.spec), int(max_journeys), int(max_groups), self.max_batch,
                                  _ptr(self.state), self.state.numel(), _stream(stream), ctypes.byref(self.handle)),
               "cv_stream_create")

    def push(self, rec, feat=None, res=None, stream=None):
        """Enqueue one batch; returns (features in input order, device result)."""
        n = int(rec["journey_id"].numel())
        dev = rec["journey_id"].device
        if feat is None:
            feat = {k: torch.empty(n, dtype=dt, device=dev) for k, dt in FEATURE_FIELDS}
        if res is None:
            res = new_result(dev)
        _check(lib().cv_stream_push(self.handle, ctypes.byref(_records_struct(rec)), ctypes.byref(_feat_struct(feat)),
                                    _ptr(res), _stream(stream)), "cv_stream_push")
        return feat, res

    def flush(self, journey_capacity, group_capacity, stream=None):
        jc, gc = int(journey_capacity), int(group_capacity)
        jo = {k: torch.empty(max(jc, 1), dtype=dt, device=self.device) for k, dt in JOURNEY_FIELDS}
        go = {k: torch.empty(max(gc, 1), dtype=dt, device=self.device) for k, dt in GROUP_FIELDS}
        res = torch.zeros(128, dtype=torch.uint8, device=self.device)
        js = CvJourneys(*(_ptr(jo[k]) for k, _ in JOURNEY_FIELDS))
        gs = CvGroups(*(_ptr(go[k]) for k, _ in GROUP_FIELDS))
        _check(lib().cv_stream_flush(self.handle, ctypes.byref(js), jc, ctypes.byref(gs), gc, _ptr(res),
                                     _stream(stream)), "cv_stream_flush")
        rj, rg = read_result(res[:64]), read_result(res[64:])
        for r in (rj, rg):
            _check(r["status"], "cv_stream_flush (device)")
        return {k: v[:rj["count"]] for k, v in jo.items()}, {k: v[:rg["count"]] for k, v in go.items()}, rj, rg

    def snapshot(self, stream=None):
        """The resident state as a pinned host uint8 tensor (the copy is
        stream-ordered; this waits for it)."""
        n = ctypes.c_size_t(0)
        _check(lib().cv_stream_snapshot_size(self.handle, ctypes.byref(n)), "cv_stream_snapshot_size")
        buf = torch.empty(n.value, dtype=torch.uint8, pin_memory=True)
        _check(lib().cv_stream_snapshot(self.handle, ctypes.c_void_p(buf.data_ptr()), n.value, _stream(stream)),
               "cv_stream_snapshot")
        torch.cuda.synchronize(self.device)
        return buf

    def restore(self, buf, stream=None):
        """Replace the resident state with a snapshot of a stream created with
        the same grid and capacities."""
        _check(lib().cv_stream_restore(self.handle, ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream(stream)),
               "cv_stream_restore")
        torch.cuda.synchronize(self.device)

    def close(self):
        if self.handle:
            lib().cv_stream_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
